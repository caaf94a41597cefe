"""rgs_qr with RGS_FLAG_GRAPH: the factorisation's device work (every column
of Algorithm 2) is captured once as a HIP graph and replayed on later calls
with the same arguments.  Each replay must equal an eager rgs_qr on the same
input bit for bit -- also after the contents of W change in place (what a
replay is for), with eager work and synchronisations between replays, after a
call with other arguments forced a new capture, and with step 1 split into
several column chunks (which the graph runs on one stream)."""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


def _buffers(n, m, k, prec):
    rgs = _rgs()
    dt = torch.float64 if prec == "fp64" else torch.float32
    dq = {"fp64": torch.float64, "fp32": torch.float32, "bf16q": torch.bfloat16}[prec]
    return (rgs.colmajor(n, m, dt), rgs.colmajor(n, m, dq), rgs.colmajor(m, m, torch.float64),
            rgs.colmajor(k, m, torch.float64))


def _eager(h, W, k, sketch, prec, seed):
    rgs = _rgs()
    n, m = W.shape
    _, Q, R, S = _buffers(n, m, k, prec)
    rep = rgs.rgs_qr(h, rgs.qr_desc(n, m, k, sketch=sketch, prec=prec, seed=seed), W, Q, R, S)
    assert rep.status == 0
    return Q, R, S


CASES = [("gaussian", "fp64", 16384, 64, 256), ("srht", "fp32", 3 * 8192 + 77, 24, 128),
         ("rademacher", "fp32", (1 << 20) + 333, 8, 64), ("gaussian", "bf16q", (1 << 20) + 45, 10, 64),
         ("srht", "fp32", (1 << 18) + 123, 150, 2048)]


@pytest.mark.parametrize("sketch,prec,n,m,k", CASES)
def test_graph_replays_equal_eager(gpu_handle, sketch, prec, n, m, k):
    rgs = _rgs()
    print("rgs_qr graph: %s %s n %d m %d k %d" % (sketch, prec, n, m, k), flush=True)
    W, Q, R, S = _buffers(n, m, k, prec)
    d = rgs.qr_desc(n, m, k, sketch=sketch, prec=prec, seed=9, flags=rgs.FLAG_GRAPH)
    for rnd in range(4):   # capture, then three replays on new contents of W
        W.copy_(torch.from_numpy(synth.svd_matrix(n, m, 10.0 ** -(2 + rnd), tag=400 + rnd)))
        Q.fill_(float("nan"))
        R.fill_(float("nan"))
        S.fill_(float("nan"))
        rep = rgs.rgs_qr(gpu_handle, d, W, Q, R, S)
        assert rep.status == 0
        Q0, R0, S0 = _eager(gpu_handle, W, k, sketch, prec, 9)   # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(Q, Q0) and torch.equal(R, R0) and torch.equal(S, S0), rnd


def test_graph_recaptured_for_other_arguments(gpu_handle):
    rgs = _rgs()
    n, m, k = 20000, 12, 96
    W1, Q1, R1, S1 = _buffers(n, m, k, "fp32")
    W2, Q2, R2, S2 = _buffers(n + 5, m, k, "fp32")
    W1.copy_(torch.from_numpy(synth.svd_matrix(n, m, 1e-3, tag=410)))
    W2.copy_(torch.from_numpy(synth.svd_matrix(n + 5, m, 1e-3, tag=411)))
    d1 = rgs.qr_desc(n, m, k, sketch="srht", prec="fp32", flags=rgs.FLAG_GRAPH)
    d2 = rgs.qr_desc(n + 5, m, k, sketch="srht", prec="fp32", flags=rgs.FLAG_GRAPH)
    for W, Q, R, S, d in ((W1, Q1, R1, S1, d1), (W2, Q2, R2, S2, d2), (W1, Q1, R1, S1, d1),
                          (W1, Q2[:n], R2, S2, d1)):   # the last: same sizes, other output buffers
        assert rgs.rgs_qr(gpu_handle, d, W, Q, R, S).status == 0
        Q0, R0, S0 = _eager(gpu_handle, W, k, "srht", "fp32", 42)
        torch.cuda.synchronize()
        assert torch.equal(Q, Q0) and torch.equal(R, R0) and torch.equal(S, S0)


def test_graph_with_kernel_timing_rejected(gpu_handle):
    rgs = _rgs()
    W, Q, R, S = _buffers(5000, 4, 32, "fp32")
    d = rgs.qr_desc(5000, 4, 32, sketch="srht", prec="fp32", flags=rgs.FLAG_GRAPH | rgs.FLAG_TIME_KERNELS)
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_qr(gpu_handle, d, W, Q, R, S)
    assert e.value.status == rgs.RGS_EINVAL


def test_graph_with_exact_table(gpu_handle):
    """RGS_FLAG_GRAPH with RGS_FLAG_THETA_EXACT: the table is made eagerly on
    every call, before the replay; each replay equals the eager call with the
    same table bit for bit."""
    rgs = _rgs()
    n, m, k = 16384 + 36, 20, 128
    W, Q, R, S = _buffers(n, m, k, "fp32")
    d = rgs.qr_desc(n, m, k, sketch="gaussian", prec="fp32", seed=9, flags=rgs.FLAG_GRAPH | rgs.FLAG_THETA_EXACT)
    de = rgs.qr_desc(n, m, k, sketch="gaussian", prec="fp32", seed=9, flags=rgs.FLAG_THETA_EXACT)
    for rnd in range(3):
        W.copy_(torch.from_numpy(synth.svd_matrix(n, m, 10.0 ** -(2 + rnd), tag=420 + rnd)))
        Q.fill_(float("nan"))
        assert rgs.rgs_qr(gpu_handle, d, W, Q, R, S).status == 0
        _, Q0, R0, S0 = _buffers(n, m, k, "fp32")
        assert rgs.rgs_qr(gpu_handle, de, W, Q0, R0, S0).status == 0
        torch.cuda.synchronize()
        assert torch.equal(Q, Q0) and torch.equal(R, R0) and torch.equal(S, S0), rnd
