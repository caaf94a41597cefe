"""GPU parity of the batched QR with the bf16 Gaussian table
(rgs_qr_batched_ex with RGS_FLAG_THETA_BF16, Algorithm 2 applied per item).

Every item uses the leading k_b x n_b block of one master matrix whose
entries are bf16(z) / sqrt(k_b), z the Philox/Box-Muller values of the
Gaussian sketch -- the oracle's GaussianBF16 sketch with instance 0, bit for
bit.  The sketch products of steps 1 and 4 run as bf16 matrix-core products
read from the table (fp32 columns split exactly into three bf16 parts), so
each product theta x is exact and only the fp32 accumulation rounds:
* items against the oracle's fp32 and bf16 models on the same sketch, with
  the bars of the drawn-Gaussian batch (fp32: R to 1e-3 and the backward
  error; bf16: backward error within 1.5x and Delta within 2x, as for the
  P-SRHT, since the entries are the oracle's own);
* S R = Theta W with the oracle's Theta, to the rounding of the stored basis;
* the nine schedules of the product give the same bits;
* the flag is refused with another sketch, and other flags are refused.
"""

import numpy as np
import pytest

import synth
from oracle import metrics, rgs as orgs, sketch as osk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


def to_dev(A, dtype):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A).T)).to(dtype=dtype, device="cuda").t()


def host(t):
    return t.detach().double().cpu().numpy()


def _data(count, seed, nlo=3000, nhi=20000, mhi=40):
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(count):
        n = int(g.integers(nlo, nhi))
        m = int(g.integers(4, mhi))
        out.append((synth.svd_matrix(n, m, 1e-3, tag=800 + b + 1000 * seed).astype(np.float32), 4 * m))
    return out


def _run(h, data, prec, mode=0):
    rgs = _rgs()
    qd = torch.bfloat16 if prec == "bf16q" else torch.float32
    items = []
    for W, k in data:
        n, m = W.shape
        items.append((to_dev(W, torch.float32), rgs.colmajor(n, m, qd), rgs.colmajor(m, m, torch.float64),
                      rgs.colmajor(k, m, torch.float64), k))
    rgs.rgs_set_tuning(h, mode)
    try:
        rep, stat, _ = rgs.rgs_qr_batched(h, items, sketch="gaussian", prec=prec, flags=rgs.FLAG_THETA_BF16)
        torch.cuda.synchronize()
    finally:
        rgs.rgs_set_tuning(h, 0)
    assert rep.status == 0 and all(v == 0 for v in stat)
    return items


@pytest.mark.parametrize("prec", ["fp32", "bf16q"])
def test_table_batch_matches_oracle(gpu_handle, prec):
    """70 items: more than one 64-column tile of the step-4 product, step-1
    tiles spanning items of different n and k, items over two 16384-row
    chunks and two 128-row sketch tiles, ragged n (not a multiple of 16)."""
    print("batched table QR, %s" % prec, flush=True)
    data = _data(70, seed=21)
    items = _run(gpu_handle, data, prec)
    for b in range(0, 70, 3):
        W, k = data[b]
        n, m = W.shape
        _, Q, R, S, _ = items[b]
        theta = osk.GaussianBF16(n, k, seed=42, instance=0)
        ref = orgs.rgs_qr(W, theta, precision=prec)
        Qh, Rh, Sh = host(Q), host(R), host(S)
        W64 = W.astype(np.float64)
        TW = theta.apply(W64)
        srw = np.linalg.norm(Sh @ Rh - TW) / np.linalg.norm(TW)
        if prec == "fp32":
            assert np.linalg.norm(Rh - ref["R"]) / np.linalg.norm(ref["R"]) <= 1e-3, b
            assert metrics.backward_error(W64, Qh, Rh) <= 1e-5, b
            assert srw <= 1e-5, (b, srw)
        else:
            assert metrics.backward_error(W64, Qh, Rh) <= 1.5 * metrics.backward_error(W64, ref["Q"], ref["R"]), b
            assert metrics.delta_2(Sh) <= 2 * metrics.delta_2(ref["S"]), b
            assert srw <= 4 * 2.0 ** -8, (b, srw)


def test_table_step1_is_exact_to_fp32_accumulation(gpu_handle):
    """Column 1 of R is r_11 = ||Theta w_1|| (steps 1 and 5 only, no
    projection): the three-part split and the bf16 products lose nothing, so
    it agrees with the oracle's fp64 sketch of the fp32 column to fp32
    accumulation error (a wrong split or a dropped part shows at 2^-8 or
    2^-16)."""
    data = _data(24, seed=22, nlo=20000, nhi=70000, mhi=12)
    items = _run(gpu_handle, data, "fp32")
    worst = 0.0
    for (W, k), (_, Q, R, S, _) in zip(data, items):
        n = W.shape[0]
        p = osk.GaussianBF16(n, k, seed=42, instance=0).apply(W[:, :1].astype(np.float64))
        e = abs(host(R)[0, 0] - np.linalg.norm(p)) / np.linalg.norm(p)
        worst = max(worst, e)
    assert worst <= 3e-6, worst


@pytest.mark.parametrize("prec", ["fp32", "bf16q"])
def test_table_schedules_give_identical_bits(gpu_handle, prec):
    data = _data(40, seed=23, nhi=30000, mhi=24)
    ref = _run(gpu_handle, data, prec, mode=1)
    for mode in range(2, 10):
        other = _run(gpu_handle, data, prec, mode=mode)
        for (_, Q, R, S, _), (_, Q1, R1, S1, _) in zip(ref, other):
            assert torch.equal(Q, Q1) and torch.equal(R, R1) and torch.equal(S, S1)


def test_table_flag_rejected(gpu_handle):
    rgs = _rgs()
    W, k = _data(1, seed=24)[0]
    n, m = W.shape
    items = [(to_dev(W, torch.float32), rgs.colmajor(n, m, torch.float32), rgs.colmajor(m, m, torch.float64),
              rgs.colmajor(k, m, torch.float64), k)]
    for sketch, flags in (("srht", rgs.FLAG_THETA_BF16), ("gaussian", rgs.FLAG_LAG),
                          ("gaussian", rgs.FLAG_THETA_BF16 | rgs.FLAG_DIAGNOSTICS)):
        with pytest.raises(rgs.RgsError) as e:
            rgs.rgs_qr_batched(gpu_handle, items, sketch=sketch, prec="fp32", flags=flags)
        assert e.value.status == rgs.RGS_EINVAL
