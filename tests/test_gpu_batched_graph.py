"""rgs_qr_batched_ex with RGS_FLAG_GRAPH: each stream's kernel sequence of the
batched QR (Algorithm 2 per item, in lockstep) is captured once as a HIP graph
and replayed on later calls with the same items.  Every replay must equal an
eager call on the same input bit for bit -- after the contents of W change in
place (what a replay is for), with eager work and synchronisations between
replays, after a call with a different batch forced a new capture, and for the
P-SRHT, the drawn Gaussian and its bf16 table, in both batched precisions,
and with step 2 by Richardson sweeps.
A Gaussian batch whose product schedule is not tuned yet runs its first call
eagerly (and tunes it); that call must match as well."""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


def _items(shapes, prec):
    """Output buffers that stay put across calls, and W of each item."""
    rgs = _rgs()
    qd = torch.bfloat16 if prec == "bf16q" else torch.float32
    return [(rgs.colmajor(n, m, torch.float32), rgs.colmajor(n, m, qd), rgs.colmajor(m, m, torch.float64),
             rgs.colmajor(k, m, torch.float64), k) for n, m, k in shapes]


def _fill(items, tag):
    for b, (W, _, _, _, _) in enumerate(items):
        n, m = W.shape
        W.copy_(torch.from_numpy(synth.svd_matrix(n, m, 1e-3, tag=tag + b).astype(np.float32)).cuda())


def _call(h, items, sketch, prec, flags):
    rgs = _rgs()
    rep, stat, _ = rgs.rgs_qr_batched(h, items, sketch=sketch, prec=prec, flags=flags)
    torch.cuda.synchronize()
    assert rep.status == 0 and all(v == 0 for v in stat)
    return [(Q.clone(), R.clone(), S.clone()) for _, Q, R, S, _ in items]


def _same(a, b):
    for (Q1, R1, S1), (Q2, R2, S2) in zip(a, b):
        assert torch.equal(Q1.view(torch.int16) if Q1.dtype == torch.bfloat16 else Q1,
                           Q2.view(torch.int16) if Q2.dtype == torch.bfloat16 else Q2)
        assert torch.equal(R1, R2) and torch.equal(S1, S2)


def _shapes(count, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(g.integers(3000, 20000))
        m = int(g.integers(4, 40))
        out.append((n, m, 4 * m))
    return out


# extra flags: 16 = the bf16 table of Theta; s << 24 = step 2 by s Richardson sweeps
CASES = [("srht", "fp32", 0), ("srht", "bf16q", 0), ("gaussian", "fp32", 0), ("gaussian", "bf16q", 0),
         ("gaussian", "fp32", 16), ("gaussian", "bf16q", 16), ("srht", "fp32", 2 << 24),
         ("gaussian", "bf16q", 1 << 24)]


@pytest.mark.parametrize("sketch,prec,extra", CASES)
def test_batched_graph_replays_match_eager(gpu_handle, sketch, prec, extra):
    rgs = _rgs()
    print("batched QR graph %s %s flags=%d" % (sketch, prec, extra), flush=True)
    h = gpu_handle
    items = _items(_shapes(37, seed=5), prec)
    flags = rgs.FLAG_GRAPH | extra
    _fill(items, 900)
    first = _call(h, items, sketch, prec, flags)     # Gaussian: eager, tunes the schedule
    ref1 = _call(h, items, sketch, prec, extra)      # eager
    _same(first, ref1)
    _fill(items, 1900)
    ref2 = _call(h, items, sketch, prec, extra)
    for rep in range(3):                             # capture, then replays
        _fill(items, 900)
        _same(_call(h, items, sketch, prec, flags), ref1)
        torch.ones(1 << 20, device="cuda").sum().item()   # eager work between replays
        _fill(items, 1900)
        _same(_call(h, items, sketch, prec, flags), ref2)
    # a smaller batch (other items): a new capture, equal to its eager call
    small = _items(_shapes(9, seed=6), prec)
    _fill(small, 2900)
    ref3 = _call(h, small, sketch, prec, extra)
    for rep in range(2):
        _same(_call(h, small, sketch, prec, flags), ref3)
    # and back to the first batch
    _fill(items, 900)
    _same(_call(h, items, sketch, prec, flags), ref1)


def test_batched_graph_single_item(gpu_handle):
    """A batch of one runs on the handle's stream only (one share)."""
    rgs = _rgs()
    items = _items([(12345, 17, 68)], "fp32")
    _fill(items, 3900)
    ref = _call(gpu_handle, items, "srht", "fp32", 0)
    for rep in range(2):
        _same(_call(gpu_handle, items, "srht", "fp32", rgs.FLAG_GRAPH), ref)


def test_batched_graph_rejects_unknown_flags(gpu_handle):
    rgs = _rgs()
    items = _items([(4000, 8, 32), (5000, 9, 36)], "fp32")
    _fill(items, 4900)
    for bad in (rgs.FLAG_DIAGNOSTICS, rgs.FLAG_TIME_KERNELS, rgs.FLAG_LAG, rgs.FLAG_GRAPH | rgs.FLAG_CERTIFY):
        with pytest.raises(rgs.RgsError) as e:
            rgs.rgs_qr_batched(gpu_handle, items, sketch="srht", prec="fp32", flags=bad)
        assert e.value.status == rgs.RGS_EINVAL


def test_batched_graph_reports_per_item_failures(gpu_handle):
    """The status words are cleared and read on every replay: a batch whose
    contents turn a zero column and a NaN into two items reports them per item
    on the replay, as the eager call does, and the next replay on healthy
    contents reports none."""
    rgs = _rgs()
    items = _items(_shapes(6, seed=8), "fp32")
    _fill(items, 5900)
    good = _call(gpu_handle, items, "srht", "fp32", 0)
    for rep in range(2):   # capture, replay
        _same(_call(gpu_handle, items, "srht", "fp32", rgs.FLAG_GRAPH), good)
    items[2][0][:, 3] = 0.0
    items[0][0][17, 2] = float("nan")
    torch.cuda.synchronize()
    for flags in (0, rgs.FLAG_GRAPH):
        rep, stat, fcol = rgs.rgs_qr_batched(gpu_handle, items, sketch="srht", prec="fp32", flags=flags)
        torch.cuda.synchronize()
        assert rep.status == rgs.RGS_ENONFINITE
        assert stat == [rgs.RGS_ENONFINITE, 0, rgs.RGS_EBREAKDOWN, 0, 0, 0]
        assert fcol == [2, -1, 3, -1, -1, -1]
    _fill(items, 5900)
    _same(_call(gpu_handle, items, "srht", "fp32", rgs.FLAG_GRAPH), good)
