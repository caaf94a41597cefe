"""GPU parity of the batched QR with the Gaussian sketch read from the exact
fp32 table of its master matrix (rgs_qr_batched_ex with RGS_FLAG_THETA_EXACT).

The table holds the very fp32 entries that the drawn products make (the same
Philox calls through the same Box-Muller, in the layout the products read),
and the products consume them in the same order, so a batch with the flag
equals the drawn batch bit for bit -- in both batched precisions, eagerly and
graph-replayed, under every one of the nine product schedules -- and through
the drawn batch it inherits that batch's parity with the oracle.
"""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


def to_dev(A, dtype):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A).T)).to(dtype=dtype, device="cuda").t()


def _data(count, seed, nlo=3000, nhi=40000, mhi=40):
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(count):
        n = int(g.integers(nlo, nhi))
        m = int(g.integers(4, mhi))
        out.append((synth.svd_matrix(n, m, 1e-3, tag=900 + b + 1000 * seed).astype(np.float32), 4 * m))
    return out


def _items(data, prec):
    rgs = _rgs()
    qd = torch.bfloat16 if prec == "bf16q" else torch.float32
    items = []
    for W, k in data:
        n, m = W.shape
        items.append((to_dev(W, torch.float32), rgs.colmajor(n, m, qd), rgs.colmajor(m, m, torch.float64),
                      rgs.colmajor(k, m, torch.float64), k))
    return items


def _run(h, items, prec, flags, mode=0):
    rgs = _rgs()
    for _, Q, R, S, _k in items:
        Q.fill_(float("nan"))
        R.fill_(float("nan"))
        S.fill_(float("nan"))
    rgs.rgs_set_tuning(h, mode)
    try:
        rep, stat, _ = rgs.rgs_qr_batched(h, items, sketch="gaussian", prec=prec, flags=flags)
        torch.cuda.synchronize()
    finally:
        rgs.rgs_set_tuning(h, 0)
    assert rep.status == 0 and all(v == 0 for v in stat)
    return [(Q.clone(), R.clone(), S.clone()) for _, Q, R, S, _k in items]


def _equal(a, b):
    return all(torch.equal(x, y) for u, v in zip(a, b) for x, y in zip(u, v))


@pytest.mark.parametrize("prec", ["fp32", "bf16q"])
def test_exact_table_batch_equals_drawn(gpu_handle, prec):
    """70 items: step-1 tiles spanning items of different n and k, items over
    several 16384-row chunks and two 128-row sketch tiles, ragged n."""
    rgs = _rgs()
    print("batched exact-table QR, %s" % prec, flush=True)
    items = _items(_data(70, seed=31), prec)
    drawn = _run(gpu_handle, items, prec, 0)
    exact = _run(gpu_handle, items, prec, rgs.FLAG_THETA_EXACT)
    assert _equal(drawn, exact)
    # graph-replayed, twice (capture, replay)
    for _ in range(2):
        assert _equal(drawn, _run(gpu_handle, items, prec, rgs.FLAG_THETA_EXACT | rgs.FLAG_GRAPH))


def test_exact_table_every_schedule(gpu_handle):
    rgs = _rgs()
    items = _items(_data(24, seed=32, mhi=130), "bf16q")
    ref = _run(gpu_handle, items, "bf16q", 0, mode=1)
    for mode in range(1, 10):
        print("  schedule %d" % mode, flush=True)
        assert _equal(ref, _run(gpu_handle, items, "bf16q", rgs.FLAG_THETA_EXACT, mode=mode)), mode


def test_exact_table_flag_rejections(gpu_handle):
    rgs = _rgs()
    items = _items(_data(2, seed=33), "fp32")
    for sk, fl in (("srht", rgs.FLAG_THETA_EXACT), ("gaussian", rgs.FLAG_THETA_EXACT | rgs.FLAG_THETA_BF16)):
        with pytest.raises(rgs.RgsError) as e:
            rgs.rgs_qr_batched(gpu_handle, items, sketch=sk, prec="fp32", flags=fl)
        assert e.value.status == rgs.RGS_EINVAL
