"""Parity at the benchmark's full size, in the launch configuration bench.py times.

The factorisation W = Q R (n = 2^22, m = 512, k = 2048, fp32 projection with
fp64 least squares; W = U diag(logspace(0,-8,m)) V^T drawn on the device) is
too large for the oracle to redo, so it is checked
* on sampled outputs the oracle recomputes one column at a time: given the
  device's Q_{i-1} and S_{i-1} as inputs, the oracle's step of Algorithm 2
  for column i must reproduce R(1:i, i), r_ii and q_i;
* on S = Theta Q at sampled columns (the oracle's own P-SRHT applied to the
  device's Q);
* on properties that hold at any size: ||W - QR|| / ||W||, and on a
  companion input with sigma down to 1e-3 the fp32-path gate ||I - S^T S||_2 <= 1e-4.
The randomized GMRES of the same suite (192^3 grid, restart 100, k = 400,
tol 1e-6) is checked by recomputing its true residual with the oracle's
operator in fp64.
"""

import math

import numpy as np
import pytest

import synth
from oracle import rgs as orgs, sketch as osk, stencil as ost

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, M, K = 1 << 22, 512, 2048


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


@pytest.fixture(scope="module")
def big_qr(gpu_handle):
    rgs = _rgs()
    W64 = synth.svd_matrix_torch(N, M, 1e-8, tag=0)
    W = rgs.colmajor(N, M, torch.float32)
    W.copy_(W64)
    del W64
    Q = rgs.colmajor(N, M, torch.float32)
    R = rgs.colmajor(M, M, torch.float64)
    S = rgs.colmajor(K, M, torch.float64)
    rep = rgs.rgs_qr(gpu_handle, rgs.qr_desc(N, M, K, sketch="srht", prec="fp32"), W, Q, R, S)
    torch.cuda.synchronize()
    assert rep.status == 0
    yield W, Q, R, S
    del W, Q, R, S
    torch.cuda.empty_cache()


def test_fullsize_backward_error(big_qr):
    W, Q, R, S = big_qr
    res = torch.linalg.norm(W.double() - Q.double() @ R) / torch.linalg.norm(W.double())
    assert float(res) <= 1e-5
    Rh = R.cpu().numpy()
    assert np.all(np.tril(Rh, -1) == 0) and np.all(np.diag(Rh) > 0)


@pytest.mark.parametrize("cols", [(0, 1, 255, 511)])
def test_fullsize_sketch_of_q(big_qr, cols):
    W, Q, R, S = big_qr
    th = osk.SRHT(N, K, seed=42)
    for c in cols:
        q = Q[:, c].cpu().numpy().astype(np.float64)
        s = S[:, c].cpu().numpy()
        sq = th.apply(q)
        assert np.linalg.norm(s - sq) <= 2e-6 * np.linalg.norm(s)


@pytest.mark.parametrize("col", [1, 64, 200])
def test_fullsize_sampled_column_steps(big_qr, col):
    W, Q, R, S = big_qr
    th = osk.SRHT(N, K, seed=42)
    Qprev = Q[:, :col].cpu().numpy()                    # device basis (float32) as the oracle's input
    Sprev = S[:, :col].cpu().numpy()
    w = W[:, col].cpu().numpy()
    st = orgs.rgs_step(Qprev, Sprev, w, th, precision="fp32")
    Rg = R[:, col].cpu().numpy()
    np.testing.assert_allclose(Rg[:col], st["r"], rtol=0, atol=2e-6 * np.abs(st["r"]).max())
    # q'_i = w_i - Q r carries fp32 rounding of order sqrt(i) u32 ||w_i|| on both
    # sides (different summation orders); relative to q'_i that is amplified by
    # ||w_i|| / ||q'_i||, which grows as the columns of W become dependent.
    amp = np.linalg.norm(w.astype(np.float64)) / np.linalg.norm(st["qp"].astype(np.float64))
    tol = 50 * 2.0 ** -24 * math.sqrt(col + 1) * amp
    assert abs(Rg[col] - st["rii"]) <= tol * st["rii"]
    qg = Q[:, col].cpu().numpy().astype(np.float64)
    assert np.linalg.norm(qg - st["q"]) <= tol * np.linalg.norm(st["q"])


def test_fullsize_companion_gate(gpu_handle):
    rgs = _rgs()
    W64 = synth.svd_matrix_torch(N, M, 1e-3, tag=1)
    W = rgs.colmajor(N, M, torch.float32)
    W.copy_(W64)
    del W64
    Q = rgs.colmajor(N, M, torch.float32)
    R = rgs.colmajor(M, M, torch.float64)
    S = rgs.colmajor(K, M, torch.float64)
    rep = rgs.rgs_qr(gpu_handle, rgs.qr_desc(N, M, K, sketch="srht", prec="fp32"), W, Q, R, S)
    torch.cuda.synchronize()
    assert rep.status == 0
    G = (S.T @ S).cpu().numpy()
    assert np.linalg.norm(np.eye(M) - G, 2) <= 1e-4
    res = torch.linalg.norm(W.double() - Q.double() @ R) / torch.linalg.norm(W.double())
    assert float(res) <= 1e-5
    del W, Q, R, S
    torch.cuda.empty_cache()


def test_fullsize_rgmres_true_residual(gpu_handle):
    """The 192^3 system with the P-SRHT (k = 400, restart 100, fp32 basis):
    true residual recomputed on the host in fp64, and the iteration count
    within +-2 of the fp64 oracle's on the same system and sketches (Sec. 4.2),
    cached in tests/golden/gmres_c3_srht.json by make_gmres_refs.py (the oracle
    takes about an hour for it)."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gmres_c3_srht.json")))
    assert (ref["N"], ref["sketch"], ref["k"], ref["restart"], ref["precision"]) == (192, "srht", 400, 100, "fp64")
    assert ref["converged"]
    rgs = _rgs()
    Ng = 192
    dims, coeffs = synth.convdiff_coeffs(Ng, 50.0)
    n = Ng ** 3
    b = synth.rhs(n, tag=0)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    rep, hist = rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs),
                              rgs.gmres_desc(100, 400, 1e-6, max_iters=5000, sketch="srht", prec="fp32"),
                              torch.from_numpy(b).cuda(), x, res_hist=5000)
    torch.cuda.synchronize()
    assert rep.status == 0 and rep.true_relres <= 1e-6
    r = b - ost.apply(x.cpu().numpy(), dims, coeffs, np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-6 * (1 + 1e-6)
    assert len(hist) == rep.iters
    assert math.isclose(rep.true_relres, np.linalg.norm(r) / np.linalg.norm(b), rel_tol=1e-6)
    print("  192^3 srht fp32 basis: %d iterations (fp64 oracle %d)" % (rep.iters, ref["iters"]), flush=True)
    assert abs(rep.iters - ref["iters"]) <= 2


def _gmres_gpu(h, N, sketch, prec, k=400, restart=100, flags=0):
    rgs = _rgs()
    dims, coeffs = synth.convdiff_coeffs(N, 50.0)
    n = N ** 3
    b = synth.rhs(n, tag=0)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    rep, hist = rgs.rgs_gmres(h, rgs.stencil7(dims, coeffs),
                              rgs.gmres_desc(restart, k, 1e-6, max_iters=5000, sketch=sketch, prec=prec, flags=flags),
                              torch.from_numpy(b).cuda(), x, res_hist=5000)
    torch.cuda.synchronize()
    r = b - ost.apply(x.cpu().numpy(), dims, coeffs, np.float64)
    return rep, hist, np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.parametrize("prec,flags", [("fp64", 0), ("fp32", 0), ("fp32", 16), ("fp64", 64), ("fp32", 64)])
def test_gauss64_iterations_vs_cached_oracle(gpu_handle, prec, flags):
    """The randomized GMRES with the drawn Gaussian sketch (k = 400, restart
    100, Pe = 50) on a 64^3 grid against the fp64 oracle's iteration count,
    cached in tests/golden/gmres_c3_gauss64.json by make_gmres_refs.py (the
    oracle draws the same Philox entries; one run takes it minutes).  The fp64
    and fp32 bases must land within +-2 of it (Sec. 4.2), drawn on the fly or
    read from the table of their exact entries (flags 64, the same sketch);
    the bf16 table of the same Gaussian entries (flags 16) is a different
    sketch: the test prints its difference."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gmres_c3_gauss64.json")))
    assert (ref["N"], ref["sketch"], ref["k"], ref["restart"]) == (64, "gaussian", 400, 100) and ref["converged"]
    print("rgmres 64^3 gaussian k=400 %s flags=%d" % (prec, flags), flush=True)
    rep, hist, relres = _gmres_gpu(gpu_handle, 64, "gaussian", prec, flags=flags)
    print("  iters %d (oracle %d), true relres %.3e" % (rep.iters, ref["iters"], relres), flush=True)
    assert rep.status == 0 and relres <= 1e-6 * (1 + 1e-6)
    assert math.isclose(rep.true_relres, relres, rel_tol=1e-6)
    if flags in (0, 64):
        assert abs(rep.iters - ref["iters"]) <= 2


def test_fullsize_rgmres_gaussian(gpu_handle):
    """The 192^3 system with the sketch the workload names (drawn Gaussian,
    k = 400, restart 100, fp32 basis): converged, true residual recomputed on
    the host in fp64, and the same iteration count as the fp64 basis within
    +-2 (no oracle count exists at this size: the oracle would take days)."""
    print("rgmres 192^3 gaussian k=400 fp32", flush=True)
    rep32, hist, relres = _gmres_gpu(gpu_handle, 192, "gaussian", "fp32")
    assert rep32.status == 0 and relres <= 1e-6 * (1 + 1e-6)
    assert math.isclose(rep32.true_relres, relres, rel_tol=1e-6)
    assert len(hist) == rep32.iters
    print("rgmres 192^3 gaussian k=400 fp64", flush=True)
    rep64, _, relres64 = _gmres_gpu(gpu_handle, 192, "gaussian", "fp64")
    assert rep64.status == 0 and relres64 <= 1e-6 * (1 + 1e-6)
    print("  iters fp32 %d fp64 %d" % (rep32.iters, rep64.iters), flush=True)
    assert abs(rep32.iters - rep64.iters) <= 2
    # the same sketch read from the table of its exact fp32 entries
    print("rgmres 192^3 gaussian k=400 fp32, exact table", flush=True)
    repx, _, relresx = _gmres_gpu(gpu_handle, 192, "gaussian", "fp32", flags=64)
    assert repx.status == 0 and relresx <= 1e-6 * (1 + 1e-6)
    print("  iters %d" % repx.iters, flush=True)
    assert abs(repx.iters - rep32.iters) <= 1
