"""GPU parity of the RGMRES path (Algorithm 3 + Sec. 4.2) against the oracle.

* the 7-point mat-vec of Algorithm 3 (fp64 bit-near, fp32 to rounding);
* restarted randomized GMRES on convection-diffusion systems of the recipe
  (grids that span several 8192-row blocks plus a ragged one): iteration
  count within +-2 of the fp64 oracle, residual history, true residual;
* fp32 basis / fp64 least squares against the fp64 oracle's iteration count;
* the identity sketch (k = n) reproduces textbook GMRES iterates;
* lucky breakdown (A = I) and the max_iters cap.
"""

import numpy as np
import pytest

import synth
from oracle import gmres as ogm, sketch as osk, stencil as ost

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stencil_apply_matches_oracle(gpu_handle, prec):
    rgs = _rgs()
    dims, coeffs = synth.convdiff_coeffs(23, 37.0)
    dims = (23, 19, 29)
    n = 23 * 19 * 29
    u = np.random.Generator(np.random.PCG64(3)).standard_normal(n)
    dt = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        u = u.astype(np.float32).astype(np.float64)
    w = torch.empty(n, dtype=dt, device="cuda")
    rgs.rgs_stencil_apply(gpu_handle, rgs.stencil7(dims, coeffs), prec, dev(u, dt), w)
    torch.cuda.synchronize()
    ref = ost.apply(u, dims, coeffs, np.float64)
    got = w.cpu().numpy().astype(np.float64)
    tol = 1e-14 if prec == "fp64" else 4e-7
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def _oracle(N, Pe, restart, k, tol, sketch, precision, tag, max_iters=100000):
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=tag)
    out = ogm.rgmres(lambda u, dt: ost.apply(u, dims, coeffs, dt), b,
                     lambda c: osk.make(sketch, n, k, seed=42, sketch_id=2 + c),
                     restart=restart, tol=tol, precision=precision, max_iters=max_iters)
    return dims, coeffs, b, out


def _gpu(h, dims, coeffs, b, restart, k, tol, sketch, prec, max_iters=100000, flags=0):
    rgs = _rgs()
    n = b.size
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    rep, hist = rgs.rgs_gmres(h, rgs.stencil7(dims, coeffs),
                              rgs.gmres_desc(restart, k, tol, max_iters=max_iters, sketch=sketch, prec=prec,
                                             flags=flags),
                              dev(b), x, res_hist=100000)
    torch.cuda.synchronize()
    return rep, np.array(hist), x.cpu().numpy()


@pytest.mark.parametrize("sketch", ["gaussian", "srht", "rademacher"])
def test_rgmres_fp64_matches_oracle(gpu_handle, sketch):
    N, Pe, restart, k, tol = 24, 50.0, 20, 96, 1e-6        # n = 13824: 2 blocks, ragged
    dims, coeffs, b, ref = _oracle(N, Pe, restart, k, tol, sketch, "fp64", tag=1)
    rep, hist, x = _gpu(gpu_handle, dims, coeffs, b, restart, k, tol, sketch, "fp64")
    assert rep.status == 0 and ref["converged"]
    assert abs(rep.iters - ref["iters"]) <= 2
    assert rep.cycles == ref["cycles"]
    assert rep.true_relres <= tol
    r = b - ost.apply(x, dims, coeffs, np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= tol
    # the residual histories agree while both are far above rounding level
    L = min(len(hist), len(ref["hist"]), restart)
    np.testing.assert_allclose(hist[:L], ref["hist"][:L], rtol=1e-8)


@pytest.mark.parametrize("sketch,prec", [("srht", "fp64"), ("rademacher", "fp64"), ("srht", "fp32"),
                                         ("srht", "bf16q")])
def test_lagged_arnoldi_step_matches_oracle(gpu_handle, sketch, prec):
    """RGS_FLAG_LAG: the mat-vec kernel sketches the stored q'_i and A q'_i
    in one pass (one reduction gives r_ii and p_{i+1}), equal to Algorithm 3
    in exact arithmetic.  fp64: iterations and cycles as the fp64 oracle's
    (+-2), histories to 1e-8 while above rounding level; fp32: +-2 of the fp64
    oracle; bf16 basis: converges with the true residual at tol and within the
    spread of the bf16 model (+-2 of the unlagged device run is not implied:
    the basis rounding is at 2^-9)."""
    rgs = _rgs()
    N, Pe, restart, k, tol = 24, 50.0, 20, 96, 1e-6        # n = 13824: 2 blocks, ragged
    dims, coeffs, b, ref = _oracle(N, Pe, restart, k, tol, sketch, "fp64", tag=1)
    rep, hist, x = _gpu(gpu_handle, dims, coeffs, b, restart, k, tol, sketch, prec, flags=rgs.FLAG_LAG)
    assert rep.status == 0 and ref["converged"]
    r = b - ost.apply(x, dims, coeffs, np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= tol
    if prec == "bf16q":
        _, _, _, refb = _oracle(N, Pe, restart, k, tol, sketch, "bf16q", tag=1)
        assert abs(rep.iters - refb["iters"]) <= max(4, refb["iters"] // 20)
        return
    assert abs(rep.iters - ref["iters"]) <= 2
    if prec == "fp64":
        assert rep.cycles == ref["cycles"]
        L = min(len(hist), len(ref["hist"]), restart)
        np.testing.assert_allclose(hist[:L], ref["hist"][:L], rtol=1e-8)


def test_rgmres_fp32_basis_iterations_near_fp64_oracle(gpu_handle):
    N, Pe, restart, k, tol = 32, 50.0, 30, 120, 1e-6        # n = 32768: 4 full blocks
    dims, coeffs, b, ref = _oracle(N, Pe, restart, k, tol, "gaussian", "fp64", tag=2)
    rep, hist, x = _gpu(gpu_handle, dims, coeffs, b, restart, k, tol, "gaussian", "fp32")
    assert rep.status == 0
    assert abs(rep.iters - ref["iters"]) <= 2
    r = b - ost.apply(x, dims, coeffs, np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= tol
    # the fp32 model of the oracle agrees as well
    _, _, _, ref32 = _oracle(N, Pe, restart, k, tol, "gaussian", "fp32", tag=2)
    assert abs(rep.iters - ref32["iters"]) <= 2


def test_identity_sketch_is_textbook_gmres(gpu_handle):
    N, Pe = 6, 30.0
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=3)
    j = 12
    rep, hist, x = _gpu(gpu_handle, dims, coeffs, b, j, n, 0.0, "identity", "fp64", max_iters=j)
    # x minimises ||b - A x|| over K_j(A, b): brute-force least squares on that space
    A = np.stack([ost.apply(e, dims, coeffs) for e in np.eye(n)], axis=1)
    K = np.empty((n, j))
    v = b.copy()
    for t in range(j):
        K[:, t] = v
        v = A @ v
    U, _ = np.linalg.qr(K)
    z, *_ = np.linalg.lstsq(A @ U, b, rcond=None)
    xref = U @ z
    assert np.abs(x - xref).max() <= 1e-9 * np.abs(xref).max()


def test_lucky_breakdown_identity_operator(gpu_handle):
    dims = (10, 10, 10)
    coeffs = (1.0, 0, 0, 0, 0, 0, 0)
    b = synth.rhs(1000, tag=4)
    rep, hist, x = _gpu(gpu_handle, dims, coeffs, b, 10, 64, 1e-12, "gaussian", "fp64")
    assert rep.status == 0 and rep.iters == 1
    assert np.abs(x - b).max() <= 1e-14 * np.abs(b).max()


def test_max_iters_cap(gpu_handle):
    rgs = _rgs()
    N = 16
    dims, coeffs = synth.convdiff_coeffs(N, 20.0)
    b = synth.rhs(N ** 3, tag=5)
    rep, hist, x = _gpu(gpu_handle, dims, coeffs, b, 10, 64, 1e-14, "gaussian", "fp32", max_iters=7)
    assert rep.status == rgs.RGS_ENOCONV
    assert rep.iters == 7 and len(hist) == 7
    assert np.all(np.diff(hist) <= 1e-12)         # GMRES residuals never increase within a cycle


@pytest.mark.parametrize("sketch,prec,sweeps,lag", [("srht", "fp64", 1, False), ("srht", "fp64", 2, False),
                                                    ("gaussian", "fp64", 2, False), ("srht", "fp32", 2, True),
                                                    ("rademacher", "fp64", 2, True)])
def test_richardson_least_squares_matches_oracle(gpu_handle, sketch, prec, sweeps, lag):
    """ls_sweeps: step 2 of every Arnoldi step by Richardson iterations on the
    normal equations (one sweep: sketched classical Gram-Schmidt; two: its
    re-orthogonalised form), against the oracle's RGMRES with the same solver
    ('richardson1' / 'richardson2'): fp64 iterations and cycles (+-2) and the
    residual histories while far above rounding; fp32 within +-2 of the fp64
    oracle.  With the lagged step (Gaussian always, P-SRHT / Rademacher with
    RGS_FLAG_LAG) the right-hand side carries the 1/r_ii of the step before."""
    rgs = _rgs()
    N, Pe, restart, k, tol = 24, 50.0, 20, 96, 1e-6
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=1)
    ref = ogm.rgmres(lambda u, dt: ost.apply(u, dims, coeffs, dt), b,
                     lambda c: osk.make(sketch, n, k, seed=42, sketch_id=2 + c),
                     restart=restart, tol=tol, precision="fp64", ls="richardson%d" % sweeps)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    rep, hist = rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs),
                              rgs.gmres_desc(restart, k, tol, sketch=sketch, prec=prec, ls_sweeps=sweeps,
                                             flags=rgs.FLAG_LAG if lag else 0),
                              dev(b), x, res_hist=100000)
    torch.cuda.synchronize()
    hist = np.array(hist)
    assert rep.status == 0 and ref["converged"]
    r = b - ost.apply(x.cpu().numpy(), dims, coeffs, np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= tol
    assert abs(rep.iters - ref["iters"]) <= 2
    if prec == "fp64":
        assert rep.cycles == ref["cycles"]
        L = min(len(hist), len(ref["hist"]), restart)
        np.testing.assert_allclose(hist[:L], ref["hist"][:L], rtol=1e-8)


def test_richardson_sweeps_rejected(gpu_handle):
    rgs = _rgs()
    dims, coeffs = synth.convdiff_coeffs(8, 10.0)
    b = dev(synth.rhs(512, tag=1))
    x = torch.empty(512, dtype=torch.float64, device="cuda")
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs), rgs.gmres_desc(5, 32, 1e-6, ls_sweeps=9), b, x)
    assert e.value.status == rgs.RGS_EINVAL
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_gmres_batched(gpu_handle, [(rgs.stencil7(dims, coeffs), b, x)],
                              rgs.gmres_desc(5, 32, 1e-6, ls_sweeps=9))
    assert e.value.status == rgs.RGS_EINVAL


def test_unknown_flag_bits_rejected(gpu_handle):
    """rgs_gmres takes RGS_FLAG_THETA_BF16, THETA_EXACT, LAG and CERTIFY; any
    other bit (the QR-only flags, an undefined bit) is an argument error."""
    rgs = _rgs()
    dims, coeffs = synth.convdiff_coeffs(8, 10.0)
    b = dev(synth.rhs(8 ** 3, tag=91))
    x = torch.empty(8 ** 3, dtype=torch.float64, device="cuda")
    for bad in (rgs.FLAG_DIAGNOSTICS, rgs.FLAG_TIME_KERNELS, rgs.FLAG_GRAPH, 1 << 10):
        with pytest.raises(rgs.RgsError) as e:
            rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs),
                          rgs.gmres_desc(10, 40, 1e-6, sketch="srht", prec="fp64", flags=bad), b, x)
        assert e.value.status == rgs.RGS_EINVAL
    rep, _ = rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs),
                           rgs.gmres_desc(10, 40, 1e-6, sketch="srht", prec="fp64", flags=rgs.FLAG_LAG), b, x)
    assert rep.status == 0
