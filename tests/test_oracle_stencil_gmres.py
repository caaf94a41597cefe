"""Pins of the oracle's stencil mat-vec and of Algorithm 3 / randomized GMRES.

* The stencil equals an independently assembled sparse matrix (Kronecker
  sums of 1-D shift operators) and, with no convection, has the discrete
  sine modes as eigenvectors with the textbook eigenvalues.
* With Theta = I and no restart, randomized GMRES is GMRES: after j steps its
  iterate minimises ||b - A x|| over the Krylov space K_j(A, b), which is
  checked against a brute-force least-squares solve on that space.
* The residual estimate |g_i| is the sketched residual ||Theta (b - A x)||
  (the identity of Sec. 4.2) -- checked against the explicit residual.
* A = I is a lucky breakdown after one step.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import stencil, gmres, sketch


def _assembled(dims, coeffs):
    nx, ny, nz = dims
    c0, cxm, cxp, cym, cyp, czm, czp = coeffs

    def shift(n, off):
        return sp.diags([np.ones(n - abs(off))], [off], shape=(n, n))

    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    A = c0 * sp.kron(Iz, sp.kron(Iy, Ix))
    A = A + cxm * sp.kron(Iz, sp.kron(Iy, shift(nx, -1))) + cxp * sp.kron(Iz, sp.kron(Iy, shift(nx, 1)))
    A = A + cym * sp.kron(Iz, sp.kron(shift(ny, -1), Ix)) + cyp * sp.kron(Iz, sp.kron(shift(ny, 1), Ix))
    A = A + czm * sp.kron(shift(nz, -1), sp.kron(Iy, Ix)) + czp * sp.kron(shift(nz, 1), sp.kron(Iy, Ix))
    return A.tocsr()


def test_stencil_matches_assembled_matrix():
    dims = (5, 4, 3)
    coeffs = (6.1, -1.2, -0.8, -1.05, -0.95, -1.3, -0.7)
    A = _assembled(dims, coeffs)
    u = np.random.Generator(np.random.PCG64(0)).standard_normal(60)
    np.testing.assert_allclose(stencil.apply(u, dims, coeffs), A @ u, rtol=1e-14, atol=1e-14)


def test_poisson_sine_modes_are_eigenvectors():
    N = 9
    dims, coeffs = synth.convdiff_coeffs(N, 0.0)
    h = 1.0 / (N + 1)
    g = np.arange(1, N + 1) * h
    a, b, c = 2, 5, 7
    u = (np.sin(c * np.pi * g)[:, None, None] * np.sin(b * np.pi * g)[None, :, None]
         * np.sin(a * np.pi * g)[None, None, :]).reshape(-1)
    lam = 6 - 2 * (math.cos(a * np.pi * h) + math.cos(b * np.pi * h) + math.cos(c * np.pi * h))
    np.testing.assert_allclose(stencil.apply(u, dims, coeffs), lam * u, atol=1e-13)


def _krylov_min_residual(A, b, j):
    K = np.empty((b.size, j))
    v = b.copy()
    for t in range(j):
        K[:, t] = v
        v = A @ v
    U, _ = np.linalg.qr(K)                      # orthonormal basis of K_j
    z, *_ = np.linalg.lstsq(A @ U, b, rcond=None)
    return U @ z


def test_identity_sketch_rgmres_is_gmres():
    N, Pe = 4, 20.0
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    A = _assembled(dims, coeffs).toarray()
    n = A.shape[0]
    b = synth.rhs(n, tag=1)
    applyA = lambda u, dt: stencil.apply(u, dims, coeffs, dt)
    for j in (1, 3, 6, 10):
        out = gmres.rgmres(applyA, b, lambda c: sketch.Identity(n), restart=j, tol=1e-30,
                           max_iters=j, max_cycles=1)
        xref = _krylov_min_residual(A, b, j)
        np.testing.assert_allclose(out["x"], xref, rtol=1e-9, atol=1e-9 * np.abs(xref).max())


@pytest.mark.parametrize("kind", ["gaussian", "srht", "rademacher"])
def test_residual_estimate_is_sketched_residual(kind):
    N, Pe = 6, 30.0
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=2)
    applyA = lambda u, dt: stencil.apply(u, dims, coeffs, dt)
    th = sketch.make(kind, n, 64, seed=42, sketch_id=2)
    out = gmres.rgmres(applyA, b, lambda c: th, restart=12, tol=1e-30, max_iters=12, max_cycles=1)
    est = out["hist"][-1] * np.linalg.norm(b)
    true_sk = np.linalg.norm(th.apply(b - applyA(out["x"], np.float64)))
    assert abs(est - true_sk) <= 1e-10 * np.linalg.norm(b)


def test_identity_operator_lucky_breakdown():
    n = 64
    b = synth.rhs(n, tag=3)
    out = gmres.rgmres(lambda u, dt: np.asarray(u, dtype=dt).copy(), b,
                       lambda c: sketch.Gaussian(n, 32, seed=1, sketch_id=2 + c),
                       restart=10, tol=1e-12)
    assert out["iters"] == 1 and out["converged"]
    assert out["true_relres"] <= 1e-14


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_convdiff_converges_restarted(precision):
    N, Pe = 10, 50.0
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=4)
    applyA = lambda u, dt: stencil.apply(u, dims, coeffs, dt)
    out = gmres.rgmres(applyA, b, lambda c: sketch.Gaussian(n, 80, seed=42, sketch_id=2 + c),
                       restart=20, tol=1e-6, precision=precision)
    assert out["converged"] and out["true_relres"] <= 1e-6
    r = b - applyA(out["x"], np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-6
    assert out["cycles"] >= 2                  # restarts really happened


def test_bf16_model_without_rounding_is_the_fp32_model(monkeypatch):
    """The bf16 basis model keeps columns unnormalised and folds 1/r_cc into the
    projection coefficients, the mat-vec input and the x update.  With the bf16
    rounding replaced by the identity on float32 it must reproduce the fp32
    model up to rounding (a wrong or missing scale anywhere fails this)."""
    N, Pe = 9, 30.0
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=6)
    applyA = lambda u, dt: stencil.apply(u, dims, coeffs, dt)
    mk = lambda c: sketch.SRHT(n, 64, seed=42, sketch_id=2 + c)
    ref = gmres.rgmres(applyA, b, mk, restart=15, tol=1e-6, precision="fp32")
    monkeypatch.setattr(gmres, "bf16_round", lambda x: np.asarray(x, dtype=np.float32).copy())
    out = gmres.rgmres(applyA, b, mk, restart=15, tol=1e-6, precision="bf16q")
    assert out["iters"] == ref["iters"] and out["cycles"] == ref["cycles"]
    np.testing.assert_allclose(out["hist"], ref["hist"], rtol=1e-4)
    assert np.linalg.norm(out["x"] - ref["x"]) <= 1e-5 * np.linalg.norm(ref["x"])


def test_bf16_model_converges_with_rounding():
    """With the bf16 rounding on, restarts still drive the fp64 true residual to tol."""
    N, Pe = 9, 30.0
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=6)
    applyA = lambda u, dt: stencil.apply(u, dims, coeffs, dt)
    out = gmres.rgmres(applyA, b, lambda c: sketch.SRHT(n, 64, seed=42, sketch_id=2 + c),
                       restart=15, tol=1e-6, precision="bf16q")
    assert out["converged"]
    r = b - applyA(out["x"], np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16q"])
def test_reversed_projection_order_is_the_same_step(precision):
    """reverse_projection only reorders the sum Q_{i-1} r of RGS step 3.  In
    fp64 that changes nothing beyond rounding (iterates within 1e-10); in the
    fp32 and bf16 models the twin is a second valid rounding: it converges,
    and it is really a different rounding (some history value differs)."""
    N, Pe = 9, 30.0
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=6)
    applyA = lambda u, dt: stencil.apply(u, dims, coeffs, dt)
    mk = lambda c: sketch.SRHT(n, 64, seed=42, sketch_id=2 + c)
    ref = gmres.rgmres(applyA, b, mk, restart=15, tol=1e-6, precision=precision)
    rev = gmres.rgmres(applyA, b, mk, restart=15, tol=1e-6, precision=precision, reverse_projection=True)
    assert rev["converged"]
    r = b - applyA(rev["x"], np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-6
    if precision == "fp64":
        assert rev["iters"] == ref["iters"]
        np.testing.assert_allclose(rev["hist"], ref["hist"], rtol=1e-8)
        assert np.linalg.norm(rev["x"] - ref["x"]) <= 1e-10 * np.linalg.norm(ref["x"])
    else:
        L = min(len(ref["hist"]), len(rev["hist"]))
        assert np.any(rev["hist"][:L] != ref["hist"][:L])


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
def test_last_cycle_basis_is_sketch_orthonormal_and_spans_the_update(kind):
    """The returned last-cycle basis: its sketch with that cycle's Theta has
    orthonormal columns (S = Theta Q of RGS, Algorithm 2, in fp64), and the
    last update of x lies in its span (x_final - x_before = Q_last y)."""
    N, Pe = 10, 50.0
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=5)
    applyA = lambda u, dt: stencil.apply(u, dims, coeffs, dt)
    make = lambda c: sketch.make(kind, n, 80, seed=42, sketch_id=2 + c)
    out = gmres.rgmres(applyA, b, make, restart=20, tol=1e-6)
    Q = out["Q_last"]
    assert out["converged"] and out["cycles"] >= 2 and Q.shape[1] >= 1
    assert out["theta_cycle_last"] == out["cycles"] - 1
    S = make(out["theta_cycle_last"]).apply(Q)
    assert np.linalg.norm(np.eye(Q.shape[1]) - S.T @ S, 2) <= 1e-12
    prev = gmres.rgmres(applyA, b, make, restart=20, tol=1e-6, max_cycles=out["cycles"] - 1)
    dx = out["x"] - prev["x"]
    y = np.linalg.lstsq(Q, dx, rcond=None)[0]
    assert np.linalg.norm(dx - Q @ y) <= 1e-12 * np.linalg.norm(out["x"])   # x rounding, not dx, sets the floor


@pytest.mark.parametrize("sk", ["srht", "gaussian"])
def test_unique_precision_model_is_sec53(sk):
    """'fp32u' is the configuration of the GMRES experiment of Sec. 5.3: RGS in
    float32 throughout, the products with A and the Givens rotations in fp64.
    * every product with A is requested in fp64 (the 'fp32' multi-precision
      model asks for float32 products inside a cycle);
    * the basis vectors and their sketches are float32 values (the 'fp32'
      model's sketches are fp64 values);
    * it reaches tol in the fp64 true residual within +-2 iterations of the
      fp64 model (Sec. 5.3: the unique-precision RGS already gives a nearly
      optimal solution);
    * it is a different rounding from the 'fp32' model: the histories agree to
      1e-3 but not to 1e-9."""
    N, Pe = 9, 30.0
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=7)
    mk = lambda c: sketch.make(sk, n, 64, seed=42, sketch_id=2 + c)
    asked = {}

    def applyA(prec):
        def f(u, dt):
            asked.setdefault(prec, set()).add(np.dtype(dt))
            return stencil.apply(u, dims, coeffs, dt)
        return f

    ref = gmres.rgmres(applyA("fp64"), b, mk, restart=15, tol=1e-6, precision="fp64")
    mp = gmres.rgmres(applyA("fp32"), b, mk, restart=15, tol=1e-6, precision="fp32")
    up = gmres.rgmres(applyA("fp32u"), b, mk, restart=15, tol=1e-6, precision="fp32u")
    assert asked["fp32u"] == {np.dtype(np.float64)}
    assert np.dtype(np.float32) in asked["fp32"]
    for key in ("Q_last", "S_last"):
        v = up[key]
        assert np.array_equal(v.astype(np.float32).astype(np.float64), v), key
    assert not np.array_equal(mp["S_last"].astype(np.float32).astype(np.float64), mp["S_last"])
    assert up["converged"] and ref["converged"]
    r = b - stencil.apply(up["x"], dims, coeffs, np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-6
    assert abs(up["iters"] - ref["iters"]) <= 2
    L = min(len(up["hist"]), len(mp["hist"]))
    np.testing.assert_allclose(up["hist"][:L], mp["hist"][:L], rtol=1e-3)
    assert np.max(np.abs(up["hist"][:L] / mp["hist"][:L] - 1)) > 1e-9
