"""Pins of the oracle's Algorithm 2 (RGS) and of its classical references.

* Closed form: in exact arithmetic S R = P = Theta W with S orthonormal and
  r_ii > 0, so R is the positive-diagonal R factor of the thin QR of Theta W
  (LAPACK through numpy), Q = W R^-1 and S = Theta W R^-1.
* Theta = I with the one-sweep Richardson solver (Sec. 2.3: "exactly
  corresponds to ... the classical Gram-Schmidt process") is CGS bit for bit.
* Theta = I with the Householder solver is exact-arithmetic Gram-Schmidt, so
  |R| agrees with |R| of a Householder QR of W.
* A fully sampled SRHT is an isometry, so the same agreement holds.
* Invariants of Theorems 3.2/3.3 and Corollary 2.2 on the outputs.
* Breakdowns and argument errors.
* Sec. 5.1 (qualitative, reduced n): in float32, CGS loses orthogonality,
  MGS degrades, multi-precision RGS keeps cond(Q) close to 1.
* The classical projectors of Sec. 1.2 themselves: MGS in exact arithmetic is
  Gram-Schmidt (|R| of a Householder QR); in floating point it loses
  orthogonality at O(u kappa) where CGS loses it at O(u kappa^2) and CGS2
  keeps it at O(u) (Bjorck; Giraud, Langou, Rozloznik); the float32 variants
  carry float32 rounding, agree with the fp64 ones to O(u32 kappa) in R, and
  keep the same ordering.
* The unique-precision model ('fp32u', every step in float32; Sec. 5.1): the
  closed form above at float32 tolerance, outputs that are float32 values,
  and rounding at the float32 level in the sketch and least-squares steps
  (not only in step 3, as in the multi-precision 'fp32').
"""

import math

import numpy as np
import pytest

import synth
from oracle import rgs, sketch, metrics

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def _wellcond(n, m, smin=1e-2, tag=0):
    return synth.svd_matrix(n, m, smin, tag=tag)


@pytest.mark.parametrize("kind,n,m,k", [("gaussian", 512, 8, 64), ("srht", 1000, 12, 96), ("rademacher", 700, 10, 80),
                                         ("gaussian", 300, 20, 20)])
def test_closed_form_R_from_qr_of_sketch(kind, n, m, k):
    W = _wellcond(n, m, tag=1)
    th = sketch.make(kind, n, k, seed=4)
    out = rgs.rgs_qr(W, th)
    P = th.apply(W)
    _, Rq = np.linalg.qr(P)
    Rq = np.sign(np.diag(Rq))[:, None] * Rq            # positive diagonal
    kappa = metrics.cond(W)
    assert np.linalg.norm(out["R"] - Rq) / np.linalg.norm(Rq) <= 1e-13 * kappa
    Qc = np.linalg.solve(Rq.T, W.T).T                    # W R^-1
    assert np.linalg.norm(out["Q"] - Qc) / np.linalg.norm(Qc) <= 1e-13 * kappa
    np.testing.assert_allclose(out["P"], P, rtol=0, atol=1e-14 * np.abs(P).max())


def test_identity_sketch_with_richardson1_is_cgs_bitwise():
    n, m = 256, 16
    W = _wellcond(n, m, smin=1e-3, tag=2)
    out = rgs.rgs_qr(W, sketch.Identity(n), ls="richardson1")
    Qc, Rc = rgs.cgs(W)
    assert np.array_equal(out["Q"], Qc)
    assert np.array_equal(out["R"], Rc)


def test_identity_sketch_with_richardson2_is_cgs2():
    """Two Richardson sweeps with Theta = I are CGS with one re-orthogonalisation
    (the same two sets of coefficients; RGS subtracts their sum in one pass,
    CGS2 in two, so the columns agree to O(u kappa))."""
    n, m = 300, 20
    W = _wellcond(n, m, smin=1e-4, tag=3)
    uk = U64 * metrics.cond(W)
    out = rgs.rgs_qr(W, sketch.Identity(n), ls="richardson2")
    Qc, Rc = rgs.cgs2(W)
    assert np.linalg.norm(out["R"] - Rc) <= 1e-13 * np.linalg.norm(Rc)
    assert np.linalg.norm(out["Q"] - Qc) <= 100 * uk * np.linalg.norm(Qc)
    assert metrics.orth_loss_2(out["Q"]) <= 100 * uk
    # one sweep (CGS) loses orthogonality at O(u kappa^2): the second sweep is what restores it
    q1 = rgs.rgs_qr(W, sketch.Identity(n), ls="richardson1")["Q"]
    assert metrics.orth_loss_2(q1) > 100 * metrics.orth_loss_2(out["Q"])


def test_identity_sketch_householder_matches_householder_qr():
    n, m = 400, 24
    W = _wellcond(n, m, smin=1e-2, tag=3)
    out = rgs.rgs_qr(W, sketch.Identity(n))
    _, Rh = np.linalg.qr(W)
    assert np.linalg.norm(np.abs(out["R"]) - np.abs(Rh)) / np.linalg.norm(Rh) <= 1e-12


def test_full_srht_matches_householder_qr():
    n, m = 200, 10                                     # s = 256
    W = _wellcond(n, m, smin=1e-2, tag=4)
    out = rgs.rgs_qr(W, sketch.SRHT(n, 256, seed=1))
    _, Rh = np.linalg.qr(W)
    assert np.linalg.norm(np.abs(out["R"]) - np.abs(Rh)) / np.linalg.norm(Rh) <= 1e-12
    assert metrics.orth_loss_2(out["Q"]) <= 1e-12


@pytest.mark.parametrize("kind", ["gaussian", "srht", "rademacher", "gaussian_bf16"])
def test_output_invariants_fp64(kind):
    n, m, k = 2048, 32, 512
    W = synth.svd_matrix(n, m, 1e-6, tag=5)
    th = sketch.make(kind, n, k, seed=42)
    out = rgs.rgs_qr(W, th)
    Q, R, S, P = out["Q"], out["R"], out["S"], out["P"]
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    assert np.max(np.abs(np.linalg.norm(S, axis=0) - 1.0)) <= 8 * U64
    assert metrics.backward_error(W, Q, R) <= 3.7 * U64 * m ** 1.5          # Thm 3.2
    assert metrics.delta_tilde_F(P, S, R) <= 6 * U64 * m ** 1.5               # Thm 3.3
    assert metrics.delta_F(S) <= 20 * U64 * m ** 2 * metrics.cond(W)          # Thm 3.3
    SQ = th.apply(Q)
    assert np.linalg.norm(S - SQ) <= 1e-13 * (np.linalg.norm(Q) + 1)
    eps = metrics.omega(SQ, Q)                                                # Cor. 2.2
    assert eps < 1
    assert metrics.cond(Q) <= math.sqrt((1 + eps) / (1 - eps)) * metrics.cond(S) * (1 + 1e-10)


def test_fp32_model_tolerances():
    n, m, k = 8192, 64, 256
    W = synth.svd_matrix(n, m, 1e-3, tag=6)
    out = rgs.rgs_qr(W, sketch.SRHT(n, k, seed=42), precision="fp32")
    assert out["Q"].dtype == np.float32
    assert metrics.backward_error(W.astype(np.float32), out["Q"], out["R"]) <= 1e-5
    assert metrics.delta_2(out["S"]) <= 1e-4


def test_breakdown_duplicate_column():
    n, m = 512, 6
    W = _wellcond(n, m, tag=7)
    W[:, 3] = W[:, 1]
    with pytest.raises(rgs.Breakdown) as e:
        rgs.rgs_qr(W, sketch.Gaussian(n, 32, seed=1))
    assert e.value.column == 3 and not e.value.nonfinite


def test_breakdown_nonfinite():
    n, m = 512, 6
    W = _wellcond(n, m, tag=8)
    W[10, 2] = np.nan
    with pytest.raises(rgs.Breakdown) as e:
        rgs.rgs_qr(W, sketch.SRHT(n, 32, seed=1))
    assert e.value.column == 2 and e.value.nonfinite


def test_k_smaller_than_m_is_rejected():
    with pytest.raises(ValueError):
        rgs.rgs_qr(np.ones((64, 10)), sketch.Gaussian(64, 8))


def test_step_function_matches_loop():
    n, m, k = 1024, 10, 64
    W = _wellcond(n, m, tag=9)
    th = sketch.SRHT(n, k, seed=2)
    out = rgs.rgs_qr(W, th)
    st = rgs.rgs_step(out["Q"][:, :6], out["S"][:, :6], W[:, 6], th)
    np.testing.assert_allclose(st["r"], out["R"][:6, 6], rtol=1e-14)
    np.testing.assert_allclose(st["rii"], out["R"][6, 6], rtol=1e-14)
    np.testing.assert_allclose(st["q"], out["Q"][:, 6], rtol=1e-13, atol=1e-16)


@pytest.mark.slow
def test_sec51_qualitative_ordering():
    # Sec. 5.1 at reduced n: float32 CGS breaks down badly, MGS degrades,
    # multi-precision RGS keeps cond(Q) close to 1 (and below MGS's).
    n, m, k = 1 << 13, 160, 1500
    W = synth.f_mu_matrix(n, m)
    Qc, _ = rgs.cgs(W, np.float32)
    Qm, _ = rgs.mgs(W, np.float32)
    out = rgs.rgs_qr(W, sketch.SRHT(n, k, seed=42), precision="fp32")
    c_cgs, c_mgs, c_rgs = metrics.cond(Qc), metrics.cond(Qm), metrics.cond(out["Q"])
    assert c_rgs < 3.0
    assert c_mgs > c_rgs
    assert c_cgs > 100 * c_rgs
    assert metrics.backward_error(W.astype(np.float32), out["Q"], out["R"]) < 1e-5
    # cond(S) estimates cond(Q) (Sec. 5.1, third panel)
    assert abs(math.log(metrics.cond(out["S"])) - math.log(c_rgs)) < math.log(2.0)


def test_bf16_rounding_matches_torch():
    import torch
    g = np.random.Generator(np.random.PCG64(11))
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.uniform(-20, 20, 20000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 1e-40])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(rgs.bf16_round(x), ref)


def test_bf16q_model_tolerances():
    # bf16 storage (u = 2^-9) sets both the backward error and Delta: the rounding
    # of q'_i to bf16 has a sketch with a component in span(S_{i-1}) of relative
    # size ~u (Theorem 3.3 bounds Delta by the storage roundoff u_crs).
    n, m, k = 8192, 48, 192
    W = synth.svd_matrix(n, m, 1e-3, tag=21).astype(np.float32)
    th = sketch.Gaussian(n, k, seed=42)
    out = rgs.rgs_qr(W, th, precision="bf16q")
    assert np.all(out["Q"] == rgs.bf16_round(out["Q"]))
    be = metrics.backward_error(W, out["Q"], out["R"])
    assert 1e-4 < be < 2e-2                      # bf16 unit roundoff 2^-9 = 2e-3
    assert 1e-4 < metrics.delta_2(out["S"]) < 2e-2
    assert metrics.cond(out["Q"]) < 5.0          # still well conditioned (Gaussian k = 4m)
    out32 = rgs.rgs_qr(W, th, precision="fp32")
    assert metrics.delta_2(out32["S"]) < 1e-2 * metrics.delta_2(out["S"])


# ---------------------------------------------------------------------------
# Classical projectors of Sec. 1.2 (MGS, CGS, CGS2) -- the Sec. 5.1 references
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fn", ["mgs", "cgs", "cgs2"])
def test_classical_gs_matches_householder_R(fn):
    """In exact arithmetic every Gram-Schmidt variant gives the positive-diagonal
    R factor of W; at kappa = 1e2 in fp64 |R| agrees with LAPACK's Householder
    |R| to rounding."""
    W = _wellcond(500, 30, smin=1e-2, tag=31)
    Q, R = getattr(rgs, fn)(W)
    _, Rh = np.linalg.qr(W)
    assert np.all(np.diag(R) > 0) and np.all(np.tril(R, -1) == 0)
    assert np.linalg.norm(np.abs(R) - np.abs(Rh)) / np.linalg.norm(Rh) <= 1e-12
    assert metrics.backward_error(W, Q, R) <= 1e-14


def test_mgs_loses_orthogonality_at_u_kappa_cgs_at_u_kappa2():
    """MGS: ||I - Q^T Q|| = O(u kappa) (Bjorck 1967); CGS: O(u kappa^2); CGS2: O(u).
    A slip that makes MGS project the original column (i.e. CGS) or drop a term
    of the rank-one updates fails the first bound."""
    W = synth.svd_matrix(2000, 40, 1e-6, tag=32)
    kap = metrics.cond(W)
    lm = metrics.orth_loss_2(rgs.mgs(W)[0])
    lc = metrics.orth_loss_2(rgs.cgs(W)[0])
    l2 = metrics.orth_loss_2(rgs.cgs2(W)[0])
    assert lm <= 10 * U64 * kap
    assert 0.05 * U64 * kap ** 2 <= lc <= 10 * U64 * kap ** 2
    assert lc >= 1e4 * lm
    assert l2 <= 100 * U64


@pytest.mark.parametrize("fn", ["mgs", "cgs", "cgs2"])
def test_classical_gs_float32_variants(fn):
    """The float32 variants compute in float32: R agrees with the fp64 variant to
    O(u32 kappa) (backward-stable R for all three) but not to fp64 accuracy,
    and the loss of orthogonality keeps its order in u32:
    MGS O(u32 kappa), CGS O(u32 kappa^2), CGS2 O(u32)."""
    W = synth.svd_matrix(1000, 30, 1e-2, tag=33)
    kap = metrics.cond(W)
    Q6, R6 = getattr(rgs, fn)(W)
    Q3, R3 = getattr(rgs, fn)(W, np.float32)
    assert Q3.dtype == np.float32 and R3.dtype == np.float32
    dr = np.linalg.norm(R3 - R6) / np.linalg.norm(R6)
    assert 0.05 * U32 <= dr <= 2 * U32 * kap
    loss = metrics.orth_loss_2(Q3)
    bound = {"mgs": 10 * U32 * kap, "cgs": 10 * U32 * kap ** 2, "cgs2": 100 * U32}[fn]
    assert loss <= bound
    if fn == "cgs":
        assert loss >= 10 * U32 * kap          # well above what MGS reaches
    assert metrics.backward_error(W.astype(np.float32), Q3, R3) <= 10 * U32


@pytest.mark.parametrize("kind,n,m,k", [("srht", 3000, 12, 48), ("gaussian", 900, 10, 40), ("rademacher", 1200, 8, 64)])
def test_unique_precision_closed_form(kind, n, m, k):
    """'fp32u': R is the positive-diagonal R factor of qr(Theta W) up to
    float32 rounding amplified by kappa(W); S R = Theta W to float32
    rounding; Q = W R^-1 likewise; every R, S entry is a float32 value."""
    W = _wellcond(n, m, smin=1e-1, tag=11)
    th = sketch.make(kind, n, k, seed=6)
    out = rgs.rgs_qr(W, th, precision="fp32u")
    R, S, Q = out["R"], out["S"], out["Q"]
    assert Q.dtype == np.float32
    assert np.array_equal(R.astype(np.float32).astype(np.float64), R)
    assert np.array_equal(S.astype(np.float32).astype(np.float64), S)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    W32 = W.astype(np.float32).astype(np.float64)
    P = th.apply(W32)
    _, Rq = np.linalg.qr(P)
    Rq = np.sign(np.diag(Rq))[:, None] * Rq
    kappa = metrics.cond(W)
    tol = 50 * U32 * math.sqrt(n) * kappa
    assert np.linalg.norm(R - Rq) / np.linalg.norm(Rq) <= tol
    assert np.linalg.norm(S @ R - P) / np.linalg.norm(P) <= tol
    Qc = np.linalg.solve(Rq.T, W32.T).T
    assert np.linalg.norm(Q.astype(np.float64) - Qc) / np.linalg.norm(Qc) <= tol


def test_unique_precision_rounds_the_sketch_space_steps_in_float32():
    """Against the multi-precision 'fp32' (float32 only in step 3) on the same
    input: the float32 sketches and least squares of 'fp32u' move R by more
    than fp64 rounding and by no more than float32 rounding, and 'fp32u' is
    the farther of the two from the fp64 factorisation."""
    n, m, k = 4096, 24, 96
    W = _wellcond(n, m, smin=1e-1, tag=12)
    th = sketch.SRHT(n, k, seed=7)
    u = rgs.rgs_qr(W, th, precision="fp32u")["R"]
    mp = rgs.rgs_qr(W, th, precision="fp32")["R"]
    d = rgs.rgs_qr(W.astype(np.float32).astype(np.float64), th, precision="fp64")["R"]
    scale = np.linalg.norm(d)
    du, dm = np.linalg.norm(u - d) / scale, np.linalg.norm(mp - d) / scale
    assert 1e-12 < np.linalg.norm(u - mp) / scale < 1e-4
    assert du > dm
