"""Pins of the oracle's a-posteriori certification (Prop. 3.7 and 3.8).

cert_extremes(Theta V, Phi V) returns the extreme singular values of
Theta V X with Phi V X orthonormal; omega_bar builds the bound from them.
They are pinned against facts that do not reuse their QR + SVD route:

* Phi = Theta: Theta V X is orthonormal, so both values are 1 and
  omega_bar = eps* exactly;
* Theta V = c Phi V: both values are |c|;
* the result depends on range(V) only: V -> V M for an invertible M (even an
  ill-conditioned one) leaves it unchanged;
* the squares of the values are the extreme generalized eigenvalues of the
  pencil ((Theta V)^T Theta V, (Phi V)^T Phi V) (scipy's symmetric-definite
  eigensolver), and for two columns the extremes of the Rayleigh quotient
  ||Theta V x||^2 / ||Phi V x||^2 over a fine grid of directions x;
* with Phi an exact isometry and eps* = 0 the bound is the distortion omega
  itself;
* Prop. 3.8: omega_bar <= (1+eps*)(1-eps')^-1 (1+omega) - 1, with eps' the
  distortion of Phi on V;
* Prop. 3.7: with Gaussian Theta, Phi of k = 600 rows and eps* = 1/4, omega
  <= omega_bar on every seeded draw.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import metrics, sketch


def _rng(tag):
    return np.random.default_rng(np.random.SeedSequence([20201110, 77, tag]))


def _V(n, m, tag, cond=1.0):
    rng = _rng(tag)
    U, _ = np.linalg.qr(rng.standard_normal((n, m)))
    Vt, _ = np.linalg.qr(rng.standard_normal((m, m)))
    return (U * np.logspace(0, -np.log10(cond), m)) @ Vt.T


def _distortion(thV, V):
    """Smallest eps with (1-eps)||Vx||^2 <= ||Theta V x||^2 <= (1+eps)||Vx||^2,
    from the generalized eigenvalues of ((Theta V)^T Theta V, V^T V)."""
    ev = scipy.linalg.eigh(thV.T @ thV, V.T @ V, eigvals_only=True)
    return max(1.0 - ev[0], ev[-1] - 1.0)


def test_same_sketch_gives_eps_star():
    V = _V(500, 12, 1)
    th = sketch.make("gaussian", 500, 64, seed=3, sketch_id=0).apply(V)
    smin, smax = metrics.cert_extremes(th, th)
    assert abs(smin - 1.0) < 1e-13 and abs(smax - 1.0) < 1e-13
    for eps in (0.0, 0.05, 0.25):
        assert abs(metrics.omega_bar(th, th, eps) - eps) < 1e-12


def test_scaled_sketch():
    V = _V(300, 7, 2)
    ph = sketch.make("srht", 300, 32, seed=5, sketch_id=1).apply(V)
    for c in (0.5, -1.5, 2.0):
        smin, smax = metrics.cert_extremes(c * ph, ph)
        assert abs(smin - abs(c)) < 1e-12 * abs(c) and abs(smax - abs(c)) < 1e-12 * abs(c)
    # the two branches of the maximum
    assert metrics.omega_bar_from(0.9, 1.0, 0.1) == pytest.approx(1 - 0.9 * 0.81)
    assert metrics.omega_bar_from(1.0, 1.1, 0.1) == pytest.approx(1.1 * 1.21 - 1)


@pytest.mark.parametrize("cond", [1.0, 1e6])
def test_depends_on_range_only(cond):
    n, m = 700, 10
    V = _V(n, m, 3)
    th = sketch.make("gaussian", n, 80, seed=7, sketch_id=0)
    ph = sketch.make("gaussian", n, 80, seed=7, sketch_id=1)
    ref = metrics.cert_extremes(th.apply(V), ph.apply(V))
    M = _V(m, m, 4, cond=cond)
    got = metrics.cert_extremes(th.apply(V @ M), ph.apply(V @ M))
    tol = 1e-13 * cond
    assert abs(got[0] - ref[0]) < tol and abs(got[1] - ref[1]) < tol


@pytest.mark.parametrize("kind", ["gaussian", "srht"])
def test_generalized_eigenvalues(kind):
    n, m, k = 900, 15, 60
    V = _V(n, m, 5, cond=1e3)
    thV = sketch.make(kind, n, k, seed=11, sketch_id=0).apply(V)
    phV = sketch.make(kind, n, k, seed=11, sketch_id=1).apply(V)
    smin, smax = metrics.cert_extremes(thV, phV)
    ev = scipy.linalg.eigh(thV.T @ thV, phV.T @ phV, eigvals_only=True)
    assert abs(smin ** 2 - ev[0]) < 1e-10 and abs(smax ** 2 - ev[-1]) < 1e-10


def test_two_columns_brute_force():
    n, k = 400, 24
    V = _V(n, 2, 6)
    thV = sketch.make("gaussian", n, k, seed=13, sketch_id=0).apply(V)
    phV = sketch.make("gaussian", n, k, seed=13, sketch_id=1).apply(V)
    t = np.linspace(0.0, np.pi, 200001)
    X = np.stack([np.cos(t), np.sin(t)])
    q = np.sum((thV @ X) ** 2, axis=0) / np.sum((phV @ X) ** 2, axis=0)
    smin, smax = metrics.cert_extremes(thV, phV)
    assert abs(smin ** 2 - q.min()) < 1e-8 and abs(smax ** 2 - q.max()) < 1e-8


def test_isometric_phi_gives_omega():
    n, m = 256, 9
    V = _V(n, m, 7, cond=1e2)
    thV = sketch.make("srht", n, 40, seed=17, sketch_id=0).apply(V)
    phV = sketch.make("srht", n, n, seed=17, sketch_id=1).apply(V)   # all rows: an isometry
    assert metrics.omega_bar(thV, phV, 0.0) == pytest.approx(_distortion(thV, V), abs=1e-12)


@pytest.mark.parametrize("tag", range(4))
def test_prop_3_8_upper_bound(tag):
    n, m, k = 800, 12, 120
    V = _V(n, m, 20 + tag, cond=1e2)
    thV = sketch.make("gaussian", n, k, seed=100 + tag, sketch_id=0).apply(V)
    phV = sketch.make("gaussian", n, k, seed=100 + tag, sketch_id=1).apply(V)
    om, eps1 = _distortion(thV, V), _distortion(phV, V)
    assert eps1 < 1.0
    for eps_star in (0.0, 0.05, 0.25):
        bound = (1 + eps_star) / (1 - eps1) * (1 + om) - 1
        assert metrics.omega_bar(thV, phV, eps_star) <= bound * (1 + 1e-12)


def test_prop_3_7_certifies():
    n, m, k = 2000, 20, 600
    for tag in range(6):
        V = _V(n, m, 40 + tag, cond=1e4)
        thV = sketch.make("gaussian", n, k, seed=200 + tag, sketch_id=0).apply(V)
        phV = sketch.make("gaussian", n, k, seed=200 + tag, sketch_id=1).apply(V)
        om = _distortion(thV, V)
        ob = metrics.omega_bar(thV, phV, 0.25)
        assert om <= ob
