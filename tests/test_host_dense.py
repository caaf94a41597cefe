"""Host-side dense fp64 routines of the certification (Cholesky, triangular
inverse, symmetric eigenvalue extremes), compiled with g++ into a small
driver and checked against numpy/LAPACK on seeded matrices.  No GPU."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_05090_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "rgs_dense.hpp"
int main() {
    char op[8]; int m;
    while (std::scanf("%7s %d", op, &m) == 2) {
        std::vector<double> A((size_t)m * m);
        for (auto& v : A) if (std::scanf("%lf", &v) != 1) return 2;
        if (op[0] == 'e') {
            double lo = 0, hi = 0;
            bool ok = rgs::dense::sym_eig_extremes(A, m, lo, hi);
            std::printf("%d %.17g %.17g\n", ok ? 1 : 0, lo, hi);
        } else if (op[0] == 'c') {
            bool ok = rgs::dense::cholesky_upper(A, m);
            std::printf("%d", ok ? 1 : 0);
            for (double v : A) std::printf(" %.17g", v);
            std::printf("\n");
        } else {
            std::vector<double> X = rgs::dense::upper_inverse(A, m);
            std::printf("1");
            for (double v : X) std::printf(" %.17g", v);
            std::printf("\n");
        }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("dense")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I" + CSRC, str(src), os.path.join(CSRC, "rgs_dense.cpp"),
                    "-o", str(exe)], check=True)
    return str(exe)


def _run(driver, op, A):
    m = A.shape[0]
    text = "%s %d %s\n" % (op, m, " ".join("%.17g" % v for v in A.flatten(order="F")))
    out = subprocess.run([driver], input=text.encode(), stdout=subprocess.PIPE, check=True).stdout.decode().split()
    return int(out[0]), np.array([float(v) for v in out[1:]])


def _rng(tag):
    return np.random.default_rng(np.random.SeedSequence([20201110, 91, tag]))


def _sym(m, tag, spread=1.0):
    rng = _rng(tag)
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    ev = 1.0 + spread * rng.uniform(-0.5, 0.5, m)
    return (U * ev) @ U.T


@pytest.mark.parametrize("m,spread,tag", [(1, 1.0, 0), (2, 1.0, 1), (3, 0.5, 2), (17, 1e-6, 3), (100, 0.8, 4),
                                          (64, 3.0, 5), (257, 0.9, 8)])
def test_eig_extremes_match_lapack(driver, m, spread, tag):
    A = _sym(m, tag, spread)
    if tag == 5:
        A -= 2.0 * np.eye(m)          # negative eigenvalues too
    ok, (lo, hi) = _run(driver, "e", A)
    ev = np.linalg.eigvalsh(A)
    assert ok == 1
    assert abs(lo - ev[0]) <= 1e-13 * max(1.0, abs(ev[-1])) * m
    assert abs(hi - ev[-1]) <= 1e-13 * max(1.0, abs(ev[-1])) * m


def test_eig_extremes_reads_lower_triangle_only(driver):
    A = _sym(20, 6)
    B = np.tril(A) + np.triu(np.full_like(A, 1e9), 1)   # garbage above the diagonal
    ok, (lo, hi) = _run(driver, "e", B)
    ev = np.linalg.eigvalsh(A)
    assert ok == 1 and abs(lo - ev[0]) < 1e-12 and abs(hi - ev[-1]) < 1e-12


def test_eig_special_cases(driver):
    ok, (lo, hi) = _run(driver, "e", np.eye(9) * 3.0)
    assert ok == 1 and lo == pytest.approx(3.0, abs=1e-14) and hi == pytest.approx(3.0, abs=1e-14)
    D = np.diag(np.arange(1.0, 11.0))
    ok, (lo, hi) = _run(driver, "e", D)
    assert ok == 1 and lo == pytest.approx(1.0, abs=1e-13) and hi == pytest.approx(10.0, abs=1e-13)
    N = _sym(5, 7)
    N[3, 1] = np.nan
    ok, _ = _run(driver, "e", N)
    assert ok == 0


@pytest.mark.parametrize("m", [1, 7, 50, 203])
def test_cholesky_and_inverse(driver, m):
    rng = _rng(10 + m)
    Z = rng.standard_normal((3 * m, m))
    G = Z.T @ Z
    ok, t = _run(driver, "c", G)
    T = t.reshape((m, m), order="F")
    assert ok == 1
    assert np.all(np.tril(T, -1) == 0) and np.all(np.diag(T) > 0)
    np.testing.assert_allclose(T.T @ T, G, rtol=0, atol=1e-12 * np.abs(G).max())
    # T agrees with the R factor of a Householder QR of Z (up to row signs)
    Rq = np.linalg.qr(Z, mode="r")
    np.testing.assert_allclose(T, np.sign(np.diag(Rq))[:, None] * Rq, rtol=0, atol=1e-10 * np.abs(Rq).max())
    ok, x = _run(driver, "i", T)
    X = x.reshape((m, m), order="F")
    np.testing.assert_allclose(T @ X, np.eye(m), rtol=0, atol=1e-12 * m)
    assert np.all(np.tril(X, -1) == 0)


def test_cholesky_rejects_indefinite(driver):
    G = _sym(6, 20) - np.diag([0, 0, 0, 0, 0, 5.0])   # one eigenvalue below zero
    ok, _ = _run(driver, "c", G)
    assert ok == 0
