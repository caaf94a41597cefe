"""Pins of the oracle's sketching operators (Sec. 2.1).

Each check is tied to something outside the code under test: the textbook
Sylvester-Hadamard matrix (scipy), the exact column norms of an SRHT, the
isometry of a fully sampled SRHT, the N(0, 1/k) law of the Gaussian entries,
the fair, independent +-1/sqrt(k) signs of the Rademacher entries,
the uniformity of a Fisher-Yates draw, and the definition of an
epsilon-embedding (Sec. 2.1, Definition 2.1) checked by brute force.
"""

import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import sketch, metrics


@pytest.mark.parametrize("s", [1, 2, 4, 8, 64, 1024, 4096])
def test_fwht_matches_sylvester_hadamard(s):
    g = np.random.Generator(np.random.PCG64(s))
    x = g.integers(-1000, 1000, size=(s, 3)).astype(np.float64)
    ref = scipy.linalg.hadamard(s).astype(np.float64) @ x if s > 1 else x
    assert np.array_equal(sketch.fwht(x), ref)          # exact on integers


@pytest.mark.parametrize("n,k", [(1000, 64), (1024, 1024), (37, 16), (4096, 300)])
def test_srht_frobenius_norm_is_exactly_n(n, k):
    th = sketch.SRHT(n, k, seed=3)
    T = th.materialize()
    # every entry is +-1/sqrt(k): each column has squared norm exactly 1
    assert np.allclose(np.abs(T) * math.sqrt(k), 1.0, atol=0, rtol=1e-15)
    assert abs((T ** 2).sum() - n) <= 1e-12 * n


@pytest.mark.parametrize("n,k", [(1000, 64), (37, 16), (4096, 300)])
def test_srht_apply_equals_dense_definition(n, k):
    th = sketch.SRHT(n, k, seed=11, sketch_id=1, instance=4)
    s = th.s
    H = scipy.linalg.hadamard(s).astype(np.float64)
    dense = H[th.rows][:, :n] * th.d[None, :] / math.sqrt(k)
    assert np.array_equal(dense, th.materialize())
    X = np.random.Generator(np.random.PCG64(1)).standard_normal((n, 5))
    np.testing.assert_allclose(th.apply(X), dense @ X, rtol=1e-12, atol=1e-12)


def test_srht_full_sample_is_an_isometry():
    n = 200                       # s = 256
    th = sketch.SRHT(n, 256, seed=5)
    T = th.materialize()
    np.testing.assert_allclose(T.T @ T, np.eye(n) * 256 / 256, atol=1e-12)


def test_srht_rows_distinct_and_in_range():
    for s, k in [(8, 8), (1024, 1000), (1 << 22, 2048)]:
        rows = sketch.srht_rows(s, k, 42, 0, 0)
        assert rows.min() >= 0 and rows.max() < s
        assert np.unique(rows).size == k
    assert np.array_equal(np.sort(sketch.srht_rows(16, 16, 1, 0, 0)), np.arange(16))


def test_fisher_yates_draw_is_uniform_over_ordered_pairs():
    # s = 5, k = 2: 20 ordered pairs, each with probability 1/20
    counts = {}
    trials = 8000
    for seed in range(trials):
        r = tuple(sketch.srht_rows(5, 2, seed, 0, 0))
        counts[r] = counts.get(r, 0) + 1
    assert len(counts) == 20
    obs = np.array(list(counts.values()))
    chi2 = ((obs - trials / 20) ** 2 / (trials / 20)).sum()
    assert chi2 < scipy.stats.chi2.ppf(0.999, 19)


def test_srht_signs_balanced():
    d = sketch.srht_signs(1 << 16, 42, 0, 0)
    assert set(np.unique(d)) == {-1.0, 1.0}
    assert abs(d.mean()) < 5 * (1 << 16) ** -0.5


def test_gaussian_entries_are_n01_over_k():
    k = 64
    T = sketch.gaussian_block(k, 42, 0, 0, 0, k, 0, 4096) * math.sqrt(k)
    z = T.reshape(-1)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3


def test_gaussian_block_views_agree():
    k = 16
    full = sketch.gaussian_block(k, 9, 1, 2, 0, k, 0, 103)
    part = sketch.gaussian_block(k, 9, 1, 2, 3, 11, 5, 94)
    assert np.array_equal(full[3:11, 5:94], part)
    th = sketch.Gaussian(103, k, seed=9, sketch_id=1, instance=2, cache_limit=0)
    X = np.random.Generator(np.random.PCG64(2)).standard_normal((103, 3))
    np.testing.assert_allclose(th.apply(X), full @ X, rtol=1e-13, atol=1e-13)


def test_gaussian_expected_gram_is_identity():
    # E[Theta^T Theta] = I: Monte-Carlo over sketch ids
    n, k, reps = 8, 32, 400
    acc = np.zeros((n, n))
    for t in range(reps):
        T = sketch.gaussian_block(k, 42, 10 + t, 0, 0, k, 0, n)
        acc += T.T @ T
    acc /= reps
    # entries of the mean have sd about sqrt(1/(k reps)) off the diagonal
    assert np.max(np.abs(acc - np.eye(n))) < 6 * math.sqrt(2.0 / (k * reps))


def test_rademacher_entries_and_frobenius_norm():
    # entries are exactly +-1/sqrt(k), so ||Theta||_F^2 = n exactly
    for n, k in ((1000, 64), (37, 16), (4099, 300)):
        T = sketch.make("rademacher", n, k, seed=3).materialize()
        assert np.all(np.abs(T) == 1.0 / math.sqrt(k))
        assert abs((T ** 2).sum() - n) < 1e-9 * n


def test_rademacher_signs_are_fair_independent_coins():
    k, n = 64, 8192
    S = sketch.rademacher_block(k, 42, 0, 0, 0, k, 0, n) * math.sqrt(k)
    b = (S.reshape(-1) < 0).astype(np.float64)
    assert abs(b.mean() - 0.5) < 5 * 0.5 / math.sqrt(b.size)
    # neighbours inside one 32-bit word, across words and across Philox calls
    for lag in (1, 31, 32, 127, 128):
        c = np.mean(S[:, lag:] * S[:, :-lag])
        assert abs(c) < 5 / math.sqrt(k * (n - lag))
    # rows and sketch ids are independent
    assert abs(np.mean(S[1:] * S[:-1])) < 5 / math.sqrt((k - 1) * n)
    S2 = sketch.rademacher_block(k, 42, 1, 0, 0, k, 0, n) * math.sqrt(k)
    assert abs(np.mean(S * S2)) < 5 / math.sqrt(k * n)
    # runs test on one long row: number of sign changes of a fair coin sequence
    row = sketch.rademacher_block(1, 7, 0, 0, 0, 1, 0, 1 << 16)[0]
    changes = np.count_nonzero(row[1:] != row[:-1])
    assert abs(changes - (row.size - 1) / 2) < 5 * math.sqrt((row.size - 1) / 4)


def test_rademacher_block_views_and_apply_agree():
    k, n = 24, 1000
    full = sketch.rademacher_block(k, 9, 1, 2, 0, k, 0, n)
    assert np.array_equal(full[3:11, 129:517], sketch.rademacher_block(k, 9, 1, 2, 3, 11, 129, 517))
    th = sketch.Rademacher(n, k, seed=9, sketch_id=1, instance=2, cache_limit=0)
    X = np.random.Generator(np.random.PCG64(2)).standard_normal((n, 3))
    np.testing.assert_allclose(th.apply(X), full @ X, rtol=1e-13, atol=1e-13)


def test_rademacher_expected_gram_is_identity():
    n, k, reps = 8, 32, 400
    acc = np.zeros((n, n))
    for t in range(reps):
        T = sketch.rademacher_block(k, 42, 10 + t, 0, 0, k, 0, n)
        acc += T.T @ T
    acc /= reps
    assert np.allclose(np.diag(acc), 1.0, rtol=0, atol=1e-15)    # exactly 1: entries are +-1/sqrt(k)
    assert np.max(np.abs(acc - np.eye(n))) < 6 * math.sqrt(1.0 / (k * reps))


def _bf16_nearest_even_bruteforce(x):
    """Nearest bfloat16 to the double x by exact integer arithmetic on its
    significand: the two grid neighbours, then the nearer (even on a tie)."""
    m, e = math.frexp(abs(x))                 # x = m 2^e, 0.5 <= m < 1
    sig = int(m * (1 << 53))                  # exact 53-bit significand
    lo, rem = divmod(sig, 1 << 45)            # 8 significant bits kept (1 implicit + 7)
    half = 1 << 44
    up = rem > half or (rem == half and (lo & 1))
    q = (lo + (1 if up else 0)) * (1 << 45)
    return math.copysign(math.ldexp(q / float(1 << 53), e), x)


def test_bf16_round_f64_is_nearest_even():
    g = np.random.Generator(np.random.PCG64(5))
    x = g.standard_normal(20000) * np.exp(g.uniform(-20, 20, 20000))
    # exact ties and near-ties in both directions
    base = sketch.bf16_round_f64(x)
    ulp = np.ldexp(1.0, np.frexp(base)[1] - 8)          # bf16 spacing at base
    x = np.concatenate([x, base + ulp / 2, base - ulp / 2, base + ulp / 2 * (1 + 2 ** -40)])
    got = sketch.bf16_round_f64(x)
    ref = np.array([_bf16_nearest_even_bruteforce(float(v)) for v in x])
    assert np.array_equal(got, ref)
    assert np.all((got.view(np.uint64) & np.uint64((1 << 45) - 1)) == 0)


def test_gaussian_bf16_entries_are_rounded_gaussians():
    k, n = 48, 3000
    G = sketch.gaussian_block(k, 42, 0, 0, 0, k, 0, n)
    B = sketch.make("gaussian_bf16", n, k, seed=42).materialize()
    assert np.all(np.abs(B - G) <= 2.0 ** -8 * np.abs(G) + 1e-300)
    Z = sketch.gaussian_bf16_block(1, 42, 0, 0, 0, k, 0, n)              # unscaled (k = 1)
    assert np.all((Z.view(np.uint64) & np.uint64((1 << 45) - 1)) == 0)   # on the bf16 grid before the scale
    assert np.array_equal(B, Z / math.sqrt(k))
    z = Z.reshape(-1)
    assert abs(z.mean()) < 5 / math.sqrt(z.size) and abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)


@pytest.mark.parametrize("kind", ["gaussian", "srht", "rademacher", "gaussian_bf16"])
def test_omega_equals_bruteforce_embedding_distortion(kind):
    # Definition 2.1: omega is the smallest eps with
    # |<x,y> - <Theta x, Theta y>| <= eps ||x|| ||y|| for all x, y in range(V).
    n, d, k = 48, 2, 24
    g = np.random.Generator(np.random.PCG64(3))
    V, _ = np.linalg.qr(g.standard_normal((n, d)))
    th = sketch.make(kind, n, k, seed=8)
    TV = th.apply(V)
    ang = np.linspace(0.0, np.pi, 721)
    A = np.stack([np.cos(ang), np.sin(ang)], axis=1)             # unit coefficient vectors
    X = A @ V.T                                                  # unit vectors in range(V)
    TX = A @ TV.T
    dev = np.abs(X @ X.T - TX @ TX.T)
    brute = dev.max()
    om = metrics.omega(TV, V)
    assert brute <= om * (1 + 1e-12)
    assert brute >= om * (1 - 1e-4)


@pytest.mark.parametrize("n,k", [(1000, 64), (4096, 128), (777, 33)])
def test_srht_float32_apply_is_exact_on_small_integers(n, k):
    """Unique-precision sketches (float32 arithmetic): on small-integer input
    every butterfly of the float32 FWHT is exact (|values| <= n * 8 < 2**24),
    so the float32 apply must equal the integer transform H_s D x, computed
    here from the dense +-1 definition in int64, times float32(k**-1/2), as
    one float32 product per entry -- bit for bit."""
    th = sketch.SRHT(n, k, seed=5)
    x = np.random.default_rng(n).integers(-8, 9, size=n)
    signs = np.rint(th.materialize() * math.sqrt(k)).astype(np.int64)   # +-1 entries of H_s D, sampled rows
    ints = signs @ x
    want = ints.astype(np.float32) * np.float32(1.0 / math.sqrt(k))
    got = th.apply(x.astype(np.float32), np.float32)
    assert got.dtype == np.float32
    assert np.array_equal(got, want)


@pytest.mark.parametrize("kind", ["gaussian", "rademacher", "srht"])
def test_float32_apply_within_the_float32_error_bound(kind):
    """The float32 apply of each sketch against the fp64 one: every entry of
    Theta x rounded once to float32, then float32 sums, so |err| <= (n + 2) u32
    sum_l |theta_jl x_l| (the standard bound for a computed inner product)."""
    n, k = 1500, 40
    th = sketch.make(kind, n, k, seed=9)
    x = np.random.default_rng(3).standard_normal(n).astype(np.float32)
    y32 = th.apply(x, np.float32)
    assert y32.dtype == np.float32
    y64 = th.apply(x.astype(np.float64))
    bound = (n + 2) * 2.0 ** -24 * (np.abs(th.materialize()) @ np.abs(x.astype(np.float64)))
    assert np.all(np.abs(y32.astype(np.float64) - y64) <= bound)
    assert np.any(y32.astype(np.float64) != y64)   # the float32 rounding is there
