"""GPU parity of the RGS QR path (Algorithm 2) and its sketches against the oracle.

Every test calls the HIP library through the C ABI (ctypes binding) on inputs
drawn by ``synth`` and compares with ``oracle`` on the same inputs:

* the sketch generated on the device (Gaussian / SRHT / identity) entry by
  entry: integer parts (SRHT signs and rows) bit for bit, Box-Muller values
  within a few ulps of the working precision;
* Theta X on ragged sizes (several 4096-row blocks plus a partial one);
* the fp64 factorisation (tolerance 1e-12, read as in the design notes: on
  backward errors, on forward agreement for a well-conditioned companion,
  and column-wise within 10 sqrt(i) u kappa(W_1:i) otherwise);
* the fp32/fp64-LS factorisation against the oracle's fp32 model;
* breakdown and non-finite inputs, bitwise run-to-run determinism.
"""

import math

import numpy as np
import pytest

import synth
from oracle import metrics, rgs as orgs, sketch as osk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


def to_dev(A, dtype):
    """numpy (n, m) -> column-major device tensor."""
    A = np.asarray(A)
    if A.ndim == 1:
        return torch.from_numpy(np.ascontiguousarray(A)).to(dtype=dtype, device="cuda")
    return torch.from_numpy(np.ascontiguousarray(A.T)).to(dtype=dtype, device="cuda").t()


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def run_qr(h, W, k, sketch, prec, seed=42, sketch_id=0, flags=0):
    rgs = _rgs()
    n, m = W.shape
    dt = torch.float64 if prec == "fp64" else torch.float32
    Wd = to_dev(W, dt)
    Q = rgs.colmajor(n, m, dt)
    R = rgs.colmajor(m, m, torch.float64)
    S = rgs.colmajor(k, m, torch.float64)
    d = rgs.qr_desc(n, m, k, sketch=sketch, prec=prec, seed=seed, sketch_id=sketch_id, flags=flags)
    rep = rgs.rgs_qr(h, d, Wd, Q, R, S)
    torch.cuda.synchronize()
    return rep, to_host(Q), to_host(R), to_host(S)


# ---------------------------------------------------------------------------
# Sketch generation and application
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gaussian_materialize_matches_oracle(gpu_handle, prec):
    rgs = _rgs()
    n, k = 1000, 48
    d = rgs.qr_desc(n, 1, k, sketch="gaussian", prec=prec, seed=123, sketch_id=3, instance=5)
    out = rgs.colmajor(k, n, torch.float64)
    rgs.rgs_sketch_materialize(gpu_handle, d, 0, k, 0, n, out)
    got = to_host(out)
    ref = osk.gaussian_block(k, 123, 3, 5, 0, k, 0, n)
    err = np.abs(got - ref)
    if prec == "fp64":
        assert err.max() <= 8 * U64 * np.abs(ref).max()
    else:
        # fp32 Box-Muller (log2 / sqrt / sincospi in fp32): a few fp32 ulps of max |theta|
        assert err.max() <= 16 * U32 * np.abs(ref).max()
    sub = rgs.colmajor(7, 19, torch.float64)
    rgs.rgs_sketch_materialize(gpu_handle, d, 5, 12, 401, 420, sub)
    assert np.array_equal(to_host(sub), got[5:12, 401:420])


def test_srht_materialize_is_bit_exact(gpu_handle):
    rgs = _rgs()
    n, k = 3000, 200                       # s = 4096, P-SRHT on a ragged n
    d = rgs.qr_desc(n, 1, k, sketch="srht", prec="fp64", seed=77, sketch_id=1, instance=2)
    out = rgs.colmajor(k, n, torch.float64)
    rgs.rgs_sketch_materialize(gpu_handle, d, 0, k, 0, n, out)
    ref = osk.SRHT(n, k, seed=77, sketch_id=1, instance=2).materialize()
    assert np.array_equal(to_host(out), ref)


@pytest.mark.parametrize("sketch,n,k", [("srht", 10000, 256), ("srht", 300, 64), ("gaussian", 9000, 96),
                                        ("identity", 777, 777), ("rademacher", 9000, 96), ("rademacher", 1000, 40),
                                        ("srht", 20000, 5000)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sketch_apply_matches_oracle(gpu_handle, sketch, n, k, prec):
    rgs = _rgs()
    g = np.random.Generator(np.random.PCG64(n + k))
    X = g.standard_normal((n, 5))
    dt = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        X = X.astype(np.float32).astype(np.float64)
    d = rgs.qr_desc(n, 1, k, sketch=sketch, prec=prec, seed=9)
    Y = rgs.colmajor(k, 5, torch.float64)
    rgs.rgs_sketch_apply(gpu_handle, d, to_dev(X, dt), Y)
    ref = osk.make(sketch, n, k, seed=9).apply(X)
    scale = np.abs(ref).max()
    tol = 1e-13 if prec == "fp64" else 2e-6
    assert np.abs(to_host(Y) - ref).max() <= tol * scale


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rademacher_materialize_is_exact(gpu_handle, prec):
    """Entries are +-1/sqrt(k) from Philox bits: bit for bit equal to the oracle's."""
    rgs = _rgs()
    n, k = 1000, 40
    d = rgs.qr_desc(n, 1, k, sketch="rademacher", prec=prec, seed=123, sketch_id=3, instance=5)
    out = rgs.colmajor(k, n, torch.float64)
    rgs.rgs_sketch_materialize(gpu_handle, d, 0, k, 0, n, out)
    ref = osk.rademacher_block(k, 123, 3, 5, 0, k, 0, n)
    assert np.array_equal(to_host(out), ref)
    sub = rgs.colmajor(7, 300, torch.float64)
    rgs.rgs_sketch_materialize(gpu_handle, d, 5, 12, 129, 429, sub)
    assert np.array_equal(to_host(sub), ref[5:12, 129:429])


def test_rademacher_fused_sketch_large_n(gpu_handle):
    """n above the split threshold: the Rademacher sketch runs inside the
    projection kernel (8192-row blocks, ragged tail)."""
    n, m, k = (1 << 20) + 333, 6, 64
    W = synth.svd_matrix(n, m, 1e-2, tag=19)
    rep, Q, R, S = run_qr(gpu_handle, W, k, "rademacher", "fp64")
    assert rep.status == 0
    th = osk.make("rademacher", n, k, seed=42)
    ref = orgs.rgs_qr(W, th)
    assert np.linalg.norm(R - ref["R"]) / np.linalg.norm(ref["R"]) <= 1e-12
    assert np.linalg.norm(S - ref["S"]) / np.linalg.norm(ref["S"]) <= 1e-12
    assert np.linalg.norm(S - th.apply(Q)) <= 1e-12 * np.linalg.norm(S)
    assert metrics.backward_error(W, Q, R) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gaussian_fused_sketch_large_n(gpu_handle, prec):
    """n above the split threshold (2^20 rows): the drawn Gaussian sketch of
    step 4 runs inside the projection kernel (8192-row blocks, ragged tail), the
    path every single Gaussian QR of 2^20 rows or more takes.  fp64: R, S vs the
    oracle to 1e-12 and S = Theta Q; fp32: against the oracle's fp32 model,
    column by column within sqrt(i) u32 kappa(W_1:i), and S = Theta Q to the
    rounding of the stored q."""
    n, m, k = (1 << 20) + 333, 8, 64
    W = synth.svd_matrix(n, m, 1e-2, tag=20)
    if prec == "fp32":
        W = W.astype(np.float32).astype(np.float64)
    print("fused Gaussian sketch, n %d m %d k %d %s" % (n, m, k, prec), flush=True)
    rep, Q, R, S = run_qr(gpu_handle, W, k, "gaussian", prec)
    assert rep.status == 0
    th = osk.Gaussian(n, k, seed=42, cache_limit=k * n)      # entries drawn once, then reused
    ref = orgs.rgs_qr(W, th, precision=prec)
    SQ = th.apply(Q)
    if prec == "fp64":
        assert np.linalg.norm(R - ref["R"]) / np.linalg.norm(ref["R"]) <= 1e-12
        assert np.linalg.norm(S - ref["S"]) / np.linalg.norm(ref["S"]) <= 1e-12
        assert np.linalg.norm(S - SQ) <= 1e-12 * np.linalg.norm(S)
        assert metrics.backward_error(W, Q, R) <= 1e-12
    else:
        # the fp32 path draws its entries with fp32 Box-Muller, within 16 fp32 ulps of
        # the oracle's fp64 entries: a sketch perturbed by up to 16 u32 relative on top
        # of the rounding noise u32 kappa of step 3
        for i in range(m):
            kap = metrics.cond(W[:, : i + 1])
            ri = ref["R"][: i + 1, i]
            assert np.linalg.norm(R[: i + 1, i] - ri) <= (math.sqrt(i + 1) * kap + 16) * U32 * np.linalg.norm(ri), i
        assert np.linalg.norm(S - SQ) <= 1e-5 * np.linalg.norm(S)
        assert metrics.backward_error(W, Q, R) <= 1e-6
        assert abs(metrics.delta_2(S) - metrics.delta_2(ref["S"])) <= 1e-5


# ---------------------------------------------------------------------------
# fp64 factorisation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sketch,n,m,k", [("gaussian", 16384, 64, 256), ("srht", 10000, 40, 256),
                                          ("srht", 4096 * 3 + 17, 24, 128), ("rademacher", 4096 * 3 + 17, 24, 128),
                                          ("srht", 8192 * 3 + 17, 24, 5000), ("gaussian", 9000, 12, 4500)])
def test_fp64_qr_wellconditioned_forward_parity(gpu_handle, sketch, n, m, k):
    W = synth.svd_matrix(n, m, 1e-2, tag=11)
    rep, Q, R, S = run_qr(gpu_handle, W, k, sketch, "fp64")
    assert rep.status == 0 and rep.failed_column == -1
    ref = orgs.rgs_qr(W, osk.make(sketch, n, k, seed=42))
    assert np.linalg.norm(R - ref["R"]) / np.linalg.norm(ref["R"]) <= 1e-12
    assert np.abs(Q - ref["Q"]).max() <= 1e-12 * np.abs(ref["Q"]).max()
    assert np.linalg.norm(S - ref["S"]) / np.linalg.norm(ref["S"]) <= 1e-12
    assert metrics.backward_error(W, Q, R) <= 1e-12


def test_fp64_qr_config1_parity(gpu_handle):
    # n = 16384, m = 64, sigma 1 -> 1e-6, Gaussian k = 256.
    n, m, k = 16384, 64, 256
    W = synth.svd_matrix(n, m, 1e-6, tag=0)
    rep, Q, R, S = run_qr(gpu_handle, W, k, "gaussian", "fp64", flags=1)
    assert rep.status == 0
    th = osk.Gaussian(n, k, seed=42)
    ref = orgs.rgs_qr(W, th)
    # backward errors on both sides
    assert metrics.backward_error(W, Q, R) <= 1e-12
    assert metrics.backward_error(W, ref["Q"], ref["R"]) <= 1e-12
    assert metrics.delta_tilde_F(th.apply(W), S, R) <= 1e-12
    # column-wise forward agreement within 10 sqrt(i) u kappa(W_1:i)
    for i in range(m):
        kap = metrics.cond(W[:, : i + 1])
        assert np.linalg.norm(Q[:, i] - ref["Q"][:, i]) <= 10 * math.sqrt(i + 1) * U64 * kap * max(
            1.0, np.linalg.norm(ref["Q"][:, i]))
    # step-8 diagnostics reported by the library agree with the oracle's metrics on its outputs
    assert abs(rep.delta_F - metrics.delta_F(S)) <= 1e-12 + 1e-6 * metrics.delta_F(S)


def test_identity_sketch_reproduces_householder_R(gpu_handle):
    n, m = 512, 16
    W = synth.svd_matrix(n, m, 1e-2, tag=12)
    rep, Q, R, S = run_qr(gpu_handle, W, n, "identity", "fp64")
    _, Rh = np.linalg.qr(W)
    assert np.linalg.norm(np.abs(R) - np.abs(Rh)) / np.linalg.norm(Rh) <= 1e-12
    assert metrics.orth_loss_2(Q) <= 1e-12


# ---------------------------------------------------------------------------
# fp32 projection / fp64 least squares
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sketch", ["srht", "gaussian", "rademacher"])
def test_fp32_qr_matches_oracle_fp32_model(gpu_handle, sketch):
    n, m, k = 4096 * 5 + 100, 48, 192
    W = synth.svd_matrix(n, m, 1e-3, tag=13).astype(np.float32).astype(np.float64)
    rep, Q, R, S = run_qr(gpu_handle, W, k, sketch, "fp32")
    assert rep.status == 0
    ref = orgs.rgs_qr(W, osk.make(sketch, n, k, seed=42), precision="fp32")
    # own-output tolerances (fp32 path)
    assert metrics.backward_error(W, Q, R) <= 1e-5
    assert metrics.delta_2(S) <= 1e-4
    # agreement with the oracle's fp32 model, column by column: both carry rounding
    # noise of order u32 kappa(W_1:i) in column i (the oracle's own fp32 and fp64
    # runs differ by at most 0.03 sqrt(i) u32 kappa(W_1:i) ||R(:, i)|| on this input);
    # the Gaussian entries of the fp32 path are fp32 Box-Muller values, within 16 fp32
    # ulps of the oracle's fp64 ones, a further relative perturbation of up to 16 u32
    extra = 16 if sketch == "gaussian" else 0
    for i in range(m):
        kap = metrics.cond(W[:, : i + 1])
        ri = ref["R"][: i + 1, i]
        assert np.linalg.norm(R[: i + 1, i] - ri) <= (math.sqrt(i + 1) * kap + extra) * U32 * np.linalg.norm(ri), i
    assert abs(metrics.delta_2(S) - metrics.delta_2(ref["S"])) <= 1e-4
    # S is the sketch of the stored Q (up to fp32 rounding of the stored q)
    SQ = osk.make(sketch, n, k, seed=42).apply(Q)
    assert np.linalg.norm(S - SQ) <= 1e-5 * np.linalg.norm(S)


def test_fp32_qr_srht_ragged_small(gpu_handle):
    n, m, k = 777, 12, 64
    W = synth.svd_matrix(n, m, 1e-2, tag=14).astype(np.float32).astype(np.float64)
    rep, Q, R, S = run_qr(gpu_handle, W, k, "srht", "fp32")
    ref = orgs.rgs_qr(W, osk.SRHT(n, k, seed=42), precision="fp32")
    assert np.linalg.norm(R - ref["R"]) / np.linalg.norm(ref["R"]) <= 1e-5
    assert metrics.backward_error(W, Q, R) <= 1e-6


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sketch,prec", [("srht", "fp64"), ("srht", "fp32"), ("gaussian", "fp32")])
def test_step1_chunks_on_second_stream(gpu_handle, sketch, prec):
    """Step 1 (P = Theta W) runs in chunks of columns (64 here: 64 row groups x
    k = 2048 fp64 partials per column), all after the first on a second stream
    beside the first columns' steps, each column waiting for its chunk.  RGS
    column i depends on columns <= i only, so the first chunk's columns equal
    a call on those columns alone bit for bit; and S R = Theta W holds for
    every column (a column read from an unfinished chunk would break it)."""
    rgs = _rgs()
    n, m, k = (1 << 18) + 123, 150, 2048
    W = synth.svd_matrix(n, m, 1e-2, tag=71)
    if prec == "fp32":
        W = W.astype(np.float32).astype(np.float64)
    rep, Q, R, S = run_qr(gpu_handle, W, k, sketch, prec, seed=5)
    rep1, Q1, R1, S1 = run_qr(gpu_handle, W[:, :64], k, sketch, prec, seed=5)
    assert rep.status == 0 and rep1.status == 0
    assert np.array_equal(Q[:, :64], Q1) and np.array_equal(R[:64, :64], R1) and np.array_equal(S[:, :64], S1)
    dt = torch.float64 if prec == "fp64" else torch.float32
    P = rgs.colmajor(k, m, torch.float64)
    rgs.rgs_sketch_apply(gpu_handle, rgs.qr_desc(n, m, k, sketch=sketch, prec=prec, seed=5), to_dev(W, dt), P)
    P = to_host(P)
    err = np.linalg.norm(S @ R - P, axis=0) / np.linalg.norm(P, axis=0)
    assert err.max() <= (1e-11 if prec == "fp64" else 1e-5), err.max()   # fp32: rounding of q' in step 3


def test_breakdown_reports_column(gpu_handle):
    rgs = _rgs()
    n, m, k = 8192, 10, 64
    W = synth.svd_matrix(n, m, 1e-2, tag=15)
    W[:, 6] = W[:, 2]
    rep, Q, R, S = run_qr(gpu_handle, W, k, "srht", "fp64")
    assert rep.status == rgs.RGS_EBREAKDOWN and rep.failed_column == 6
    ref = orgs.rgs_qr(W[:, :6], osk.SRHT(n, k, seed=42))
    assert np.linalg.norm(R[:6, :6] - ref["R"]) <= 1e-12 * np.linalg.norm(ref["R"])


def test_nonfinite_input(gpu_handle):
    rgs = _rgs()
    n, m, k = 5000, 5, 32
    W = synth.svd_matrix(n, m, 1e-2, tag=16)
    W[123, 3] = np.inf
    rep, *_ = run_qr(gpu_handle, W, k, "gaussian", "fp64")
    assert rep.status == rgs.RGS_ENONFINITE and rep.failed_column == 3


def test_single_column(gpu_handle):
    n, k = 4096, 8
    W = synth.svd_matrix(n, 1, 1.0, tag=17)
    rep, Q, R, S = run_qr(gpu_handle, W, k, "srht", "fp64")
    p = osk.SRHT(n, k, seed=42).apply(W[:, 0])
    assert abs(R[0, 0] - np.linalg.norm(p)) <= 1e-14 * np.linalg.norm(p)
    assert np.abs(Q[:, 0] - W[:, 0] / R[0, 0]).max() <= 1e-15


def test_invalid_arguments_rejected(gpu_handle):
    rgs = _rgs()
    n, m, k = 1000, 10, 8                      # k < m
    dt = torch.float64
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_qr(gpu_handle, rgs.qr_desc(n, m, k, prec="fp64"), rgs.colmajor(n, m, dt), rgs.colmajor(n, m, dt),
                   rgs.colmajor(m, m, dt), rgs.colmajor(k, m, dt))
    assert e.value.status == rgs.RGS_EINVAL
    with pytest.raises(rgs.RgsError):         # SRHT with k > s
        rgs.rgs_qr(gpu_handle, rgs.qr_desc(100, 4, 200, sketch="srht", prec="fp64"),
                   rgs.colmajor(100, 4, dt), rgs.colmajor(100, 4, dt), rgs.colmajor(4, 4, dt),
                   rgs.colmajor(200, 4, dt))


@pytest.mark.parametrize("n,m,k", [(100, 0, 8), (0, 1, 1), (0, 0, 0)])
def test_empty_inputs_rejected(gpu_handle, n, m, k):
    """An empty factorisation (no columns, or no rows) is an argument error,
    reported before any device work."""
    rgs = _rgs()
    dt = torch.float64
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_qr(gpu_handle, rgs.qr_desc(n, m, k, prec="fp64"), rgs.colmajor(n, m, dt), rgs.colmajor(n, m, dt),
                   rgs.colmajor(m, m, dt), rgs.colmajor(k, m, dt))
    assert e.value.status == rgs.RGS_EINVAL


def test_empty_batches_rejected(gpu_handle):
    rgs = _rgs()
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_qr_batched(gpu_handle, [], sketch="srht", prec="fp32")
    assert e.value.status == rgs.RGS_EINVAL
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_gmres_batched(gpu_handle, [], rgs.gmres_desc(10, 32, 1e-6, sketch="srht", prec="fp32"))
    assert e.value.status == rgs.RGS_EINVAL


def test_one_row_one_column(gpu_handle):
    """n = m = k = 1: the factorisation is W = sign * |W|: q = w / |w| exactly,
    R = |w| (the sketch of one entry is +-w)."""
    rgs = _rgs()
    for sketch in ("gaussian", "srht", "rademacher"):
        W = np.array([[-3.25]])
        rep, Q, R, S = run_qr(gpu_handle, W, 1, sketch, "fp64")
        assert rep.status == 0
        assert R[0, 0] > 0 and abs(abs(S[0, 0]) - 1.0) <= 1e-15
        assert abs(Q[0, 0] * R[0, 0] - W[0, 0]) <= 1e-15 * abs(W[0, 0])


@pytest.mark.parametrize("sketch", ["srht", "gaussian", "rademacher"])
def test_bitwise_deterministic(gpu_handle, sketch):
    W = synth.svd_matrix(20000, 32, 1e-4, tag=18)
    a = run_qr(gpu_handle, W, 128, sketch, "fp32")
    b = run_qr(gpu_handle, W, 128, sketch, "fp32")
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(x, y)
