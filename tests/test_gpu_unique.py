"""GPU parity of the unique-precision model RGS_P_FP32 ('fp32u': Algorithm 2
with u_crs = u_fine = float32, the comparison of Sec. 5.1) against the
oracle's 'fp32u' model on the same W and Theta.

* The float32 sketch (rgs_sketch_apply in fp32u): on small-integer input the
  P-SRHT's float32 sums are exact, so the device equals the oracle bit for bit
  (the integer transform times float32(k**-1/2)); on Gaussian input every
  sketch stays within the float32 inner-product error bound of the fp64 one,
  and carries float32 rounding.
* The factorisation: R and S hold float32 values; R against the oracle's model
  within a bar set by the model's own rounding (four times its distance from
  the fp64 factorisation, the spread two valid float32 evaluations of the same
  steps can have); S R = Theta W and Q = W R^-1 to float32 rounding; and the
  rounding of the sketch-space steps is at the float32 level (the device sits
  farther from the fp64 result than the multi-precision 'fp32' does).
* Rejected: Richardson sweeps and the batched calls (GMRES takes the precision
  in the configuration of Sec. 5.3, test_gpu_gmres_unique.py).
"""

import math

import numpy as np
import pytest

import synth
from oracle import metrics, rgs as orgs, sketch as osk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


def to_dev(A, dtype):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A).T)).to(dtype=dtype, device="cuda").t()


def host(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.parametrize("n,k", [(1000, 64), (70000, 256), ((1 << 20) + 333, 512)])
def test_srht_float32_sketch_is_exact_on_integers(gpu_handle, n, k):
    rgs = _rgs()
    print("fp32u srht sketch n=%d k=%d" % (n, k), flush=True)
    g = np.random.default_rng(n)
    X = g.integers(-8, 9, size=(n, 3)).astype(np.float32)
    th = osk.SRHT(n, k, seed=42)
    want = th.apply(X, np.float32)
    Y = rgs.colmajor(k, 3, torch.float64)
    rgs.rgs_sketch_apply(gpu_handle, rgs.qr_desc(n, 3, k, sketch="srht", prec="fp32u"), to_dev(X, torch.float32), Y)
    torch.cuda.synchronize()
    assert np.array_equal(host(Y), want.astype(np.float64))


@pytest.mark.parametrize("sketch", ["srht", "gaussian", "rademacher"])
def test_float32_sketch_within_the_error_bound(gpu_handle, sketch):
    rgs = _rgs()
    n, k = 30000, 128
    X = np.random.default_rng(5).standard_normal((n, 2)).astype(np.float32)
    th = osk.make(sketch, n, k, seed=42)
    Y = rgs.colmajor(k, 2, torch.float64)
    rgs.rgs_sketch_apply(gpu_handle, rgs.qr_desc(n, 2, k, sketch=sketch, prec="fp32u"), to_dev(X, torch.float32), Y)
    torch.cuda.synchronize()
    y = host(Y)
    assert np.array_equal(y.astype(np.float32).astype(np.float64), y)      # float32 values
    y64 = th.apply(X.astype(np.float64))
    # Gaussian: the device's fp32 draws differ from the oracle's fp64 entries by at most 16 ulp
    ent = (16 if sketch == "gaussian" else 1) * U32
    bound = ((n + 2) * U32 + ent) * (np.abs(th.materialize()) @ np.abs(X.astype(np.float64)))
    assert np.all(np.abs(y - y64) <= bound)
    assert np.any(y != y64)


def _qr(h, W, k, sketch, prec):
    rgs = _rgs()
    n, m = W.shape
    Wd = to_dev(W, torch.float32)
    Q = rgs.colmajor(n, m, torch.float32)
    R = rgs.colmajor(m, m, torch.float64)
    S = rgs.colmajor(k, m, torch.float64)
    rep = rgs.rgs_qr(h, rgs.qr_desc(n, m, k, sketch=sketch, prec=prec), Wd, Q, R, S)
    torch.cuda.synchronize()
    assert rep.status == 0
    return host(Q), host(R), host(S)


@pytest.mark.parametrize("sketch,n,m,k", [("srht", 20000, 24, 96), ("srht", (1 << 20) + 333, 16, 128),
                                          ("gaussian", 9000, 12, 48), ("rademacher", 12000, 16, 64)])
def test_unique_precision_qr_matches_the_oracle_model(gpu_handle, sketch, n, m, k):
    print("fp32u qr %s n=%d m=%d k=%d" % (sketch, n, m, k), flush=True)
    W = synth.svd_matrix(n, m, 1e-2, tag=31).astype(np.float32)
    th = osk.make(sketch, n, k, seed=42)
    Q, R, S = _qr(gpu_handle, W, k, sketch, "fp32u")
    assert np.array_equal(R.astype(np.float32).astype(np.float64), R)
    assert np.array_equal(S.astype(np.float32).astype(np.float64), S)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    orc = orgs.rgs_qr(W, th, precision="fp32u")
    ref = orgs.rgs_qr(W.astype(np.float64), th, precision="fp64")
    scale = np.linalg.norm(ref["R"])
    model_err = np.linalg.norm(orc["R"] - ref["R"]) / scale
    dev_err = np.linalg.norm(R - orc["R"]) / scale
    print("  ||R - R_oracle||/||R|| %.2e, oracle model vs fp64 %.2e" % (dev_err, model_err), flush=True)
    assert dev_err <= 4 * model_err
    # column by column on the well-determined entries
    for c in range(m):
        tol = 8 * math.sqrt(c + 1) * model_err * scale
        assert np.max(np.abs(R[: c + 1, c] - orc["R"][: c + 1, c])) <= max(tol, 64 * U32 * abs(orc["R"][c, c]))
    # S R = Theta W and Q = W R^-1 to float32 rounding
    P = th.apply(W.astype(np.float64))
    kappa = metrics.cond(W.astype(np.float64))
    assert np.linalg.norm(S @ R - P) / np.linalg.norm(P) <= 50 * U32 * math.sqrt(k) * kappa
    assert metrics.backward_error(W, Q.astype(np.float32), R) <= 50 * U32 * math.sqrt(m)


def test_unique_precision_rounds_the_sketch_space_in_float32(gpu_handle):
    """The device's fp32u factorisation is farther from the fp64 one than its
    multi-precision fp32 factorisation of the same W (whose sketches and least
    squares are fp64), by the float32 rounding of the sketch-space steps."""
    n, m, k = 40000, 32, 128
    W = synth.svd_matrix(n, m, 1e-1, tag=32).astype(np.float32)
    th = osk.SRHT(n, k, seed=42)
    _, Ru, _ = _qr(gpu_handle, W, k, "srht", "fp32u")
    _, Rm, _ = _qr(gpu_handle, W, k, "srht", "fp32")
    d = orgs.rgs_qr(W.astype(np.float64), th, precision="fp64")["R"]
    scale = np.linalg.norm(d)
    du, dm = np.linalg.norm(Ru - d) / scale, np.linalg.norm(Rm - d) / scale
    print("  fp32u %.2e, fp32 (multi-precision) %.2e from fp64" % (du, dm), flush=True)
    assert du > dm and 1e-9 < du < 1e-4


def test_unique_precision_rejections(gpu_handle):
    rgs = _rgs()
    n, m, k = 5000, 8, 32
    W = to_dev(synth.svd_matrix(n, m, 1e-1, tag=33).astype(np.float32), torch.float32)
    Q = rgs.colmajor(n, m, torch.float32)
    R = rgs.colmajor(m, m, torch.float64)
    S = rgs.colmajor(k, m, torch.float64)
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_qr(gpu_handle, rgs.qr_desc(n, m, k, sketch="srht", prec="fp32u", ls_sweeps=1), W, Q, R, S)
    assert e.value.status == rgs.RGS_EINVAL
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_qr_batched(gpu_handle, [(W, Q, R, S, k)], sketch="srht", prec="fp32u")
    assert e.value.status == rgs.RGS_EINVAL
    # (rgs_gmres takes the precision in the configuration of Sec. 5.3: test_gpu_gmres_unique.py)


def test_unique_precision_breakdown_and_nonfinite(gpu_handle):
    """The float32 chain keeps the breakdown tests: an exactly zero column is a
    breakdown at that column (r_ii = 0), a NaN a non-finite sketch; the
    columns before it match the oracle's fp32u model."""
    rgs = _rgs()
    n, m, k = 12000, 10, 64
    W = synth.svd_matrix(n, m, 1e-1, tag=34).astype(np.float32)
    W[:, 6] = 0.0
    Wd = to_dev(W, torch.float32)
    Q = rgs.colmajor(n, m, torch.float32)
    R = rgs.colmajor(m, m, torch.float64)
    S = rgs.colmajor(k, m, torch.float64)
    rep = rgs.rgs_qr(gpu_handle, rgs.qr_desc(n, m, k, sketch="srht", prec="fp32u"), Wd, Q, R, S)
    torch.cuda.synchronize()
    assert rep.status == rgs.RGS_EBREAKDOWN and rep.failed_column == 6
    orc = orgs.rgs_qr(W[:, :6], osk.SRHT(n, k, seed=42), precision="fp32u")
    Rh = host(R)[:6, :6]
    assert np.linalg.norm(Rh - orc["R"]) <= 1e-5 * np.linalg.norm(orc["R"])
    W[:, 6] = W[:, 1]
    W[99, 4] = np.nan
    rep = rgs.rgs_qr(gpu_handle, rgs.qr_desc(n, m, k, sketch="srht", prec="fp32u"), to_dev(W, torch.float32), Q, R,
                     S)
    torch.cuda.synchronize()
    assert rep.status == rgs.RGS_ENONFINITE and rep.failed_column == 4
