"""GPU parity of the Gaussian sketch with bf16 entries (RGS_FLAG_THETA_BF16).

The device fills a table with the entries bf16(z), z the fp64 Box-Muller
value of the Gaussian sketch rounded once to nearest even, and every later
sketch reads it.  The oracle's GaussianBF16 is the same definition, so:

* the materialized entries are equal bit for bit (both sides round an fp64
  z whose two computations differ by a few fp64 ulps: a bf16 rounding
  boundary between them has probability ~2^-40 per entry);
* Theta X, the fp64 factorisation (<= 1e-12, split and fused paths), the
  fp32 factorisation (against the oracle's fp32 model), RGMRES (iterations
  +-2, histories) and the certificate (Phi = the Gaussian sketch) agree with
  the oracle run with GaussianBF16.
"""

import numpy as np
import pytest

import synth
from oracle import gmres as ogm, metrics, rgs as orgs, sketch as osk, stencil as ost

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


def to_dev(A, dtype):
    A = np.asarray(A)
    if A.ndim == 1:
        return torch.from_numpy(np.ascontiguousarray(A)).to(dtype=dtype, device="cuda")
    return torch.from_numpy(np.ascontiguousarray(A.T)).to(dtype=dtype, device="cuda").t()


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def run_qr(h, W, k, prec, flags=0):
    rgs = _rgs()
    n, m = W.shape
    dt = torch.float64 if prec == "fp64" else torch.float32
    Q, R, S = rgs.colmajor(n, m, dt), rgs.colmajor(m, m, torch.float64), rgs.colmajor(k, m, torch.float64)
    d = rgs.qr_desc(n, m, k, sketch="gaussian", prec=prec, flags=rgs.FLAG_THETA_BF16 | flags)
    rep = rgs.rgs_qr(h, d, to_dev(W, dt), Q, R, S)
    torch.cuda.synchronize()
    return rep, to_host(Q), to_host(R), to_host(S)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_table_entries_equal_oracle(gpu_handle, prec):
    rgs = _rgs()
    n, k = 1003, 40
    d = rgs.qr_desc(n, 1, k, sketch="gaussian", prec=prec, seed=77, sketch_id=2, instance=1,
                    flags=rgs.FLAG_THETA_BF16)
    out = rgs.colmajor(k, n, torch.float64)
    rgs.rgs_sketch_materialize(gpu_handle, d, 0, k, 0, n, out)
    got = to_host(out)
    ref = osk.gaussian_bf16_block(k, 77, 2, 1, 0, k, 0, n)
    # the device scales by the fp64 reciprocal of sqrt(k), the oracle divides: compare the bf16 values
    zg, zr = osk.bf16_round_f64(got * np.sqrt(k)), osk.bf16_round_f64(ref * np.sqrt(k))
    assert np.array_equal(zg, zr)
    assert np.array_equal(zr, osk.gaussian_bf16_block(1, 77, 2, 1, 0, k, 0, n))
    assert np.abs(got - ref).max() <= 2.0 ** -52 * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_table_sketch_apply(gpu_handle, prec):
    rgs = _rgs()
    n, k = 9000 + 5, 96
    X = np.random.Generator(np.random.PCG64(3)).standard_normal((n, 37))
    dt = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        X = X.astype(np.float32).astype(np.float64)
    d = rgs.qr_desc(n, 1, k, sketch="gaussian", prec=prec, seed=9, flags=rgs.FLAG_THETA_BF16)
    Y = rgs.colmajor(k, 37, torch.float64)
    rgs.rgs_sketch_apply(gpu_handle, d, to_dev(X, dt), Y)
    ref = osk.make("gaussian_bf16", n, k, seed=9).apply(X)
    tol = 1e-13 if prec == "fp64" else 2e-6
    assert np.abs(to_host(Y) - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("n,m,k", [(16384 + 77, 40, 256), ((1 << 20) + 333, 6, 64)])
def test_table_fp64_qr_matches_oracle(gpu_handle, n, m, k):
    """Split small-n path, and the fused projection path above 2^20 rows."""
    W = synth.svd_matrix(n, m, 1e-2, tag=71)
    rep, Q, R, S = run_qr(gpu_handle, W, k, "fp64")
    assert rep.status == 0
    th = osk.make("gaussian_bf16", n, k, seed=42)
    ref = orgs.rgs_qr(W, th)
    assert np.linalg.norm(R - ref["R"]) / np.linalg.norm(ref["R"]) <= 1e-12
    assert np.abs(Q - ref["Q"]).max() <= 1e-12 * np.abs(ref["Q"]).max()
    assert np.linalg.norm(S - ref["S"]) / np.linalg.norm(ref["S"]) <= 1e-12
    assert metrics.backward_error(W, Q, R) <= 1e-12


def test_table_fp32_qr_matches_oracle_fp32_model(gpu_handle):
    n, m, k = 4096 * 5 + 100, 48, 192
    W = synth.svd_matrix(n, m, 1e-3, tag=72).astype(np.float32).astype(np.float64)
    rep, Q, R, S = run_qr(gpu_handle, W, k, "fp32")
    assert rep.status == 0
    ref = orgs.rgs_qr(W, osk.make("gaussian_bf16", n, k, seed=42), precision="fp32")
    assert metrics.backward_error(W, Q, R) <= 1e-5
    assert metrics.delta_2(S) <= 1e-4
    assert np.linalg.norm(R - ref["R"]) / np.linalg.norm(ref["R"]) <= 1e-3


def test_table_certificate(gpu_handle):
    rgs = _rgs()
    n, m, k = 3 * 8192 + 123, 30, 192
    W = synth.svd_matrix(n, m, 1e-2, tag=73)
    rep, Q, R, S = run_qr(gpu_handle, W, k, "fp64", flags=rgs.FLAG_CERTIFY)
    assert rep.status == 0
    th = osk.make("gaussian_bf16", n, k, seed=42, sketch_id=0)
    ph = osk.make("gaussian", n, k, seed=42, sketch_id=1)
    for V, got in ((Q, (rep.cert_smin_q, rep.cert_smax_q)), (W, (rep.cert_smin_w, rep.cert_smax_w))):
        phV = ph.apply(V)
        ref = metrics.cert_extremes(th.apply(V), phV)
        tol = 64 * 2.0 ** -53 * 64 * metrics.cond(phV)
        assert abs(got[0] - ref[0]) <= tol * ref[1] and abs(got[1] - ref[1]) <= tol * ref[1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_table_rgmres_matches_oracle(gpu_handle, prec):
    rgs = _rgs()
    N, Pe, restart, k, tol = 24, 50.0, 20, 96, 1e-6
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=74)
    ref = ogm.rgmres(lambda u, dt: ost.apply(u, dims, coeffs, dt), b,
                     lambda c: osk.make("gaussian_bf16", n, k, seed=42, sketch_id=2 + c),
                     restart=restart, tol=tol, precision="fp64", max_iters=3000)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    rep, hist = rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs),
                              rgs.gmres_desc(restart, k, tol, max_iters=3000, sketch="gaussian", prec=prec,
                                             flags=rgs.FLAG_THETA_BF16),
                              to_dev(b, torch.float64), x, res_hist=10000)
    torch.cuda.synchronize()
    assert rep.status == 0 and ref["converged"]
    assert abs(rep.iters - ref["iters"]) <= 2
    r = b - ost.apply(x.cpu().numpy(), dims, coeffs, np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= tol
    L = min(len(hist), len(ref["hist"]), restart)
    np.testing.assert_allclose(hist[:L], ref["hist"][:L], rtol=1e-8 if prec == "fp64" else 1e-4)


def test_table_flag_rejected_for_other_sketches(gpu_handle):
    rgs = _rgs()
    n, m, k = 1000, 4, 32
    W = synth.svd_matrix(n, m, 1e-1, tag=75)
    for sk in ("srht", "rademacher"):
        d = rgs.qr_desc(n, m, k, sketch=sk, prec="fp64", flags=rgs.FLAG_THETA_BF16)
        with pytest.raises(rgs.RgsError) as e:
            rgs.rgs_qr(gpu_handle, d, to_dev(W, torch.float64), rgs.colmajor(n, m, torch.float64),
                       rgs.colmajor(m, m, torch.float64), rgs.colmajor(k, m, torch.float64))
        assert e.value.status == rgs.RGS_EINVAL
