"""GPU parity of randomized GMRES in the configuration of Sec. 5.3
(rgs_gmres with RGS_P_FP32): unique-precision RGS -- every step of the
Arnoldi vector's orthogonalisation in float32 -- with the products with A in
fp64 from the float32 basis vector, and the Givens rotations, x and the
restart residual in fp64.

* the mat-vec hook in this precision is the fp64 product of the float32
  vector, rounded once (against the oracle's fp64 stencil);
* RGMRES against the oracle's 'fp32u' model (P-SRHT, drawn Gaussian,
  Rademacher): iteration counts within +-2 of it and of the fp64 oracle,
  residual histories to float32 rounding, the true residual recomputed on the
  host;
* the 192^3 system with the P-SRHT against the cached fp64 oracle count;
* the precision is refused with Richardson least squares, by the single and
  the batched solver (the batched solver takes it otherwise: its bitwise
  tests sit with the other batched GMRES tests).
"""

import json
import os

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


def test_fp64_product_of_float32_vectors(gpu_handle):
    rgs = _rgs()
    dims = (23, 19, 29)
    _, coeffs = synth.convdiff_coeffs(23, 37.0)
    n = 23 * 19 * 29
    u = np.random.Generator(np.random.PCG64(4)).standard_normal(n).astype(np.float32)
    w = torch.empty(n, dtype=torch.float32, device="cuda")
    rgs.rgs_stencil_apply(gpu_handle, rgs.stencil7(dims, coeffs), "fp32u", dev(u, torch.float32), w)
    torch.cuda.synchronize()
    ref = ost.apply(u.astype(np.float64), dims, coeffs, np.float64)
    got = w.cpu().numpy().astype(np.float64)
    # one rounding of the fp64 result (its own rounding order aside): within one float32 ulp
    assert np.all(np.abs(got - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-30)
    # and not the float32 product (which is further off on some rows)
    w32 = torch.empty(n, dtype=torch.float32, device="cuda")
    rgs.rgs_stencil_apply(gpu_handle, rgs.stencil7(dims, coeffs), "fp32", dev(u, torch.float32), w32)
    torch.cuda.synchronize()
    assert np.abs(w32.cpu().numpy().astype(np.float64) - ref).max() > np.abs(got - ref).max()


@pytest.mark.parametrize("sketch", ["srht", "gaussian", "rademacher"])
def test_unique_precision_rgmres_matches_oracle(gpu_handle, sketch):
    rgs = _rgs()
    N, Pe, restart, k, tol = 24, 50.0, 20, 96, 1e-6
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=95)
    applyA = lambda u, dt: ost.apply(u, dims, coeffs, dt)
    mk = lambda c: osk.make(sketch, n, k, seed=42, sketch_id=2 + c)
    up = ogm.rgmres(applyA, b, mk, restart=restart, tol=tol, precision="fp32u", max_iters=3000)
    ref = ogm.rgmres(applyA, b, mk, restart=restart, tol=tol, precision="fp64", max_iters=3000)
    print("rgmres fp32u %s: oracle fp32u %d, fp64 %d" % (sketch, up["iters"], ref["iters"]), flush=True)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    rep, hist = rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs),
                              rgs.gmres_desc(restart, k, tol, max_iters=3000, sketch=sketch, prec="fp32u"),
                              dev(b), x, res_hist=10000)
    torch.cuda.synchronize()
    print("  gpu %d iterations, %d cycles" % (rep.iters, rep.cycles), flush=True)
    assert rep.status == 0 and up["converged"]
    r = b - ost.apply(x.cpu().numpy(), dims, coeffs, np.float64)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= tol * (1 + 1e-6)
    assert abs(rep.iters - up["iters"]) <= 2 and abs(rep.iters - ref["iters"]) <= 2
    L = min(len(hist), len(up["hist"]), restart)
    np.testing.assert_allclose(hist[:L], up["hist"][:L], rtol=2e-3)


def test_unique_precision_rgmres_full_size(gpu_handle):
    """192^3, P-SRHT k = 400, restart 100: the fp64 oracle's cached count +-2."""
    rgs = _rgs()
    ref = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gmres_c3_srht.json")))
    N = ref["N"]
    dims, coeffs = synth.convdiff_coeffs(N, ref["Pe"])
    n = N ** 3
    b = synth.rhs(n, tag=0)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    print("rgmres 192^3 srht fp32u", flush=True)
    rep, _ = rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs),
                           rgs.gmres_desc(ref["restart"], ref["k"], ref["tol"], max_iters=5000, sketch="srht",
                                          prec="fp32u"),
                           dev(b), x, res_hist=0)
    torch.cuda.synchronize()
    r = b - ost.apply(x.cpu().numpy(), dims, coeffs, np.float64)
    print("  %d iterations (fp64 oracle %d)" % (rep.iters, ref["iters"]), flush=True)
    assert rep.status == 0 and np.linalg.norm(r) / np.linalg.norm(b) <= 1e-6 * (1 + 1e-6)
    assert abs(rep.iters - ref["iters"]) <= 2


def test_unique_precision_refusals(gpu_handle):
    rgs = _rgs()
    dims, coeffs = synth.convdiff_coeffs(8, 10.0)
    b = dev(synth.rhs(8 ** 3, tag=96))
    x = torch.empty(8 ** 3, dtype=torch.float64, device="cuda")
    A = rgs.stencil7(dims, coeffs)
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_gmres(gpu_handle, A, rgs.gmres_desc(10, 40, 1e-6, sketch="srht", prec="fp32u", ls_sweeps=1), b, x)
    assert e.value.status == rgs.RGS_EINVAL
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_gmres_batched(gpu_handle, [(A, b, x)],
                              rgs.gmres_desc(10, 40, 1e-6, sketch="srht", prec="fp32u", ls_sweeps=1))
    assert e.value.status == rgs.RGS_EINVAL
