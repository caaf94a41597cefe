"""The a-posteriori certificate (Prop. 3.7) in randomized GMRES
(rgs_gmres with RGS_FLAG_CERTIFY): the last restart cycle's Theta certified
on the basis vectors its update of x used (Sec. 5.3 reports omega for this
basis), against the oracle's certificate of the oracle's own basis of that
cycle (same system, same sketches: cycle c draws Theta with sketch_id 2 + c,
Phi has sketch_id 1).  With the same iteration and cycle counts the two bases
agree to the precision model's rounding, so the extreme singular values of
(Theta V) X do too; Prop. 3.7's omega <= omega_bar is checked on the oracle's
basis, and cond(Phi V) against the oracle's.
"""

import math

import numpy as np
import pytest

import synth
from oracle import gmres as ogm, metrics, sketch as osk, stencil as ost

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


@pytest.mark.parametrize("sketch,prec,rtol", [("srht", "fp64", 1e-8), ("gaussian", "fp64", 1e-8),
                                              ("rademacher", "fp64", 1e-8), ("srht", "fp32", 1e-3)])
def test_gmres_certificate_matches_the_oracle(gpu_handle, sketch, prec, rtol):
    rgs = _rgs()
    N, Pe, restart, k, tol = 20, 50.0, 150, 300, 1e-6   # one cycle of 59 steps: a 59-column basis
    print("gmres certificate %s %s" % (sketch, prec), flush=True)
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = synth.rhs(n, tag=6)
    make = lambda c: osk.make(sketch, n, k, seed=42, sketch_id=2 + c)
    ref = ogm.rgmres(lambda u, dt: ost.apply(u, dims, coeffs, dt), b, make, restart=restart, tol=tol,
                     precision=prec)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    rep, _ = rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs),
                           rgs.gmres_desc(restart, k, tol, sketch=sketch, prec=prec, flags=rgs.FLAG_CERTIFY),
                           torch.from_numpy(b).cuda(), x)
    torch.cuda.synchronize()
    assert rep.status == 0 and ref["converged"]
    assert (rep.iters, rep.cycles) == (ref["iters"], ref["cycles"])
    V = ref["Q_last"]
    TV = make(ref["theta_cycle_last"]).apply(V)
    PV = osk.make(sketch, n, k, seed=42, sketch_id=1).apply(V)
    smin, smax = metrics.cert_extremes(TV, PV)
    print("  device smin %.6f smax %.6f, oracle %.6f %.6f, cond(Phi V) %.3f" %
          (rep.cert_smin_q, rep.cert_smax_q, smin, smax, rep.cert_cond_phi_q), flush=True)
    assert math.isclose(rep.cert_smin_q, smin, rel_tol=rtol)
    assert math.isclose(rep.cert_smax_q, smax, rel_tol=rtol)
    assert math.isclose(rep.cert_cond_phi_q, metrics.cond(PV), rel_tol=max(rtol, 1e-6))
    assert math.isnan(rep.cert_smin_w) and math.isnan(rep.cert_smax_w)
    assert V.shape[1] >= 40
    # Prop. 3.7 on the oracle's basis: omega <= omega_bar (eps* = 0.05)
    obar = rgs.rgs_omega_bar(rep.cert_smin_q, rep.cert_smax_q, 0.05)
    assert metrics.omega(TV, V) <= obar


def test_gmres_certificate_off_by_default_and_rejected_for_identity(gpu_handle):
    rgs = _rgs()
    N = 12
    dims, coeffs = synth.convdiff_coeffs(N, 10.0)
    b = torch.from_numpy(synth.rhs(N ** 3, tag=7)).cuda()
    x = torch.empty_like(b)
    rep, _ = rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs), rgs.gmres_desc(10, 40, 1e-6, sketch="srht"), b, x)
    assert math.isnan(rep.cert_smin_q) and math.isnan(rep.cert_smax_q)
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_gmres(gpu_handle, rgs.stencil7(dims, coeffs),
                      rgs.gmres_desc(10, N ** 3, 1e-6, sketch="identity", flags=rgs.FLAG_CERTIFY), b, x)
    assert e.value.status == rgs.RGS_EINVAL
