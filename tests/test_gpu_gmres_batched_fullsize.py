"""GPU parity of the batched randomized GMRES at its full benchmark size: 256
convection-diffusion systems on grids N^3, N ~ U{32..96} (85.9e6 unknowns in
all), Pe ~ U[1, 100], b ~ N(0, 1), restart 50, k = 200, tol 1e-6, P-SRHT, one
graph-replayed rgs_gmres_batched call -- the workload and launch configuration
bench.py times -- with the bf16 and with the fp32 basis.

* every system converges (status 0), and its true relative residual
  ||b - A x|| / ||b||, recomputed on the host with the oracle's operator in
  fp64, is <= tol and equals the reported one to 1e-6 relative;
* the two smallest systems against the oracle's RGMRES with the same sketches
  (fp64 model for the fp32 basis, the bf16 model for the bf16 basis):
  iteration counts within +-2.
"""

import numpy as np
import pytest

import synth
from oracle import gmres as ogm, sketch as osk, stencil as ost

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BATCH, RESTART, K, TOL = 256, 50, 200, 1e-6


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


@pytest.fixture(scope="module")
def systems():
    Ns, Pes = synth.batch_gmres_sizes(BATCH)
    out = []
    for i, (N, Pe) in enumerate(zip(Ns, Pes)):
        dims, coeffs = synth.convdiff_coeffs(int(N), float(Pe))
        out.append((dims, coeffs, synth.rhs(int(N) ** 3, tag=1000 + i)))
    return out


@pytest.mark.parametrize("prec,model", [("bf16q", "bf16q"), ("fp32", "fp64")])
def test_full_batch(gpu_handle, systems, prec, model):
    rgs = _rgs()
    print("batched RGMRES, srht, %s basis, %d systems" % (prec, len(systems)), flush=True)
    sy = []
    for dims, coeffs, b in systems:
        bd = torch.from_numpy(b).to("cuda")
        sy.append((rgs.stencil7(dims, coeffs), bd, torch.full_like(bd, np.nan)))
    desc = rgs.gmres_desc(RESTART, K, TOL, max_iters=20000, sketch="srht", prec=prec, flags=rgs.FLAG_GRAPH)
    st, stat, reps, _ = rgs.rgs_gmres_batched(gpu_handle, sy, desc)
    torch.cuda.synchronize()
    assert st == 0 and all(v == 0 for v in stat)
    worst = 0.0
    for (dims, coeffs, b), (_, _, x), rep in zip(systems, sy, reps):
        r = b - ost.apply(x.cpu().numpy(), dims, coeffs, np.float64)
        relres = np.linalg.norm(r) / np.linalg.norm(b)
        assert relres <= TOL and abs(relres - rep.true_relres) <= 1e-6 * relres, (dims, relres, rep.true_relres)
        worst = max(worst, relres)
    print("  max true relative residual %.3e" % worst, flush=True)
    del sy
    torch.cuda.empty_cache()

    for i in np.argsort([b.size for _, _, b in systems], kind="stable")[:2]:
        dims, coeffs, b = systems[int(i)]
        n = b.size
        print("  oracle check: system %d, grid %s" % (int(i), dims), flush=True)
        ref = ogm.rgmres(lambda u, dt: ost.apply(u, dims, coeffs, dt), b,
                         lambda c: osk.make("srht", n, K, seed=42, sketch_id=2 + c),
                         restart=RESTART, tol=TOL, precision=model, max_iters=20000)
        assert ref["converged"]
        assert abs(reps[int(i)].iters - ref["iters"]) <= 2, (dims, reps[int(i)].iters, ref["iters"])
