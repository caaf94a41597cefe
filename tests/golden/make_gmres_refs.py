"""Writes the cached oracle references of the randomized GMRES tests.

Runs only ``oracle/`` (Algorithm 3 and the restarted randomized GMRES of
Sec. 4.2) on inputs drawn by ``synth``; nothing here touches the device
library.  The runs are too long to repeat inside a test (the 192^3 system
takes the oracle about an hour on one core), so the results are stored as
JSON beside this script and the GPU tests compare against them.

    python tests/golden/make_gmres_refs.py c3_srht        # 192^3, P-SRHT k = 400, fp64
    python tests/golden/make_gmres_refs.py c3_gauss64     # 64^3, Gaussian k = 400, fp64
    python tests/golden/make_gmres_refs.py c5_subset [-j 6]  # 32 of the 256 batched systems, fp64 + bf16 models
    python tests/golden/make_gmres_refs.py c5_twin [-j 6]    # adds the bf16 model with step 3 summed in
                                                             # reverse column order ("bf16q_rev")

Workloads (the synthetic stand-ins of the convection-diffusion systems):
  * single system: -Lap u + Pe (1,1,1).grad u on the unit cube, Pe = 50,
    N^3 grid (h = 1/(N+1)), b ~ N(0, 1) (synth.rhs tag 0), x0 = 0,
    restart 100, k = 400, tol 1e-6, fresh sketch per cycle (sketch_id 2 + c);
  * batched systems: the draws of synth.batch_gmres_sizes(256) (N in 32..96,
    Pe in [1, 100]), b tag 1000 + index, restart 50, k = 200, P-SRHT,
    tol 1e-6; the 32 systems at ranks round(linspace(0, 255, 32)) of the
    order by n.
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import gmres as ogm, sketch as osk, stencil as ost  # noqa: E402

BATCH, B_RESTART, B_K, TOL = 256, 50, 200, 1e-6


def _solve(N, Pe, b, kind, k, restart, precision, reverse=False):
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    t0 = time.time()

    def theta(c):
        if kind == "gaussian":   # entries drawn once per cycle and kept dense (k n fp64 values)
            return osk.Gaussian(n, k, seed=synth.SKETCH_SEED, sketch_id=2 + c, cache_limit=k * n)
        return osk.make(kind, n, k, seed=synth.SKETCH_SEED, sketch_id=2 + c)

    ref = ogm.rgmres(lambda u, dt: ost.apply(u, dims, coeffs, dt), b, theta,
                     restart=restart, tol=TOL, precision=precision, max_iters=20000,
                     reverse_projection=reverse)
    return {"N": int(N), "Pe": float(Pe), "n": int(n), "sketch": kind, "k": int(k), "restart": int(restart),
            "tol": TOL, "precision": precision, "iters": int(ref["iters"]), "cycles": int(ref["cycles"]),
            "true_relres": float(ref["true_relres"]), "converged": bool(ref["converged"]),
            "oracle_seconds": round(time.time() - t0, 1)}


def c3_srht():
    N = 192
    return _solve(N, 50.0, synth.rhs(N ** 3, tag=0), "srht", 400, 100, "fp64")


def c3_gauss64():
    N = 64
    return _solve(N, 50.0, synth.rhs(N ** 3, tag=0), "gaussian", 400, 100, "fp64")


def c5_indices():
    Ns, _ = synth.batch_gmres_sizes(BATCH)
    order = np.argsort(np.asarray(Ns) ** 3, kind="stable")
    ranks = np.unique(np.round(np.linspace(0, BATCH - 1, 32)).astype(int))
    return [int(order[r]) for r in ranks]


def _c5_one(args):
    i, precision = args
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    Ns, Pes = synth.batch_gmres_sizes(BATCH)
    N, Pe = int(Ns[i]), float(Pes[i])
    rev = precision.endswith("_rev")
    out = _solve(N, Pe, synth.rhs(N ** 3, tag=1000 + i), "srht", B_K, B_RESTART, precision.replace("_rev", ""),
                 reverse=rev)
    out["precision"] = precision
    out["index"] = i
    print("system %d N=%d Pe=%.1f %s: %d iters (%.0f s)" % (i, N, Pe, precision, out["iters"],
                                                           out["oracle_seconds"]), flush=True)
    return out


def c5_subset(jobs, precisions=("fp64", "bf16q")):
    import multiprocessing as mp
    work = [(i, p) for i in c5_indices() for p in precisions]
    work.sort(key=lambda a: -synth.batch_gmres_sizes(BATCH)[0][a[0]])   # largest first
    with mp.get_context("fork").Pool(jobs) as pool:
        res = pool.map(_c5_one, work, chunksize=1)
    by = {}
    for r in res:
        by.setdefault(r["index"], {})[r["precision"]] = r
    return {"batch": BATCH, "restart": B_RESTART, "k": B_K, "sketch": "srht", "tol": TOL,
            "systems": [by[i] for i in sorted(by)]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["c3_srht", "c3_gauss64", "c5_subset", "c5_twin"])
    ap.add_argument("-j", type=int, default=6)
    a = ap.parse_args()
    if a.what == "c5_twin":   # merged into the c5_subset file
        path = os.path.join(HERE, "gmres_c5_subset.json")
        out = json.load(open(path))
        twin = c5_subset(a.j, ("bf16q_rev",))
        by = {s["bf16q_rev"]["index"]: s["bf16q_rev"] for s in twin["systems"]}
        for s in out["systems"]:
            s["bf16q_rev"] = by[s["fp64"]["index"]]
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        print("wrote", path)
        return
    if a.what == "c5_subset":
        out = c5_subset(a.j)
    else:
        out = {"c3_srht": c3_srht, "c3_gauss64": c3_gauss64}[a.what]()
    path = os.path.join(HERE, "gmres_%s.json" % a.what)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
