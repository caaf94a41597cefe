"""Writes the cached oracle reference of the reduced-size headline QR test.

Runs only ``oracle/`` (Algorithm 2 in the multi-precision model of Sec. 2.3:
fp32 storage and step 3, fp64 sketches, least squares and normalisation) on
an input drawn by ``synth``; nothing here touches the device library.

    python tests/golden/make_qr_refs.py

Workload: W = U diag(sigma) V^T with n = 2^18, m = 512, sigma log-spaced
1 -> 1e-8 (synth.svd_matrix tag 40, rounded to float32), P-SRHT with
k = 2048, seed 42, sketch_id 0.  At this conditioning W is numerically
singular in float32 (sigma_min < u32), so Delta, cond(S) and cond(Q) are set
by rounding noise; the test compares the device's values with these within a
factor of 3.  The same quantities at sigma -> 1e-3 (tag 41) are stored as the
well-conditioned companion.
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import metrics, rgs as orgs, sketch as osk  # noqa: E402

N, M, K = 1 << 18, 512, 2048


def one(sigma_min, tag):
    W = synth.svd_matrix(N, M, sigma_min, tag=tag).astype(np.float32)
    th = osk.SRHT(N, K, seed=synth.SKETCH_SEED)
    t0 = time.time()
    out = orgs.rgs_qr(W, th, precision="fp32")
    dt = time.time() - t0
    Q, R, S = out["Q"], out["R"], out["S"]
    return {"n": N, "m": M, "k": K, "sketch": "srht", "sigma_min": sigma_min, "tag": tag, "precision": "fp32",
            "delta_2": float(metrics.delta_2(S)), "delta_F": float(metrics.delta_F(S)),
            "cond_S": float(metrics.cond(S)), "cond_Q": float(metrics.cond(Q)),
            "orth_loss_2": float(metrics.orth_loss_2(Q)),
            "backward_error": float(metrics.backward_error(W.astype(np.float64), Q, R)),
            "oracle_seconds": round(dt, 1)}


def main():
    out = {"headline_sigma_1e-8": one(1e-8, 40), "companion_sigma_1e-3": one(1e-3, 41)}
    path = os.path.join(HERE, "qr_fp32_srht_n262144_m512_k2048.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
