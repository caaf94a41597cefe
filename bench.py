#!/usr/bin/env python3
"""Benchmark of the randomized Gram-Schmidt hot path on one MI355X.

One step = one complete RGS QR factorisation (Algorithm 2 of Balabanov &
Grigori, every column: sketch, fp64 sketched least squares, fused fp32
projection + sketch, normalisation) of W = U diag(sigma) V^T with
n = 2^22, m = 512, sigma log-spaced 1 -> 1e-8, P-SRHT sketch k = 2048, fp32
working precision with fp64 least squares.  Inputs are resident in HBM before
the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints ONE JSON line on stdout; progress goes to stderr.  ``value`` is the
algorithmic bandwidth of the whole factorisation in GB/s,
  B = b * n * (m(m-1)/2 + 4m) bytes per QR (b = 4 for fp32):
  step 3 reads Q_{i-1} and w_i and writes q'_i, step 1 reads w_i, step 7
  writes q_i.
"""

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def qr_bytes(n, m, b):
    return b * n * (m * (m - 1) / 2 + 4 * m)


def project_bytes(n, m, b):
    """Algorithmic bytes of all projection+sketch launches of one QR:
    column 0 reads w and writes q'; column i >= 1 reads Q_{i-1} (i columns),
    reads w_i, writes q'_i and writes the normalised q_{i-1}."""
    return b * n * (2 + sum(i + 3 for i in range(1, m)))


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_project_srht_f32_n4194304_m512_k2048_traffic.json")


def measured_traffic(n, m, k):
    """HBM bytes per launch of the projection kernel from the committed counter
    record, or None when the record is for another size or the kernel sources
    have changed since the counters were taken."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
    except (OSError, ValueError):
        return None
    if (n, m, k) != (1 << 22, 512, 2048):
        return None
    if sources_sha256(rec["source_files"]) != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


# Gaussian sketch on the fly: VALU instructions per entry of Theta in the
# generated code (one Philox4x32-10 call and two Box-Muller pairs give four
# entries in 89 instructions -- 16 of them 64-bit multiply-adds and 8
# transcendental steps, each counted once -- and one fma applies each entry),
# and the chip's non-packed fp32 VALU issue rate: 256 CUs x 64 lanes x 2.4 GHz
VALU_INSTR_PER_ENTRY = 23.25
VALU_LANE_RATE = 256 * 64 * 2.4e9

# the projection kernel and everything its code is built from
TRAFFIC_SOURCES = ["paper_2011_05090_amd/csrc/rgs_project.hip", "paper_2011_05090_amd/csrc/rgs_proj.hpp",
                   "paper_2011_05090_amd/csrc/rgs_block.hpp", "paper_2011_05090_amd/csrc/rgs_device.hpp",
                   "paper_2011_05090_amd/csrc/rgs_types.hpp"]
PROJECT_KERNEL = "k_project<float, float, float, 1, false>"      # fp32 basis, P-SRHT, normalised storage


def sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def classical_gs_fp32(torch, W, variant):
    """The classical Gram-Schmidt processes the paper compares RGS with
    (Sec. 1.2, Sec. 5.1), in float32 throughout, on the GPU through torch
    (comparison code, not part of the library): 'cgs' q' = w - Q (Q^T w);
    'cgs2' the same projection twice; 'mgs' one previous column at a time;
    then q = q' / ||q'||.  Returns Q (float32) and R (float32)."""
    n, m = W.shape
    Q = torch.empty((m, n), dtype=torch.float32, device=W.device).t()
    R = torch.zeros((m, m), dtype=torch.float32, device=W.device)
    for i in range(m):
        v = W[:, i].float().clone()
        if i > 0:
            Qi = Q[:, :i]
            if variant == "mgs":
                for j in range(i):
                    c = torch.dot(Q[:, j], v)
                    v.sub_(c * Q[:, j])
                    R[j, i] = c
            else:
                y = Qi.t().mv(v)
                v.sub_(Qi.mv(y))
                if variant == "cgs2":
                    y2 = Qi.t().mv(v)
                    v.sub_(Qi.mv(y2))
                    y = y + y2
                R[:i, i] = y
        nv = torch.linalg.vector_norm(v)
        R[i, i] = nv
        Q[:, i] = v / nv
    return Q, R


def cgs2_fp64(torch, W, Q, R):
    """Classical Gram-Schmidt with reorthogonalisation in fp64 on the GPU, for
    the comparison the workload names (not part of the library; torch's
    matrix-vector products, i.e. rocBLAS dgemv): per column
    q' = w - Q (Q^T w), q'' = q' - Q (Q^T q'), q = q'' / ||q''||, with R
    accumulating both coefficient vectors.  Four passes over Q_{i-1} per column
    (8 n (i - 1) bytes each) against RGS's one."""
    import numpy as np
    n, m = W.shape
    R.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(m):
        v = W[:, i].clone()
        if i > 0:
            Qi = Q[:, :i]
            y1 = Qi.t().mv(v)
            v.sub_(Qi.mv(y1))
            y2 = Qi.t().mv(v)
            v.sub_(Qi.mv(y2))
            R[:i, i] = y1 + y2
        nv = torch.linalg.vector_norm(v)
        R[i, i] = nv
        Q[:, i] = v / nv
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = float(torch.linalg.norm(W - Q @ R) / torch.linalg.norm(W))
    o2 = float(np.linalg.norm(np.eye(m) - (Q.t() @ Q).cpu().numpy(), 2))
    nbytes = 4.0 * 8 * n * m * (m - 1) / 2 + 3.0 * 8 * n * m
    return {"ms_per_qr": dt * 1000.0, "algorithmic_bytes": nbytes, "gbs": nbytes / dt / 1e9,
            "backward_error": res, "norm2_I_minus_QtQ": o2,
            "how": "torch fp64: two Q^T v / v - Q y passes per column (rocBLAS dgemv), one run"}


def calibration_copy(torch, dev):
    """A plain 1 GiB device-to-device copy (1 GiB read + 1 GiB written): the
    reference the HBM byte counters of a run are scaled by."""
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log("calibration copy: 1 GiB read + 1 GiB written")
    del src, dst


def _pmc_rows(db, counter):
    import sqlite3
    con = sqlite3.connect(db)
    out = list(con.execute("select dispatch_id, kernel_name, value from counters_collection "
                           "where counter_name=? order by dispatch_id", (counter,)))
    con.close()
    return out


def write_batched_traffic_record(fetch_db, write_db, sketch, batch=2048):
    """HBM traffic of one batched QR call (the leg's second call: the first
    warms up and, for the Gaussian products, tunes their schedule) from two
    rocprofv3 --pmc databases: every library kernel of the call, summed, with
    the counters scaled by the closing 1 GiB copy; beside the call's
    algorithmic bytes.  A call ends with the closing scale pass of each of its
    two shares, and the host waits for it before the next call, so the second
    call is every dispatch after the first call's last scale pass up to its
    own last one (the table generation of the bf16-table sketch included).
    Written to profiles/rgs_qr_batched_2048_<sketch>_traffic.json."""
    import synth
    per = {}
    kernels = {}
    for name, db, counter in (("fetch", fetch_db, "FETCH_SIZE"), ("write", write_db, "WRITE_SIZE")):
        r = _pmc_rows(db, counter)
        copies = [v for _, kn, v in r if "copyBuffer" in kn]
        ends = [d for d, kn, _ in r if "kb_scale" in kn]
        if not copies or len(ends) < 4:
            raise SystemExit("%s: expected two calls (two shares each) and a closing copy" % db)
        after, last = ends[1], ends[3]
        factor = copies[-1] * 1024.0 / (1 << 30)
        tot = 0.0
        for d, kn, v in r:
            if after < d <= last and "rgs::" in kn:
                tot += v
                key = kn.split("(")[0]
                kernels.setdefault(key, {"fetch_kib": 0.0, "write_kib": 0.0, "dispatches": 0})
                kernels[key][name + "_kib"] += v
                if name == "fetch":
                    kernels[key]["dispatches"] += 1
        per[name] = (tot, copies[-1], factor)
    ns, ms = synth.batch_qr_sizes(batch)
    alg = float(sum(batched_qr_bytes(int(n), int(m)) for n, m in zip(ns, ms)))
    traffic = per["fetch"][0] * 1024.0 / per["fetch"][2] + per["write"][0] * 1024.0 / per["write"][2]
    rec = {"workload": "batched RGS QR, %d factorisations, n ~ U{4096..262144}, m ~ U{16..128}, k = 4m, fp32 W, "
                       "bf16 Q, sketch %s; one call" % (batch, sketch),
           "fetch_kib_raw": per["fetch"][0], "write_kib_raw": per["write"][0],
           "copy_calibration": {"fetch_size_kib": per["fetch"][1], "write_size_kib": per["write"][1],
                                "fetch_factor": per["fetch"][2], "write_factor": per["write"][2]},
           "traffic_bytes": traffic, "algorithmic_bytes": alg, "traffic_over_algorithmic": traffic / alg,
           "kernels": {k: dict(v, fetch_bytes=v["fetch_kib"] * 1024.0 / per["fetch"][2],
                               write_bytes=v["write_kib"] * 1024.0 / per["write"][2])
                       for k, v in sorted(kernels.items(), key=lambda x: -x[1]["fetch_kib"])}}
    path = os.path.join(ROOT, "profiles", "rgs_qr_batched_2048_%s_traffic.json" % sketch)
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({k: v for k, v in rec.items() if k != "kernels"}, indent=1))


def write_traffic_record(fetch_db, write_db, n=1 << 22, m=512, k=2048):
    """Turn two rocprofv3 --pmc databases (FETCH_SIZE, then WRITE_SIZE, of
    ``bench.py --steps 1 --warmup 0 --no-extra --no-cpu-baseline --no-gmres
    --calibrate-copy``) into the HBM-traffic record read by ``measured_traffic``.
    The counters are scaled by what they read for the closing 1 GiB device copy."""
    import sqlite3

    def rows(db, counter):
        con = sqlite3.connect(db)
        out = list(con.execute("select dispatch_id, kernel_name, value from counters_collection "
                               "where counter_name=? order by dispatch_id", (counter,)))
        con.close()
        return out

    rec = {"kernel": "rgs::" + PROJECT_KERNEL,
           "workload": "RGS QR fp32/fp64-LS, P-SRHT, n=%d, m=%d, k=%d (one factorisation = %d launches)" % (n, m, k, m)}
    per = {}
    for name, db, counter in (("fetch", fetch_db, "FETCH_SIZE"), ("write", write_db, "WRITE_SIZE")):
        r = rows(db, counter)
        proj = [v for _, kn, v in r if PROJECT_KERNEL in kn]
        copies = [v for _, kn, v in r if "copyBuffer" in kn]
        if len(proj) != m or not copies:
            raise SystemExit("%s: expected %d projection dispatches and a closing copy, found %d and %d" %
                             (db, m, len(proj), len(copies)))
        cal_kib = copies[-1]
        factor = cal_kib * 1024.0 / (1 << 30)       # counter KiB per byte moved, from the 1 GiB copy
        per[name] = (sum(proj) / m, cal_kib, factor)
    fetch_kib, fcal, ff = per["fetch"]
    write_kib, wcal, wf = per["write"]
    traffic = fetch_kib * 1024.0 / ff + write_kib * 1024.0 / wf
    alg = project_bytes(n, m, 4) / m
    rec.update({"launches": m, "fetch_size_kib_per_launch_raw": fetch_kib, "write_size_kib_per_launch_raw": write_kib,
                "copy_calibration": {"kernel": "__amd_rocclr_copyBuffer", "bytes_read": 1 << 30,
                                     "bytes_written": 1 << 30, "fetch_size_kib": fcal, "write_size_kib": wcal,
                                     "fetch_factor": ff, "write_factor": wf},
                "traffic_bytes_per_launch": traffic, "algorithmic_bytes_per_launch": alg,
                "source_files": TRAFFIC_SOURCES, "source_sha256": sources_sha256(TRAFFIC_SOURCES),
                "traffic_over_algorithmic": traffic / alg})
    with open(TRAFFIC_RECORD, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def run_steps(rgs, torch, h, desc, W, Q, R, S, steps, warmup):
    for _ in range(warmup):
        rgs.rgs_qr(h, desc, W, Q, R, S)
    torch.cuda.synchronize()
    kern_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        rep = rgs.rgs_qr(h, desc, W, Q, R, S)
        kern_ms += rep.proj_kernel_ms
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1000.0 / steps, kern_ms, rep


def quality(torch, W, Q, R, S):
    """||W - QR||_F/||W||_F, ||I - S^T S||_2, ||I - Q^T Q||_2 in fp64 (not timed).
    Products on the device, the m x m spectral norms on the host."""
    import numpy as np
    W64 = W.double()
    Q64 = Q.double()
    res = torch.linalg.norm(W64 - Q64 @ R) / torch.linalg.norm(W64)
    m = S.shape[1]
    I = np.eye(m)
    d2 = np.linalg.norm(I - (S.T @ S).cpu().numpy(), 2)
    o2 = np.linalg.norm(I - (Q64.T @ Q64).cpu().numpy(), 2)
    del W64, Q64
    return float(res), float(d2), float(o2)


def host_info():
    """CPU model, logical cores and RAM of the host, and the BLAS thread count."""
    info = {"logical_cpus": os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    try:
        import threadpoolctl
        info["blas_threads"] = max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info())
    except Exception:
        pass
    return info


def cpu_baseline(n=1 << 16, m=512, k=2048):
    """The oracle (fp32 model, P-SRHT) on a bounded sample of the headline
    workload -- the same m, k, sketch and conditioning, n cut to 2^16 -- on the
    host cores."""
    import numpy as np
    import synth
    from oracle import rgs as orgs, sketch as osk
    W = synth.svd_matrix(n, m, 1e-8, tag=0).astype(np.float32)
    th = osk.SRHT(n, k, seed=42)
    t0 = time.perf_counter()
    orgs.rgs_qr(W, th, precision="fp32")
    dt = time.perf_counter() - t0
    hi = host_info()
    cores = hi.get("blas_threads") or os.cpu_count()
    return {"value": qr_bytes(n, m, 4) / dt / 1e9, "unit": "GB/s", "cores": int(cores), "kind": "oracle",
            "sample": "oracle fp32-model RGS, P-SRHT k=%d, W %dx%d (sigma 1..1e-8; the headline's m, k and "
                      "conditioning at n = 2^16), %.1f s wall" % (k, n, m, dt),
            "host": hi}


def small_fp64_leg(rgs, torch, synth, h, n=16384, m=64, k=256, steps=20, warmup=3):
    """Plain fp64 RGS with the Gaussian sketch at n = 16384, m = 64, k = 256: a
    latency-bound size (64 dependent column steps), reported in us per column,
    launched eagerly and replayed as one captured HIP graph (RGS_FLAG_GRAPH;
    the first warmup call captures it)."""
    W = rgs.colmajor(n, m, torch.float64)
    W.copy_(torch.from_numpy(synth.svd_matrix(n, m, 1e-6, tag=0)))
    Q = rgs.colmajor(n, m, torch.float64)
    R = rgs.colmajor(m, m, torch.float64)
    S = rgs.colmajor(k, m, torch.float64)
    d = rgs.qr_desc(n, m, k, sketch="gaussian", prec="fp64")
    ms, _, rep = run_steps(rgs, torch, h, d, W, Q, R, S, steps, warmup)
    res, d2, o2 = quality(torch, W, Q, R, S)
    out = {"n": n, "m": m, "k": k, "sketch": "gaussian", "ms_per_qr": ms, "us_per_column": 1000.0 * ms / m,
           "gbs": qr_bytes(n, m, 8) / (ms / 1000.0) / 1e9, "status": rep.status, "backward_error": res,
           "norm2_I_minus_StS": d2}
    log("  fp64 RGS n=%d m=%d k=%d Gaussian: %.3f ms/QR (%.1f us/column), ||W-QR||/||W|| %.2e" %
        (n, m, k, ms, 1000.0 * ms / m, res))
    dg = rgs.qr_desc(n, m, k, sketch="gaussian", prec="fp64", flags=rgs.FLAG_GRAPH)
    ms_g, _, rep_g = run_steps(rgs, torch, h, dg, W, Q, R, S, steps, warmup)
    res_g, _, _ = quality(torch, W, Q, R, S)
    out["graph"] = {"ms_per_qr": ms_g, "us_per_column": 1000.0 * ms_g / m, "status": rep_g.status,
                    "backward_error": res_g}
    log("  same, graph-replayed: %.3f ms/QR (%.1f us/column)" % (ms_g, 1000.0 * ms_g / m))
    # the same sketch read from the table of its exact fp64 entries (made once per call)
    for key, fl in (("exact_table", rgs.FLAG_THETA_EXACT), ("exact_table_graph", rgs.FLAG_THETA_EXACT | rgs.FLAG_GRAPH)):
        dx = rgs.qr_desc(n, m, k, sketch="gaussian", prec="fp64", flags=fl)
        ms_x, _, rep_x = run_steps(rgs, torch, h, dx, W, Q, R, S, steps, warmup)
        res_x, _, _ = quality(torch, W, Q, R, S)
        out[key] = {"ms_per_qr": ms_x, "us_per_column": 1000.0 * ms_x / m, "status": rep_x.status,
                    "backward_error": res_x}
        log("  same, %s: %.3f ms/QR (%.1f us/column)" % (key.replace("_", " "), ms_x, 1000.0 * ms_x / m))
    return out


def batched_qr_bytes(n, m):
    """Algorithmic bytes of one bf16-stored factorisation (fp32 W, bf16 Q):
    P = Theta W reads W (4nm), the projections read w_i (4nm) and Q_{i-1}
    (2n i per column, 2n m(m-1)/2 in all) and write q'_i (2nm), and the closing
    scale pass reads and writes Q (4nm)."""
    return n * (m * (m - 1) + 14 * m)


def gmres_bytes(n, iters, cycles, restart, bq, bw):
    """Algorithmic bytes of a restarted randomized GMRES solve on n unknowns
    (basis element bq bytes, mat-vec output element bw bytes), from its
    iteration and cycle counts (every cycle but the last taken as full):
    inner step i (i-th new basis vector) -- the mat-vec reads q_{i-1} and
    writes w, the projection reads Q_{i-1} (i columns) and w and writes q'_i:
    n (bq (i + 2) + 2 bw); per cycle -- the first column (read r in fp64, write
    w, project: 8n + 2 bw n + bq n), the update x += Q y (read the used
    columns, read and write x: bq n u + 16 n) and the restart residual (read b
    and x, write r: 24 n)."""
    total = 0.0
    left = int(iters)
    for c in range(int(cycles)):
        u = min(int(restart), left) if c < cycles - 1 else left
        left -= u
        total += n * (bq * (u * (u + 1) / 2 + 2 * u) + 2 * bw * u)
        total += 8 * n + 2 * bw * n + bq * n + bq * n * u + 16 * n + 24 * n
    return total


def copy_ceiling(torch, dev, reps=7):
    """Measured HBM ceiling of a plain device copy: (bytes read + written) / time,
    median over reps of a 1 GiB fp32 copy, timed with events on the current stream."""
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1000.0)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / sorted(times)[len(times) // 2] / 1e9


def rademacher_leg(rgs, torch, synth, h, n=1 << 22, m=512, k=2048, steps=1, warmup=1):
    """fp32 RGS with the Rademacher sketch at the headline size (W = U Sigma V^T,
    sigma 1..1e-8): time per QR, the fused projection + sketch kernel per
    column (events around every launch), and the quality.  A profiling aid
    for the kernel's counters (`--only rademacher`)."""
    W64 = synth.svd_matrix_torch(n, m, 1e-8, tag=0)
    W = rgs.colmajor(n, m, torch.float32)
    W.copy_(W64)
    del W64
    Q = rgs.colmajor(n, m, torch.float32)
    R = rgs.colmajor(m, m, torch.float64)
    S = rgs.colmajor(k, m, torch.float64)
    d = rgs.qr_desc(n, m, k, sketch="rademacher", prec="fp32", flags=rgs.FLAG_TIME_KERNELS)
    ms, kern_ms, rep = run_steps(rgs, torch, h, d, W, Q, R, S, steps, warmup)
    res, d2, o2 = quality(torch, W, Q, R, S)
    per_col = kern_ms / steps / m
    out = {"n": n, "m": m, "k": k, "ms_per_qr": ms, "status": rep.status,
           "projection_ms_per_column": per_col,
           "projection_gbs": project_bytes(n, m, 4) / m / (per_col / 1000) / 1e9,
           "backward_error": res, "norm2_I_minus_StS": d2, "norm2_I_minus_QtQ": o2}
    log("  rademacher fp32: %.1f ms/QR, fused kernel %.3f ms per column (%.0f GB/s), ||W-QR||/||W|| %.2e" %
        (ms, per_col, out["projection_gbs"], res))
    del W, Q, R, S
    torch.cuda.empty_cache()
    return out


def batched_qr_leg(rgs, torch, synth, h, batch=2048,
                   sketches=("srht", "srht_richardson2", "gaussian", "gaussian_exact_table",
                             "gaussian_bf16_table"), steps=2,
                   warmup=1, gaussian_batch=2048, graph=True):
    """Batched RGS QR: ``batch`` factorisations with n ~ U{4096..262144},
    m ~ U{16..128}, k = 4m, sigma 1..1e-6, fp32 W and bf16-stored Q, all in
    one rgs_qr_batched call, with the P-SRHT, with the Gaussian sketch (the
    factorisations share one master Gaussian matrix, entries drawn in the
    products) and with that master matrix's bf16 entries made once per call
    into a table that the products read through bf16 matrix cores
    (RGS_FLAG_THETA_BF16), and with its exact fp32 entries made once per call
    into a table that the fp32 products read instead of drawing them
    (RGS_FLAG_THETA_EXACT: the drawn call's bits); ``srht_richardson2`` is the
    P-SRHT with step 2 by two Richardson sweeps (RGS_FLAG_LS_SWEEPS(2)).  With
    ``graph`` each sketch is timed again with the calls replayed from captured
    graphs (RGS_FLAG_GRAPH)."""
    ns, ms_ = synth.batch_qr_sizes(batch)
    items = []
    t0 = time.perf_counter()
    for b in range(batch):
        n, m = int(ns[b]), int(ms_[b])
        k = 4 * m
        W64 = synth.svd_matrix_torch(n, m, 1e-6, tag=1000 + b)
        W = rgs.colmajor(n, m, torch.float32)
        W.copy_(W64)
        del W64
        items.append((W, rgs.colmajor(n, m, torch.bfloat16), rgs.colmajor(m, m, torch.float64),
                      rgs.colmajor(k, m, torch.float64), k))
    torch.cuda.synchronize()
    log("  generated %d inputs in %.1f s" % (batch, time.perf_counter() - t0))
    out = {"batch": batch, "n_range": [4096, 262144], "m_range": [16, 128], "k": "4m", "q_dtype": "bf16",
           "sigma_min": 1e-6}
    for sketch in sketches:
        lib_sketch = "srht" if sketch.startswith("srht") else "gaussian"
        its = items if lib_sketch == "srht" else items[:gaussian_batch]
        B = sum(batched_qr_bytes(W.shape[0], W.shape[1]) for W, *_ in its)
        flags = {"gaussian_bf16_table": rgs.FLAG_THETA_BF16, "gaussian_exact_table": rgs.FLAG_THETA_EXACT,
                 "srht_richardson2": rgs.flag_ls_sweeps(2)}.get(sketch, 0)
        for _ in range(warmup):
            rgs.rgs_qr_batched(h, its, sketch=lib_sketch, prec="bf16q", flags=flags)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rep, stat, _ = rgs.rgs_qr_batched(h, its, sketch=lib_sketch, prec="bf16q", flags=flags)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        bad = sum(1 for v in stat if v != 0)
        # the same calls replayed from captured graphs (RGS_FLAG_GRAPH; the first call captures)
        dt_graph = None
        if graph:
            rgs.rgs_qr_batched(h, its, sketch=lib_sketch, prec="bf16q", flags=flags | rgs.FLAG_GRAPH)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                rep_g, stat_g, _ = rgs.rgs_qr_batched(h, its, sketch=lib_sketch, prec="bf16q",
                                                      flags=flags | rgs.FLAG_GRAPH)
            torch.cuda.synchronize()
            dt_graph = (time.perf_counter() - t0) / steps
            bad += sum(1 for v in stat_g if v != 0)
        # quality on a few items (fp64 on the device, spectral norms on the host)
        import numpy as np
        worst_be, worst_d2 = 0.0, 0.0
        for W, Q, R, S, _ in its[:: max(1, len(its) // 8)]:
            be, d2, _ = quality(torch, W, Q.float(), R, S)
            worst_be, worst_d2 = max(worst_be, be), max(worst_d2, d2)
        if lib_sketch != "srht":   # autotuned sketch-product schedule (1..9)
            out[sketch + "_schedule"] = rgs.rgs_last_tuning(h)
        out[sketch] = {"items": len(its), "seconds": dt, "algorithmic_bytes": B, "gbs": B / dt / 1e9,
                       "pct_hbm_peak": 100.0 * B / dt / 1e9 / HBM_PEAK_GBS, "graph_seconds": dt_graph,
                       "failed_items": bad,
                       "status": rep.status, "sampled_max_backward_error": worst_be,
                       "sampled_max_norm2_I_minus_StS": worst_d2}
        log("  batched %s x%d: %.3f s (graph replay %s s), %.1f GB/s algorithmic, max sampled "
            "||W-QR||/||W|| %.2e, ||I-S^TS||_2 %.2e, failed %d"
            % (sketch, len(its), dt, "-" if dt_graph is None else "%.3f" % dt_graph, B / dt / 1e9,
               worst_be, worst_d2, bad))
    del items
    torch.cuda.empty_cache()
    return out


def batched_gmres_leg(rgs, torch, synth, h, batch=256, restart=50, k=200, tol=1e-6, gaussian_batch=32):
    """Batched randomized GMRES: ``batch`` convection-diffusion systems on grids
    N^3, N ~ U{32..96}, Pe ~ U[1, 100], b ~ N(0, 1), restart 50, k = 200,
    tol 1e-6, one rgs_gmres_batched call with graph-replayed cycles.  The bf16
    and fp32 bases are compared with plain fp64 on the same GPU (iteration
    counts per system).  The Gaussian sketch drawn on the fly regenerates its
    entries per system, so it runs on the first ``gaussian_batch`` systems
    only; the Gaussian sketch with bf16 entries (one table per cycle shared by
    all systems) runs on the whole batch."""
    Ns, Pes = synth.batch_gmres_sizes(batch)
    systems = []
    for i, (N, Pe) in enumerate(zip(Ns, Pes)):
        dims, coeffs = synth.convdiff_coeffs(int(N), float(Pe))
        b = torch.from_numpy(synth.rhs(int(N) ** 3, tag=1000 + i)).to("cuda")
        systems.append((rgs.stencil7(dims, coeffs), b, torch.empty_like(b)))
    n_tot = int(sum(int(N) ** 3 for N in Ns))
    out = {"batch": batch, "N_range": [32, 96], "Pe_range": [1.0, 100.0], "restart": restart, "k": k, "tol": tol,
           "unknowns": n_tot}
    for variant in ("srht", "gaussian", "gaussian_bf16_table"):
        sketch = "srht" if variant == "srht" else "gaussian"
        flags = rgs.FLAG_GRAPH | (rgs.FLAG_THETA_BF16 if variant == "gaussian_bf16_table" else 0)
        sy = systems[:gaussian_batch] if variant == "gaussian" else systems
        res = {"systems": len(sy)}
        iters = {}
        for prec in ("bf16q", "fp32", "fp64"):
            d = rgs.gmres_desc(restart, k, tol, max_iters=20000, sketch=sketch, prec=prec, flags=flags)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, stat, reps, _ = rgs.rgs_gmres_batched(h, sy, d)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            iters[prec] = [r.iters for r in reps]
            bq, bw = {"bf16q": (2, 4), "fp32": (4, 4), "fp64": (8, 8)}[prec]
            nbytes = sum(gmres_bytes(A.nx * A.ny * A.nz, r.iters, r.cycles, restart, bq, bw)
                         for (A, _, _), r in zip(sy, reps))
            res[prec] = {"seconds_to_tol": dt, "status": st, "converged": sum(1 for v in stat if v == 0),
                         "total_iters": int(sum(iters[prec])), "max_cycles": max(r.cycles for r in reps),
                         "max_true_relres": max(r.true_relres for r in reps),
                         "algorithmic_bytes": nbytes, "gbs": nbytes / dt / 1e9,
                         "pct_hbm_peak": 100.0 * nbytes / dt / 1e9 / HBM_PEAK_GBS}
            log("  batched rgmres %s/%s x%d: %.3f s, %d converged, max cycles %d, max relres %.2e, "
                "%.0f GB/s algorithmic" % (variant, prec, len(sy), dt, res[prec]["converged"],
                                           res[prec]["max_cycles"], res[prec]["max_true_relres"], nbytes / dt / 1e9))
        for prec in ("bf16q", "fp32"):
            diff = [a - b for a, b in zip(iters[prec], iters["fp64"])]
            res[prec]["iters_minus_fp64"] = {"min": min(diff), "max": max(diff),
                                             "within_2": sum(1 for v in diff if abs(v) <= 2)}
            res[prec]["speedup_vs_fp64"] = res["fp64"]["seconds_to_tol"] / res[prec]["seconds_to_tol"]
        out[variant] = res
    # variants of the P-SRHT systems, graph-replayed: step 2 by two Richardson sweeps on the normal
    # equations (Sec. 2.3's remark), the lagged Arnoldi step (RGS_FLAG_LAG: both sketches of a step in
    # the mat-vec pass), and the unique-precision model of Sec. 5.3 (float32 RGS, fp64 products with A)
    for key, label, prec, extra_flags, sweeps in (
            ("srht_richardson2_bf16q", "srht/bf16q, 2 Richardson sweeps", "bf16q", 0, 2),
            ("srht_lag_bf16q", "srht/bf16q, lagged step", "bf16q", rgs.FLAG_LAG, 0),
            ("srht_fp32u", "srht/fp32u (Sec. 5.3)", "fp32u", 0, 0)):
        d = rgs.gmres_desc(restart, k, tol, max_iters=20000, sketch="srht", prec=prec,
                           flags=rgs.FLAG_GRAPH | extra_flags, ls_sweeps=sweeps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, stat, reps, _ = rgs.rgs_gmres_batched(h, systems, d)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[key] = {"seconds_to_tol": dt, "status": st, "converged": sum(1 for v in stat if v == 0),
                    "total_iters": int(sum(r.iters for r in reps)),
                    "max_true_relres": max(r.true_relres for r in reps)}
        log("  batched rgmres %s, x%d: %.3f s, %d converged, %d iterations in all" %
            (label, len(systems), dt, out[key]["converged"], out[key]["total_iters"]))
    return out


def sec51_leg(rgs, torch, synth, h, n=10 ** 6, m=300, ks=(1500, 5000), prefixes=(25, 50, 100, 150, 200, 250, 300),
              eps_star=0.05, classical=True):
    """The synthetic-function experiment of Sec. 5.1 at the paper's size: W_ij =
    f_mu_j(x_i) = sin(10 (mu_j + x_i)) / (cos(100 (mu_j - x_i)) + 1.1) on n = 10^6
    evenly spaced x in [0, 1] and m = 300 evenly spaced mu in [0, 1], fp32 W,
    multi-precision RGS (fp32 projection, fp64 least squares) with P-SRHT
    k in {1500, 5000}.  For prefixes W_i (factorised with the a-posteriori
    certificate, Phi of Theta's size, eps* = 0.05) it reports what the paper
    plots: cond(Q_i), cond(S_i), ||W_i - Q_i R_i|| / ||W_i||, the embedding
    distortion omega of Theta on range(Q_i) and its bound omega_bar.  The
    paper's classical comparisons CGS, MGS and CGS2 run in float32 throughout
    (inner products, projections and norms), as torch / rocBLAS operations on
    the same GPU (comparison code, not part of the library); with
    ``classical`` also RGS with Theta = I (one and two Richardson sweeps, the
    Householder solve).  The unique-precision RGS (RGS_P_FP32: every step in
    float32) runs on the same prefixes and sketches as the multi-precision
    one (keys up_k1500, up_k5000).  Metrics are computed in fp64 on the device
    (measurement code)."""
    import numpy as np
    W = rgs.colmajor(n, m, torch.float32)
    W.copy_(torch.from_numpy(synth.f_mu_matrix(n, m, np.float64)).to("cuda"))
    W64 = W.double()
    out = {"n": n, "m": m, "eps_star": eps_star, "precision": "fp32 projection, fp64 LS", "sketch": "srht",
           "up_precision": "float32 throughout (unique precision)"}
    for prec, key in (("fp32", "k%d"), ("fp32u", "up_k%d")):
        for k in ks:
            rows = []
            for i in prefixes:
                Wi = W[:, :i]
                Q = rgs.colmajor(n, i, torch.float32)
                R = rgs.colmajor(i, i, torch.float64)
                S = rgs.colmajor(k, i, torch.float64)
                d = rgs.qr_desc(n, i, k, sketch="srht", prec=prec, flags=rgs.FLAG_CERTIFY)
                rep = rgs.rgs_qr(h, d, Wi, Q, R, S)
                torch.cuda.synchronize()
                Q64 = Q.double()
                G = Q64.T @ Q64
                ev = torch.linalg.eigvalsh(G)
                cond_q = float(torch.sqrt(ev[-1] / ev[0])) if float(ev[0]) > 0 else float("inf")
                sv = torch.linalg.svdvals(S)
                cond_s = float(sv[0] / sv[-1])
                err = float(torch.linalg.norm(W64[:, :i] - Q64 @ R) / torch.linalg.norm(W64[:, :i]))
                omega = float("nan")
                if cond_q < 1e6:
                    # omega: distortion of Theta on range(Q_i), from an l2-orthonormal basis U = Q C^-1
                    C = torch.linalg.cholesky(G, upper=True)
                    U = Q64 @ torch.linalg.inv(C)          # i x i inverse: cond(Q_i) is moderate
                    TU = rgs.colmajor(k, i, torch.float64)
                    rgs.rgs_sketch_apply(h, rgs.qr_desc(n, i, k, sketch="srht", prec="fp64"),
                                         U.contiguous().T.contiguous().T, TU)
                    torch.cuda.synchronize()
                    omega = float(torch.linalg.matrix_norm(torch.eye(i, dtype=torch.float64, device="cuda") -
                                                           TU.T @ TU, 2))
                    del C, U, TU
                obar = rgs.rgs_omega_bar(rep.cert_smin_q, rep.cert_smax_q, eps_star)
                rows.append({"i": i, "status": rep.status, "cond_Q": cond_q, "cond_S": cond_s, "error": err,
                             "omega": omega, "omega_bar": obar, "seconds": rep.seconds})
                log("  sec5.1 %s k=%d i=%d: cond(Q) %.3f cond(S) %.3f err %.2e omega %.3f omega_bar %.3f (%.1f ms)" %
                    (prec, k, i, cond_q, cond_s, err, omega, obar, 1000 * rep.seconds))
                del Q, R, S, Q64, G
            out[key % k] = rows
    # the classical comparisons in float32 throughout (torch on the device)
    for name in ("cgs_fp32", "mgs_fp32", "cgs2_fp32"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Q, R = classical_gs_fp32(torch, W, name.split("_")[0])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rows = []
        for i in prefixes:
            Q64 = Q[:, :i].double()
            ev = torch.linalg.eigvalsh(Q64.T @ Q64)
            cond_q = float(torch.sqrt(ev[-1] / ev[0])) if float(ev[0]) > 0 else float("inf")
            err = float(torch.linalg.norm(W64[:, :i] - Q64 @ R[:i, :i].double()) / torch.linalg.norm(W64[:, :i]))
            rows.append({"i": i, "cond_Q": cond_q, "error": err})
            log("  sec5.1 %s i=%d: cond(Q) %.3e err %.2e" % (name, i, cond_q, err))
            del Q64
        out[name] = {"seconds": dt, "rows": rows, "precision": "float32 throughout (torch on the GPU, comparison)"}
        del Q, R
    # Theta = I (k = n): with one Richardson sweep of the least squares the
    # column step is classical Gram-Schmidt (fp32 projection, inner products in
    # fp64; the paper's CGS is float32 throughout); two sweeps refine the
    # coefficients only (CGS2 in
    # exact arithmetic, but the rounded projection is not projected again);
    # the Householder solve is Gram-Schmidt with an exact least squares.
    # Column i depends on columns <= i only, so one factorisation of all m
    # columns gives every prefix.
    # (about 30 s each: the sketch space is n-dimensional, so they run with
    # --only sec51, not in the default run)
    for name, sweeps in (("cgs", 1), ("identity_richardson2", 2), ("identity_householder", 0)) if classical else ():
        Q = rgs.colmajor(n, m, torch.float32)
        R = rgs.colmajor(m, m, torch.float64)
        S = rgs.colmajor(n, m, torch.float64)
        d = rgs.qr_desc(n, m, n, sketch="identity", prec="fp32", ls_sweeps=sweeps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = rgs.rgs_qr(h, d, W, Q, R, S)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rows = []
        for i in prefixes:
            if rep.status != 0 and i > rep.failed_column:
                break
            Q64 = Q[:, :i].double()
            ev = torch.linalg.eigvalsh(Q64.T @ Q64)
            cond_q = float(torch.sqrt(ev[-1] / ev[0])) if float(ev[0]) > 0 else float("inf")
            err = float(torch.linalg.norm(W64[:, :i] - Q64 @ R[:i, :i]) / torch.linalg.norm(W64[:, :i]))
            rows.append({"i": i, "cond_Q": cond_q, "error": err})
            log("  sec5.1 %s i=%d: cond(Q) %.3e err %.2e" % (name, i, cond_q, err))
            del Q64
        out[name] = {"status": rep.status, "failed_column": rep.failed_column, "seconds": dt, "rows": rows,
                     "precision": "fp32 projection, fp64 least squares, Theta = I, %s" %
                                  ("%d Richardson sweep%s" % (sweeps, "" if sweeps == 1 else "s") if sweeps
                                   else "Householder least squares")}
        del Q, R, S
    del W, W64
    return out


def gmres_leg(rgs, torch, synth, h, N=192, Pe=50.0, restart=100, k=400, tol=1e-6):
    """Time-to-1e-6 of restarted randomized GMRES on the 7-point convection-diffusion
    system (N^3 unknowns, b ~ N(0,1)), fp32 basis vs plain fp64, Gaussian and SRHT."""
    dims, coeffs = synth.convdiff_coeffs(N, Pe)
    n = N ** 3
    b = torch.from_numpy(synth.rhs(n, tag=0)).to("cuda")
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    A = rgs.stencil7(dims, coeffs)
    res = {"grid": N, "n": n, "Pe": Pe, "restart": restart, "k": k, "tol": tol}
    for sketch in ("gaussian", "srht"):
        for prec in ("fp32", "fp64"):
            d = rgs.gmres_desc(restart, k, tol, max_iters=20000, sketch=sketch, prec=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep, _ = rgs.rgs_gmres(h, A, d, b, x)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            bq = 4 if prec == "fp32" else 8
            nbytes = gmres_bytes(n, rep.iters, rep.cycles, restart, bq, bq)
            res["%s_%s" % (sketch, prec)] = {"seconds_to_tol": dt, "iters": rep.iters, "cycles": rep.cycles,
                                             "true_relres": rep.true_relres, "status": rep.status,
                                             "algorithmic_bytes": nbytes, "gbs": nbytes / dt / 1e9,
                                             "pct_hbm_peak": 100.0 * nbytes / dt / 1e9 / HBM_PEAK_GBS}
            log("  rgmres %s/%s: %d iters, %d cycles, relres %.2e, %.3f s, %.0f GB/s algorithmic" %
                (sketch, prec, rep.iters, rep.cycles, rep.true_relres, dt, nbytes / dt / 1e9))
        res["%s_speedup_fp32_vs_fp64" % sketch] = (res["%s_fp64" % sketch]["seconds_to_tol"] /
                                                   res["%s_fp32" % sketch]["seconds_to_tol"])
    # the Gaussian sketch with bf16 entries, made once per cycle into a table (RGS_FLAG_THETA_BF16)
    d = rgs.gmres_desc(restart, k, tol, max_iters=20000, sketch="gaussian", prec="fp32", flags=rgs.FLAG_THETA_BF16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep, _ = rgs.rgs_gmres(h, A, d, b, x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res["gaussian_bf16_table_fp32"] = {"seconds_to_tol": dt, "iters": rep.iters, "cycles": rep.cycles,
                                       "true_relres": rep.true_relres, "status": rep.status,
                                       "speedup_vs_fp64_gaussian": res["gaussian_fp64"]["seconds_to_tol"] / dt}
    log("  rgmres gaussian(bf16 table)/fp32: %d iters, %d cycles, relres %.2e, %.3f s" %
        (rep.iters, rep.cycles, rep.true_relres, dt))
    # the same Gaussian sketch with its entries made once per cycle into a table in the
    # working precision (RGS_FLAG_THETA_EXACT): the sketch becomes a memory stream
    for prec in ("fp32", "fp64"):
        d = rgs.gmres_desc(restart, k, tol, max_iters=20000, sketch="gaussian", prec=prec,
                           flags=rgs.FLAG_THETA_EXACT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep, _ = rgs.rgs_gmres(h, A, d, b, x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bq = 4 if prec == "fp32" else 8
        nbytes = gmres_bytes(n, rep.iters, rep.cycles, restart, bq, bq)
        res["gaussian_exact_table_%s" % prec] = {
            "seconds_to_tol": dt, "iters": rep.iters, "cycles": rep.cycles, "true_relres": rep.true_relres,
            "status": rep.status, "table_bytes": bq * k * ((n + 7) // 8 * 8),
            "speedup_vs_drawn": res["gaussian_%s" % prec]["seconds_to_tol"] / dt}
        log("  rgmres gaussian(exact table)/%s: %d iters, %d cycles, relres %.2e, %.3f s (%.2fx the drawn sketch)" %
            (prec, rep.iters, rep.cycles, rep.true_relres, dt, res["gaussian_%s" % prec]["seconds_to_tol"] / dt))
    # the configuration of the GMRES experiment of Sec. 5.3: unique-precision (float32) RGS with the
    # products with A in fp64 (RGS_P_FP32)
    for sketch in ("srht", "gaussian"):
        d = rgs.gmres_desc(restart, k, tol, max_iters=20000, sketch=sketch, prec="fp32u")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep, _ = rgs.rgs_gmres(h, A, d, b, x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nbytes = gmres_bytes(n, rep.iters, rep.cycles, restart, 4, 4)
        res["%s_fp32u" % sketch] = {"seconds_to_tol": dt, "iters": rep.iters, "cycles": rep.cycles,
                                    "true_relres": rep.true_relres, "status": rep.status,
                                    "algorithmic_bytes": nbytes, "gbs": nbytes / dt / 1e9,
                                    "speedup_vs_fp64": res["%s_fp64" % sketch]["seconds_to_tol"] / dt}
        log("  rgmres %s/fp32u (Sec. 5.3: float32 RGS, fp64 mat-vec): %d iters, %d cycles, relres %.2e, %.3f s" %
            (sketch, rep.iters, rep.cycles, rep.true_relres, dt))
    # the P-SRHT with the lagged Arnoldi step (RGS_FLAG_LAG): both sketches of a step in the mat-vec pass
    for prec in ("fp32", "fp64"):
        d = rgs.gmres_desc(restart, k, tol, max_iters=20000, sketch="srht", prec=prec, flags=rgs.FLAG_LAG)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep, _ = rgs.rgs_gmres(h, A, d, b, x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bq = 4 if prec == "fp32" else 8
        nbytes = gmres_bytes(n, rep.iters, rep.cycles, restart, bq, bq)
        res["srht_lag_%s" % prec] = {"seconds_to_tol": dt, "iters": rep.iters, "cycles": rep.cycles,
                                     "true_relres": rep.true_relres, "status": rep.status,
                                     "algorithmic_bytes": nbytes, "gbs": nbytes / dt / 1e9,
                                     "pct_hbm_peak": 100.0 * nbytes / dt / 1e9 / HBM_PEAK_GBS}
        log("  rgmres srht(lagged step)/%s: %d iters, %d cycles, relres %.2e, %.3f s" %
            (prec, rep.iters, rep.cycles, rep.true_relres, dt))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--m", type=int, default=512)
    ap.add_argument("--k", type=int, default=2048)
    ap.add_argument("--no-extra", action="store_true", help="skip the fp64 / Gaussian / companion QR legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gmres", action="store_true", help="skip the randomized GMRES leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched and small fp64 QR legs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--only", choices=["small", "batched-qr", "batched-gmres", "gmres", "sec51", "rademacher"],
                    help="profiling aid: run only this leg and print its JSON (not the benchmark line)")
    ap.add_argument("--traffic-record", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write the projection kernel's HBM-traffic record from two rocprofv3 --pmc "
                         "databases (no GPU needed) and exit")
    ap.add_argument("--sketches", default=None,
                    help="with --only batched-qr: comma-separated legs (srht, srht_richardson2, gaussian, "
                         "gaussian_exact_table, gaussian_bf16_table)")
    ap.add_argument("--leg-steps", type=int, default=None, help="with --only: timed calls per leg")
    ap.add_argument("--leg-warmup", type=int, default=None, help="with --only: untimed calls per leg")
    ap.add_argument("--no-graph", action="store_true",
                    help="with --only batched-qr: skip the graph-replayed timing")
    ap.add_argument("--batched-traffic", nargs=3, metavar=("FETCH_DB", "WRITE_DB", "SKETCH"),
                    help="write the HBM-traffic record of one batched QR call from two rocprofv3 --pmc "
                         "databases of 'bench.py --only batched-qr --sketches SKETCH --leg-warmup 1 --no-graph "
                         "--leg-steps 1 --calibrate-copy' (no GPU needed) and exit")
    args = ap.parse_args()
    if args.traffic_record:
        write_traffic_record(*args.traffic_record)
        return
    if args.batched_traffic:
        write_batched_traffic_record(*args.batched_traffic)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(rows would be sharded by blocks with one all-reduce of the sketch per column); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2011_05090_amd as rgs

    if args.only:
        h = rgs.Handle(0)
        leg = {"small": small_fp64_leg, "batched-qr": batched_qr_leg, "batched-gmres": batched_gmres_leg,
               "gmres": gmres_leg, "sec51": sec51_leg, "rademacher": rademacher_leg}[args.only]
        kw = {}
        if args.leg_steps is not None:
            kw["steps"] = args.leg_steps
        if args.leg_warmup is not None:
            kw["warmup"] = args.leg_warmup
        if args.sketches and args.only == "batched-qr":
            kw["sketches"] = tuple(args.sketches.split(","))
        if args.no_graph and args.only == "batched-qr":
            kw["graph"] = False
        res = leg(rgs, torch, synth, h, **kw)
        if args.calibrate_copy:
            calibration_copy(torch, torch.device("cuda:0"))
        h.close()
        print(json.dumps({"only": args.only, "result": res}), flush=True)
        return
    n, m, k = args.n, args.m, args.k
    dev = torch.device("cuda:0")
    log("generating W (%d x %d, sigma 1..1e-8) on the device" % (n, m))
    W64 = synth.svd_matrix_torch(n, m, 1e-8, tag=0, device=dev)
    W32 = rgs.colmajor(n, m, torch.float32)
    W32.copy_(W64)
    Q = rgs.colmajor(n, m, torch.float32)
    R = rgs.colmajor(m, m, torch.float64)
    S = rgs.colmajor(k, m, torch.float64)
    h = rgs.Handle(0)

    desc = rgs.qr_desc(n, m, k, sketch="srht", prec="fp32", flags=rgs.FLAG_TIME_KERNELS)
    log("fp32/fp64-LS RGS, SRHT: warmup %d, steps %d" % (args.warmup, args.steps))
    ms, kern_ms, rep = run_steps(rgs, torch, h, desc, W32, Q, R, S, args.steps, args.warmup)
    if rep.status != 0:
        raise SystemExit("rgs_qr failed: status %d at column %d" % (rep.status, rep.failed_column))
    B = qr_bytes(n, m, 4)
    value = B / (ms / 1000.0) / 1e9
    avg_launch_ms = kern_ms / (args.steps * m)
    avg_launch_bytes = project_bytes(n, m, 4) / m
    achieved = avg_launch_bytes / (avg_launch_ms / 1000.0) / 1e9
    res, d2, o2 = quality(torch, W32, Q, R, S)
    copy_gbs = copy_ceiling(torch, dev)
    log("  device copy ceiling: %.1f GB/s (read + write bytes)" % copy_gbs)
    log("  %.2f ms/QR  %.1f GB/s  (%.1f%% of HBM peak); projection kernel %.1f GB/s; "
        "||W-QR||/||W|| %.2e  ||I-S^TS||_2 %.2e  ||I-Q^TQ||_2 %.2e" %
        (ms, value, 100 * value / HBM_PEAK_GBS, achieved, res, d2, o2))
    out = {
        "metric": "RGS QR GB/s (% HBM peak) & RGMRES time-to-1e-6 vs plain FP64 RGS, 1 GPU",
        "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "RGS QR, fp32 projection + fp64 sketched least squares, P-SRHT sketch",
                   "n": n, "m": m, "k": k, "sketch": "srht", "ls_dtype": "f64",
                   "W": "U diag(logspace(0,-8,m)) V^T, U,V from QR of seeded N(0,1)",
                   "pct_hbm_peak": 100 * value / HBM_PEAK_GBS, "bytes_per_step": B},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(n, m, k),
                     "kernel": "rgs::" + PROJECT_KERNEL,
                     "avg_launch_ms": avg_launch_ms, "avg_launch_bytes": avg_launch_bytes,
                     "copy_ceiling": {"gbs": copy_gbs, "frac_of_peak": copy_gbs / HBM_PEAK_GBS,
                                      "how": "torch copy_ of 1 GiB fp32, (read + write bytes) / time, median of 7"}},
        "quality": {"backward_error": res, "norm2_I_minus_StS": d2, "norm2_I_minus_QtQ": o2},
    }
    if not args.no_extra:
        extra = {}
        # plain fp64 RGS on the same GPU, same sketch
        Q64 = rgs.colmajor(n, m, torch.float64)
        d64 = rgs.qr_desc(n, m, k, sketch="srht", prec="fp64")
        log("plain fp64 RGS, SRHT: 1 warmup, 2 steps")
        ms64, _, rep64 = run_steps(rgs, torch, h, d64, W64, Q64, R, S, 2, 1)
        extra["fp64_rgs_srht"] = {"ms_per_qr": ms64, "gbs": qr_bytes(n, m, 8) / (ms64 / 1000) / 1e9,
                                  "status": rep64.status}
        extra["speedup_fp32_vs_fp64"] = ms64 / ms
        log("  %.2f ms/QR (fp32 path %.2fx faster)" % (ms64, ms64 / ms))
        # plain fp64 CGS2 on the same GPU, for comparison (not part of the library):
        # torch / rocBLAS matrix-vector products, two projections per column
        log("fp64 CGS2 (torch/rocBLAS, comparison): 1 step")
        extra["fp64_cgs2_torch"] = cgs2_fp64(torch, W64, Q64, R)
        log("  %.1f ms/QR (fp32 RGS %.1fx faster), ||W-QR||/||W|| %.2e, ||I-Q^TQ||_2 %.2e" %
            (extra["fp64_cgs2_torch"]["ms_per_qr"], extra["fp64_cgs2_torch"]["ms_per_qr"] / ms,
             extra["fp64_cgs2_torch"]["backward_error"], extra["fp64_cgs2_torch"]["norm2_I_minus_QtQ"]))
        extra["fp64_cgs2_torch"]["fp32_rgs_speedup"] = extra["fp64_cgs2_torch"]["ms_per_qr"] / ms
        del Q64
        # Gaussian sketch, fp32 path (VALU-bound on generation)
        dg = rgs.qr_desc(n, m, k, sketch="gaussian", prec="fp32")
        log("fp32 RGS, Gaussian sketch: 1 warmup, 1 step")
        msg, _, repg = run_steps(rgs, torch, h, dg, W32, Q, R, S, 1, 1)
        gres, gd2, go2 = quality(torch, W32, Q, R, S)
        draws = float(k) * n * (2 * m - 1)
        # VALU bound of the per-column sketches alone: k n entries per column, each
        # drawn and applied in about VALU_INSTR_PER_ENTRY instructions, at the
        # non-packed fp32 issue rate of the chip
        valu_ms = 1000.0 * k * n * m * VALU_INSTR_PER_ENTRY / VALU_LANE_RATE
        extra["fp32_rgs_gaussian"] = {"ms_per_qr": msg, "gbs": B / (msg / 1000) / 1e9, "status": repg.status,
                                      "backward_error": gres, "norm2_I_minus_StS": gd2, "norm2_I_minus_QtQ": go2,
                                      "gaussian_draws_per_s": draws / (msg / 1000),
                                      "valu_roofline": {"bound": "alu", "instr_per_entry": VALU_INSTR_PER_ENTRY,
                                                        "peak_lane_instr_per_s": VALU_LANE_RATE,
                                                        "bound_ms_per_qr": valu_ms, "frac": valu_ms / msg}}
        log("  %.2f ms/QR (VALU bound of the column sketches %.0f ms: %.0f%%), ||W-QR||/||W|| %.2e, "
            "||I-S^TS||_2 %.2e" % (msg, valu_ms, 100 * valu_ms / msg, gres, gd2))
        # Gaussian sketch with bf16 entries, made once into a table and read by every column
        dgt = rgs.qr_desc(n, m, k, sketch="gaussian", prec="fp32", flags=rgs.FLAG_THETA_BF16)
        log("fp32 RGS, Gaussian sketch with bf16 entries (table): 1 warmup, 2 steps")
        msgt, _, repgt = run_steps(rgs, torch, h, dgt, W32, Q, R, S, 2, 1)
        tres, td2, to2 = quality(torch, W32, Q, R, S)
        extra["fp32_rgs_gaussian_bf16_table"] = {"ms_per_qr": msgt, "gbs": B / (msgt / 1000) / 1e9,
                                                 "status": repgt.status, "table_bytes": 2 * k * n,
                                                 "backward_error": tres, "norm2_I_minus_StS": td2,
                                                 "norm2_I_minus_QtQ": to2}
        log("  %.2f ms/QR, ||W-QR||/||W|| %.2e, ||I-S^TS||_2 %.2e" % (msgt, tres, td2))
        # the same Gaussian sketch as the drawn leg, its fp32 entries made once into a table
        dgx = rgs.qr_desc(n, m, k, sketch="gaussian", prec="fp32", flags=rgs.FLAG_THETA_EXACT)
        log("fp32 RGS, Gaussian sketch from its exact fp32 table: 1 warmup, 1 step")
        msgx, _, repgx = run_steps(rgs, torch, h, dgx, W32, Q, R, S, 1, 1)
        xres, xd2, xo2 = quality(torch, W32, Q, R, S)
        extra["fp32_rgs_gaussian_exact_table"] = {"ms_per_qr": msgx, "gbs": B / (msgx / 1000) / 1e9,
                                                  "status": repgx.status, "table_bytes": 4 * k * n,
                                                  "speedup_vs_drawn": msg / msgx,
                                                  "backward_error": xres, "norm2_I_minus_StS": xd2,
                                                  "norm2_I_minus_QtQ": xo2}
        log("  %.2f ms/QR (%.2fx the drawn sketch), ||W-QR||/||W|| %.2e, ||I-S^TS||_2 %.2e" %
            (msgx, msg / msgx, xres, xd2))
        # Rademacher sketch, fp32 path: dense like the Gaussian, 128 signs per Philox call
        dr = rgs.qr_desc(n, m, k, sketch="rademacher", prec="fp32", flags=rgs.FLAG_TIME_KERNELS)
        log("fp32 RGS, Rademacher sketch: 1 warmup, 2 steps")
        msr, kern_r, repr_ = run_steps(rgs, torch, h, dr, W32, Q, R, S, 2, 1)
        rres, rd2, _ = quality(torch, W32, Q, R, S)
        extra["fp32_rgs_rademacher"] = {"ms_per_qr": msr, "gbs": B / (msr / 1000) / 1e9, "status": repr_.status,
                                        "projection_gbs": project_bytes(n, m, 4) / (kern_r / 2 / 1000) / 1e9,
                                        "backward_error": rres, "norm2_I_minus_StS": rd2}
        log("  %.2f ms/QR (%.1f GB/s), projection+sketch kernel %.1f GB/s, ||W-QR||/||W|| %.2e" %
            (msr, B / (msr / 1000) / 1e9, extra["fp32_rgs_rademacher"]["projection_gbs"], rres))
        # step 2 by two Richardson sweeps on the normal equations instead of Householder
        drich = rgs.qr_desc(n, m, k, sketch="srht", prec="fp32", ls_sweeps=2)
        log("fp32 RGS, SRHT, Richardson least squares (2 sweeps): 1 warmup, 2 steps")
        msr2, _, repr2 = run_steps(rgs, torch, h, drich, W32, Q, R, S, 2, 1)
        r2res, r2d2, _ = quality(torch, W32, Q, R, S)
        extra["fp32_rgs_srht_richardson2"] = {"ms_per_qr": msr2, "status": repr2.status, "backward_error": r2res,
                                              "norm2_I_minus_StS": r2d2}
        log("  %.2f ms/QR, ||W-QR||/||W|| %.2e, ||I-S^TS||_2 %.2e" % (msr2, r2res, r2d2))
        # the same factorisation with the a-posteriori certification of Theta (Prop. 3.7)
        dcert = rgs.qr_desc(n, m, k, sketch="srht", prec="fp32", flags=rgs.FLAG_CERTIFY)
        log("fp32 RGS, SRHT, with certification: 1 warmup, 2 steps")
        msc, _, repc = run_steps(rgs, torch, h, dcert, W32, Q, R, S, 2, 1)
        extra["certified_qr_srht"] = {
            "ms_per_qr": msc, "overhead_ms": msc - ms, "status": repc.status,
            "sigma_q": [repc.cert_smin_q, repc.cert_smax_q], "sigma_w": [repc.cert_smin_w, repc.cert_smax_w],
            "omega_bar_q_eps0.05": rgs.rgs_omega_bar(repc.cert_smin_q, repc.cert_smax_q, 0.05),
            "omega_bar_w_eps0.05": rgs.rgs_omega_bar(repc.cert_smin_w, repc.cert_smax_w, 0.05),
            "cond_phi_q": repc.cert_cond_phi_q}
        log("  %.2f ms/QR (+%.2f ms), omega_bar(Q) %.4f, omega_bar(W) %.4f (eps* = 0.05)" %
            (msc, msc - ms, extra["certified_qr_srht"]["omega_bar_q_eps0.05"],
             extra["certified_qr_srht"]["omega_bar_w_eps0.05"]))
        # companion input, sigma 1 -> 1e-3: the 1e-4 gate on ||I - S^T S||_2
        del W64
        Wc64 = synth.svd_matrix_torch(n, m, 1e-3, tag=1, device=dev)
        W32.copy_(Wc64)
        del Wc64
        d1 = rgs.qr_desc(n, m, k, sketch="srht", prec="fp32")
        log("companion sigma->1e-3, fp32/fp64-LS RGS, SRHT: 1 warmup, 2 steps")
        msc32, _, _ = run_steps(rgs, torch, h, d1, W32, Q, R, S, 2, 1)
        cres, cd2, co2 = quality(torch, W32, Q, R, S)
        # the same factorisation in plain fp64 on the same input: the >= 2x claim
        # is measured where the fp32 path passes the ||I - S^T S||_2 <= 1e-4 gate
        Wc64 = synth.svd_matrix_torch(n, m, 1e-3, tag=1, device=dev)
        Q64 = rgs.colmajor(n, m, torch.float64)
        log("companion sigma->1e-3, plain fp64 RGS, SRHT: 1 warmup, 1 step")
        msc64, _, _ = run_steps(rgs, torch, h, d64, Wc64, Q64, R, S, 1, 1)
        c64res, c64d2, _ = quality(torch, Wc64, Q64, R, S)
        del Wc64, Q64
        torch.cuda.empty_cache()
        extra["companion_sigma_1e-3"] = {"backward_error": cres, "norm2_I_minus_StS": cd2,
                                         "norm2_I_minus_QtQ": co2, "ms_per_qr_fp32": msc32,
                                         "ms_per_qr_fp64": msc64, "speedup_fp32_vs_fp64": msc64 / msc32,
                                         "fp64_backward_error": c64res, "fp64_norm2_I_minus_StS": c64d2,
                                         "gate_norm2_I_minus_StS_le_1e-4": cd2 <= 1e-4}
        log("  companion sigma->1e-3: ||W-QR||/||W|| %.2e  ||I-S^TS||_2 %.2e; fp32 %.2f ms, fp64 %.2f ms "
            "(%.2fx)" % (cres, cd2, msc32, msc64, msc64 / msc32))
        out["extra"] = extra
    if not args.no_batched:
        log("plain fp64 RGS, small size (latency-bound)")
        out.setdefault("extra", {})["fp64_rgs_n16384_m64"] = small_fp64_leg(rgs, torch, synth, h)
    if not args.no_gmres:
        out.setdefault("extra", {})["rgmres_convdiff_192"] = gmres_leg(rgs, torch, synth, h)
    if not args.no_extra:
        log("Sec. 5.1 synthetic functions, n = 10^6, m = 300")
        out.setdefault("extra", {})["sec51_functions"] = sec51_leg(rgs, torch, synth, h, classical=False)
    if not args.no_batched:
        log("batched RGS QR (bf16 Q)")
        out["extra"]["batched_qr_2048"] = batched_qr_leg(rgs, torch, synth, h)
        log("batched randomized GMRES")
        out["extra"]["batched_rgmres_256"] = batched_gmres_leg(rgs, torch, synth, h)
    if args.calibrate_copy:
        calibration_copy(torch, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        out["cpu_baseline"] = cpu_baseline()
        log("  %s" % out["cpu_baseline"])
    h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
