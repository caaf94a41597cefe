"""RGS-Arnoldi (Algorithm 3) and randomized GMRES (Sec. 4.2) -- oracle; test infrastructure.

One restart cycle builds the Krylov basis with RGS, Algorithm 2, column by
column: w_1 = r_0 (the current residual; b on the first cycle, since x0 = 0),
then w_i = A q_{i-1}.  The Hessenberg matrix is H = R(1:i, 2:i) (Sec. 4.1),
and y = argmin_z || H z - r_11 e_1 || is solved with Givens rotations in fp64
(Sec. 4.2 and the experiment of Sec. 5.3); x_{i-1} = Q_{i-1} y.  By the
identity of Sec. 4.2, |g_i| after the i-th rotation is the sketched residual
|| Theta (b - A x_{i-1}) ||.

Readings (the paper runs a single unrestarted Arnoldi process):
  * restart after ``restart`` inner steps (restart + 1 basis vectors);
  * cycle c uses a fresh sketch (sketch_id = 2 + c) unless ``reuse_theta``;
  * inner stop when |g_i| / ||b|| <= tol, outer stop on the true residual
    ||b - A x|| / ||b|| <= tol computed in fp64; x is kept in fp64;
  * h_{i,i-1} = r_ii below 2**-50 ||p_i|| is a lucky breakdown: the cycle
    ends with the current H;
  * iteration count = total number of inner steps (mat-vecs A q).
Precision 'fp32' follows the multi-precision model: basis, mat-vec and the
projection in float32, sketches / least squares / Givens / x in fp64.
Precision 'bf16q' is 'fp32' with the basis stored in bfloat16, as in the
'bf16q' model of ``oracle.rgs``: column i is kept unnormalised as
qb_i = bf16(q'_i) with the fp64 scale 1/r_ii, its sketch is taken of qb_i, the
mat-vec input is fl32(qb_{i-1} / r_{i-1,i-1}), the projection uses the stored
columns with coefficients fl32(y_c / r_cc), and x += sum_c qb_c (y_c / r_cc).
Precision 'fp32u' is the configuration of the GMRES experiment of Sec. 5.3:
unique-precision RGS, i.e. every step of Algorithm 2 in float32 (the
sketches, the least squares, the projection, r_ii, s_i and q_i, as the
'fp32u' model of ``oracle.rgs``), while the products with A are computed in
fp64 (from the float32 basis vector, the result rounded once to float32 for
the RGS step) and the Givens rotations, x and the restart residual stay in
fp64.
"""

import numpy as np
import scipy.linalg

from .rgs import _ls, bf16_round, BREAKDOWN_RATIO


def _givens(a, b):
    """c, s, rho with [c s; -s c] [a; b] = [rho; 0]."""
    if b == 0.0:
        return 1.0, 0.0, a
    rho = np.hypot(a, b)
    return a / rho, b / rho, rho


def rgmres(apply_A, b, make_theta, restart, tol, max_iters=100000, precision="fp64",
           ls="householder", reuse_theta=False, max_cycles=None, reverse_projection=False):
    """Restarted randomized GMRES.

    apply_A(u, dtype) -> A u in arithmetic ``dtype``; make_theta(cycle) -> sketch.
    ``reverse_projection`` forms Q_{i-1} r of RGS step 3 over the columns in
    reverse order: the same step with another summation order, which the
    precision models leave open (a second valid rounding of the same model).
    Returns dict(x, hist, iters, cycles, true_relres, converged, Q_last,
    S_last, theta_cycle_last): hist[t] = |g| / ||b|| after global inner step t;
    Q_last holds the last cycle's basis vectors the update used (its first
    ``used`` stored columns, in fp64; unnormalised in the bf16 model), S_last
    their sketches s_i (fp64 array) and theta_cycle_last the argument of
    make_theta for that cycle.
    """
    if precision not in ("fp64", "fp32", "bf16q", "fp32u"):
        raise ValueError(precision)
    store = np.float64 if precision == "fp64" else np.float32
    bf16 = precision == "bf16q"
    unique = precision == "fp32u"
    # arithmetic of the sketches and of RGS steps 2 and 4-7
    fine = np.float32 if unique else np.float64
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    bnorm = np.linalg.norm(b)
    x = np.zeros(n)
    r0 = b.copy()
    hist = []
    iters = 0
    cycle = 0
    converged = False
    true_relres = 1.0
    Q_last, S_last, theta_last = np.zeros((n, 0)), None, None
    while iters < max_iters and (max_cycles is None or cycle < max_cycles):
        theta_last = 0 if reuse_theta else cycle
        theta = make_theta(theta_last)
        k = theta.k
        mmax = restart + 1
        Q = np.zeros((n, mmax), dtype=store)     # bf16q: the stored, unnormalised columns
        scale = np.zeros(mmax)                   # bf16q: 1 / r_ii of each stored column
        S = np.zeros((k, mmax))
        R = np.zeros((mmax, mmax))
        # step 1-2 of Algorithm 3: w_1 = r_0, first RGS iteration
        w = r0.astype(store)
        if bf16:
            Q[:, 0] = bf16_round(w)
            p = theta.apply(Q[:, 0].astype(np.float64))
        else:
            p = theta.apply(w.astype(fine), fine)
        r11 = np.linalg.norm(p)
        if r11 == 0.0:
            converged = True
            break
        R[0, 0] = r11
        S[:, 0] = p / r11
        if bf16:
            scale[0] = 1.0 / r11
        else:
            Q[:, 0] = (w.astype(fine) / r11).astype(store)
        g = np.zeros(mmax)
        g[0] = r11
        cs = np.zeros(mmax)
        sn = np.zeros(mmax)
        used = 0                                    # columns of H (= inner steps)
        for i in range(1, mmax):                    # 0-based index of the new column
            if bf16:
                q_prev = (Q[:, i - 1].astype(np.float64) * scale[i - 1]).astype(store)
            else:
                q_prev = Q[:, i - 1]
            if unique:                              # step 3 of Algorithm 3, in fp64 (Sec. 5.3)
                w = apply_A(q_prev, np.float64).astype(store)
            else:
                w = apply_A(q_prev, store)          # step 3 of Algorithm 3
            p = theta.apply(w.astype(fine), fine)   # RGS step 1
            r = _ls(S[:, :i] if not unique else S[:, :i].astype(fine), p, ls)   # RGS step 2
            R[:i, i] = r
            cols = slice(i - 1, None, -1) if reverse_projection else slice(0, i)
            if bf16:
                qp = w - Q[:, cols] @ (r * scale[:i])[cols].astype(store)   # RGS step 3 on the stored columns
                Q[:, i] = bf16_round(qp)
                sp = theta.apply(Q[:, i].astype(np.float64))        # RGS step 4 of the stored column
            else:
                qp = w - Q[:, cols] @ r[cols].astype(store)     # RGS step 3
                sp = theta.apply(qp.astype(fine), fine)  # RGS step 4
            rii = np.linalg.norm(sp)                # RGS step 5
            lucky = rii == 0.0 or rii <= BREAKDOWN_RATIO * np.linalg.norm(p)
            R[i, i] = 0.0 if lucky else rii
            if not lucky:
                S[:, i] = sp / rii                  # RGS step 6
                if bf16:
                    scale[i] = 1.0 / rii            # RGS step 7, kept as a scale
                else:
                    Q[:, i] = (qp.astype(fine) / rii).astype(store)  # RGS step 7
            # Hessenberg column i-1 (0-based) = R(0:i+1, i); Givens in fp64
            h = R[: i + 1, i].copy()
            for t in range(i - 1):
                a, bb = h[t], h[t + 1]
                h[t] = cs[t] * a + sn[t] * bb
                h[t + 1] = -sn[t] * a + cs[t] * bb
            c, s, rho = _givens(h[i - 1], h[i])
            cs[i - 1], sn[i - 1] = c, s
            h[i - 1], h[i] = rho, 0.0
            R[: i + 1, i] = h                       # keep the rotated column
            g[i] = -s * g[i - 1]
            g[i - 1] = c * g[i - 1]
            used = i
            iters += 1
            hist.append(abs(g[i]) / bnorm)
            if lucky or abs(g[i]) / bnorm <= tol or iters >= max_iters:
                break
        # y = argmin || H z - r11 e1 ||: back substitution on the rotated H
        Hr = R[:used, 1:used + 1]
        y = scipy.linalg.solve_triangular(Hr, g[:used], lower=False)
        if bf16:
            y = y * scale[:used]
        x = x + Q[:, :used].astype(np.float64) @ y
        Q_last = Q[:, :used].astype(np.float64)
        S_last = S[:, :used].copy()
        r0 = b - apply_A(x, np.float64)
        true_relres = np.linalg.norm(r0) / bnorm
        cycle += 1
        if true_relres <= tol:
            converged = True
            break
    return {"x": x, "hist": np.array(hist), "iters": iters, "cycles": cycle,
            "true_relres": true_relres, "converged": converged, "Q_last": Q_last,
            "S_last": S_last, "theta_cycle_last": theta_last}
