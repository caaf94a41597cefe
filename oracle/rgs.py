"""Randomized Gram-Schmidt, Algorithm 2 (oracle side; test infrastructure).

The loop below takes the steps of Algorithm 2 (Sec. 2.3) in the paper's order
and notation, one column at a time, with no blocking or fusion:

  1. p_i = Theta w_i                                       (u_fine)
  2. R(1:i-1, i) = argmin_y || S_{i-1} y - p_i ||          (u_fine)
  3. q'_i = w_i - Q_{i-1} R(1:i-1, i)                      (u_crs)
  4. s'_i = Theta q'_i                                     (u_fine)
  5. r_ii = || s'_i ||                                     (u_fine)
  6. s_i  = s'_i / r_ii                                    (u_fine)
  7. q_i  = q'_i / r_ii                                    (u_fine, stored at u_crs)

At i = 1 the least-squares problem is empty, q'_1 = w_1 and s'_1 = p_1 (the
convention stated after Algorithm 2).  Step 4 sketches the computed q'_i and
never uses p_i - S_{i-1} r (the remark after Algorithm 2 says that shortcut
is less stable).

Least-squares solvers for step 2 (Sec. 2.3, the discussion before Alg. 2):
  'householder'  Householder QR of S_{i-1} (LAPACK geqrf through numpy),
                 then a triangular solve -- the solver of the experiments
                 (Sec. 5, first paragraph) and of Theorem 3.3;
  'richardson1'  x = S^T p: one Richardson sweep on the normal equations from
                 x = 0, i.e. classical GS in the sketched inner product;
  'richardson2'  two sweeps, x <- x + S^T (p - S x).

Precision models (Sec. 2.3, the paragraph after Algorithm 2):
  'fp64'  u_crs = u_fine = fp64;
  'fp32'  multi-precision: W and Q stored in float32 and step 3 done in
          float32 arithmetic with float32 accumulation; all other steps fp64.
  'bf16q' as 'fp32', but the basis is stored in bfloat16 (round to nearest
          even).  To keep S the sketch of what is stored, column i is kept
          unnormalised as qb_i = bf16(q'_i) with an fp64 scale 1/r_ii, step 4
          sketches qb_i, and step 3 uses the stored columns with the
          coefficients y_c / r_cc rounded to float32.  The returned Q is
          bf16(qb_i / r_ii).
  'fp32u' unique precision u_crs = u_fine = float32 (the comparison of
          Sec. 5.1): every step in float32 arithmetic -- the sketches of
          steps 1 and 4 (entries rounded to float32 once), the least squares
          of step 2 (LAPACK's float32 Householder QR, sgeqrf, and a float32
          triangular solve),
          steps 3, 5, 6 and 7.  R, S and P are returned as fp64 arrays that
          hold float32 values.

Breakdown (not specified by the paper): a non-finite p_i or s'_i, r_ii = 0,
or r_ii <= 2**-50 ||p_i|| stops the factorisation and reports the column.
"""

import numpy as np
import scipy.linalg

BREAKDOWN_RATIO = 2.0 ** -50


class Breakdown(Exception):
    def __init__(self, column, nonfinite):
        super().__init__("breakdown at column %d%s" % (column, " (non-finite)" if nonfinite else ""))
        self.column = column
        self.nonfinite = nonfinite


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)) << np.uint64(16)
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).reshape(x.shape)


def _ls(S, p, method):
    """Step 2: argmin_y ||S y - p|| for S (k x j), in the arithmetic of the
    operands (fp64, or float32 for the unique-precision model)."""
    if method == "householder":
        if S.dtype == np.float32:   # LAPACK sgeqrf / sorgqr: numpy's qr would work in fp64
            Qs, Rs = scipy.linalg.qr(S, mode="economic")
        else:
            Qs, Rs = np.linalg.qr(S, mode="reduced")
        return scipy.linalg.solve_triangular(Rs, Qs.T @ p, lower=False)
    if method == "richardson1":
        return S.T @ p
    if method == "richardson2":
        x = S.T @ p
        return x + S.T @ (p - S @ x)
    raise ValueError(method)


def rgs_qr(W, theta, ls="householder", precision="fp64"):
    """Algorithm 2 on W (n x m) with sketch ``theta`` (an ``oracle.sketch`` object).

    Returns dict(Q, R, S, P).  Q has the storage type of the precision model
    (fp64, or float32 for 'fp32'); R, S and P are fp64.  Raises Breakdown.
    """
    if precision not in ("fp64", "fp32", "bf16q", "fp32u"):
        raise ValueError(precision)
    store = np.float64 if precision == "fp64" else np.float32
    bf16 = precision == "bf16q"
    # arithmetic of steps 1, 2 and 4-7 (u_fine)
    fine = np.float32 if precision == "fp32u" else np.float64
    W = np.asarray(W).astype(store)
    n, m = W.shape
    k = theta.k
    if not (1 <= m <= k):
        raise ValueError("need 1 <= m <= k")
    Q = np.zeros((n, m), dtype=store)
    Qb = np.zeros((n, m), dtype=np.float32) if bf16 else None   # stored unnormalised columns
    scale = np.zeros(m)
    R = np.zeros((m, m))
    S = np.zeros((k, m))
    P = np.zeros((k, m))
    for i in range(m):                                   # 0-based column index
        w = W[:, i]
        p = theta.apply(w.astype(fine), fine)            # step 1
        P[:, i] = p
        if not np.all(np.isfinite(p)):
            raise Breakdown(i, True)
        if bf16:
            if i == 0:
                qp = w.copy()
            else:
                r = _ls(S[:, :i], p, ls)                 # step 2
                R[:i, i] = r
                qp = w - Qb[:, :i] @ (r * scale[:i]).astype(np.float32)   # step 3 on stored columns
            Qb[:, i] = bf16_round(qp)
            sp = theta.apply(Qb[:, i].astype(np.float64))                 # step 4: sketch of the stored column
        elif i == 0:
            qp = w.copy()                                # q'_1 = w_1
            sp = p.copy()                                # s'_1 = p_1
        else:
            Si = S[:, :i] if fine == np.float64 else S[:, :i].astype(fine)
            r = _ls(Si, p, ls)                           # step 2
            R[:i, i] = r
            qp = w - Q[:, :i] @ r.astype(store)          # step 3 (u_crs)
            sp = theta.apply(qp.astype(fine), fine)      # step 4
        rii = np.linalg.norm(sp)                         # step 5
        if not np.isfinite(rii) or not np.all(np.isfinite(sp)):
            raise Breakdown(i, True)
        if rii == 0.0 or rii <= BREAKDOWN_RATIO * np.linalg.norm(p):
            raise Breakdown(i, False)
        R[i, i] = rii
        S[:, i] = sp / rii                               # step 6
        if bf16:
            scale[i] = 1.0 / rii
            Q[:, i] = bf16_round((Qb[:, i].astype(np.float64) * scale[i]).astype(np.float32))   # step 7
        else:
            Q[:, i] = (qp.astype(fine) / rii).astype(store)   # step 7
    return {"Q": Q, "R": R, "S": S, "P": P}


def rgs_step(Qprev, Sprev, w, theta, ls="householder", precision="fp64"):
    """One column of Algorithm 2 given an existing basis (for sampled checks).

    Qprev (n x j) and Sprev (k x j) are the basis and its sketch so far.
    Returns dict(p, r, qp, sp, rii, s, q).
    """
    store = np.float64 if precision == "fp64" else np.float32
    w = np.asarray(w).astype(store)
    p = theta.apply(w.astype(np.float64))
    j = Qprev.shape[1]
    if j == 0:
        r = np.zeros(0)
        qp = w.copy()
        sp = p.copy()
    else:
        r = _ls(np.asarray(Sprev, dtype=np.float64), p, ls)
        qp = w - np.asarray(Qprev).astype(store) @ r.astype(store)
        sp = theta.apply(qp.astype(np.float64))
    rii = np.linalg.norm(sp)
    return {"p": p, "r": r, "qp": qp, "sp": sp, "rii": rii, "s": sp / rii,
            "q": (qp.astype(np.float64) / rii).astype(store)}


# ----------------------------------------------------------------------------
# Classical projectors of Sec. 1.2 (stability references and pins)
# ----------------------------------------------------------------------------

def cgs(W, dtype=np.float64):
    """Classical Gram-Schmidt: projector I - Q Q^T (Sec. 1.2, first choice)."""
    W = np.asarray(W).astype(dtype)
    n, m = W.shape
    Q = np.zeros((n, m), dtype=dtype)
    R = np.zeros((m, m), dtype=dtype)
    for i in range(m):
        w = W[:, i]
        h = Q[:, :i].T @ w
        qp = w - Q[:, :i] @ h
        R[:i, i] = h
        R[i, i] = np.linalg.norm(qp)
        Q[:, i] = qp / R[i, i]
    return Q, R


def cgs2(W, dtype=np.float64):
    """CGS with one re-orthogonalisation: projector (I - Q Q^T)^2 (Sec. 1.2)."""
    W = np.asarray(W).astype(dtype)
    n, m = W.shape
    Q = np.zeros((n, m), dtype=dtype)
    R = np.zeros((m, m), dtype=dtype)
    for i in range(m):
        w = W[:, i]
        h1 = Q[:, :i].T @ w
        v = w - Q[:, :i] @ h1
        h2 = Q[:, :i].T @ v
        v = v - Q[:, :i] @ h2
        R[:i, i] = h1 + h2
        R[i, i] = np.linalg.norm(v)
        Q[:, i] = v / R[i, i]
    return Q, R


def mgs(W, dtype=np.float64):
    """Modified Gram-Schmidt: product of rank-one projectors (Sec. 1.2)."""
    W = np.asarray(W).astype(dtype)
    n, m = W.shape
    Q = np.zeros((n, m), dtype=dtype)
    R = np.zeros((m, m), dtype=dtype)
    for i in range(m):
        v = W[:, i].copy()
        for c in range(i):
            R[c, i] = Q[:, c] @ v
            v = v - R[c, i] * Q[:, c]
        R[i, i] = np.linalg.norm(v)
        Q[:, i] = v / R[i, i]
    return Q, R
