"""Quantities the paper reports for a factorisation (oracle; test infrastructure).

* Delta_m = ||I - S^T S||_F and tilde Delta_m = ||P - S R||_F / ||P||_F:
  step 8 of Algorithm 2 and the start of Sec. 3.1.
* ||W - Q R||_F / ||W||_F: the backward error of Theorem 3.2.
* cond(Q), cond(S): Corollary 2.2 and the plots of Sec. 5.
* omega = ||I - (Theta V)^T Theta V||_2 for an orthonormal basis V of range(V):
  the smallest epsilon in the definition of an epsilon-embedding (Sec. 2.1).
* omega_bar: the probabilistic upper bound of Prop. 3.7 from two sketches
  (cert_extremes gives the two singular values it is built from).
"""

import numpy as np


def delta_F(S):
    m = S.shape[1]
    return np.linalg.norm(np.eye(m) - S.T @ S, "fro")


def delta_2(S):
    m = S.shape[1]
    return np.linalg.norm(np.eye(m) - S.T @ S, 2)


def delta_tilde_F(P, S, R):
    return np.linalg.norm(P - S @ R, "fro") / np.linalg.norm(P, "fro")


def backward_error(W, Q, R):
    W = np.asarray(W, dtype=np.float64)
    return np.linalg.norm(W - np.asarray(Q, dtype=np.float64) @ R, "fro") / np.linalg.norm(W, "fro")


def cond(A):
    sv = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return sv[0] / sv[-1]


def orth_loss_2(Q):
    Q = np.asarray(Q, dtype=np.float64)
    return np.linalg.norm(np.eye(Q.shape[1]) - Q.T @ Q, 2)


def omega(theta_V, V):
    """Smallest eps for which Theta is an eps-embedding of range(V).

    theta_V = Theta @ V.  With V = U T (U orthonormal, by a QR of V), the
    distortion is ||I - (Theta U)^T (Theta U)||_2 and Theta U = theta_V T^-1.
    """
    V = np.asarray(V, dtype=np.float64)
    _, T = np.linalg.qr(V)
    TU = np.linalg.solve(T.T, np.asarray(theta_V, dtype=np.float64).T).T
    return np.linalg.norm(np.eye(V.shape[1]) - TU.T @ TU, 2)


def cert_extremes(theta_V, phi_V):
    """Extreme singular values (smin, smax) of Theta V X, where X makes Phi V
    orthonormal (Prop. 3.7).  X = T^-1 from a QR  Phi V = U T; any other
    choice gives the same singular values."""
    _, T = np.linalg.qr(np.asarray(phi_V, dtype=np.float64))
    Y = np.linalg.solve(T.T, np.asarray(theta_V, dtype=np.float64).T).T   # Theta V T^-1
    sv = np.linalg.svd(Y, compute_uv=False)
    return float(sv[-1]), float(sv[0])


def omega_bar_from(smin, smax, eps_star):
    """Prop. 3.7: max(1 - (1-eps*) smin^2, (1+eps*) smax^2 - 1)."""
    return max(1.0 - (1.0 - eps_star) * smin ** 2, (1.0 + eps_star) * smax ** 2 - 1.0)


def omega_bar(theta_V, phi_V, eps_star):
    """Prop. 3.7: the a-posteriori bound on the embedding distortion of Theta
    for range(V) from the sketches Theta V and Phi V (Phi independent of V)."""
    return omega_bar_from(*cert_extremes(theta_V, phi_V), eps_star)
