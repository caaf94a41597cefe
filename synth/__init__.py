"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the method: it only draws inputs.  The
sketch's own random numbers are NOT drawn here; each side regenerates them
from the counter-based generator definition.

Recipes (the paper's datasets are not available; these stand in for them):

* ``svd_matrix``: W = U diag(sigma) V^T, U = qr(G_{n x m}).Q and
  V = qr(G_{m x m}).Q with G ~ N(0, 1), sigma log-spaced from 1 to sigma_min --
  a matrix of prescribed conditioning, the role played by the snapshot
  matrices of Sec. 5.
* ``f_mu_matrix``: the synthetic functions of Sec. 5.1,
  W[i, j] = sin(10 (mu_j + x_i)) / (cos(100 (mu_j - x_i)) + 1.1) on evenly
  spaced x in [0, 1] and mu in [0, 1], endpoints included.
* ``convdiff_coeffs``: -Lap u + v.grad u on the unit cube, v = Pe (1, 1, 1),
  Dirichlet 0, h = 1/(N+1), central differences, rows scaled by h^2:
  diagonal 6, x/y/z neighbours -1 -+ Pe h / 2 (minus side / plus side).
* ``rhs``: b ~ N(0, 1).
* ``batch_sizes``: per-instance (n, m) or (N, Pe) draws for batched runs.

Data RNG: numpy PCG64 seeded from SeedSequence(ROOT_ENTROPY) with a
per-purpose spawn key, so every input is reproducible on any host.
"""

import numpy as np

ROOT_ENTROPY = 20201110
SKETCH_SEED = 42

_PURPOSE = {"U": 0, "V": 1, "b": 2, "sizes": 3, "misc": 4}


def rng(purpose, *extra):
    key = (_PURPOSE[purpose],) + tuple(int(e) for e in extra)
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_ENTROPY, spawn_key=key)))


def svd_matrix(n, m, sigma_min, tag=0, dtype=np.float64):
    """W = U diag(logspace(0, log10 sigma_min, m)) V^T (fp64 construction, cast at the end)."""
    G = rng("U", n, m, tag).standard_normal((n, m))
    U, _ = np.linalg.qr(G)
    del G
    H = rng("V", m, tag).standard_normal((m, m))
    V, _ = np.linalg.qr(H)
    sigma = np.logspace(0.0, np.log10(sigma_min), m)
    W = (U * sigma[None, :]) @ V.T
    return W.astype(dtype)


def f_mu_matrix(n, m, dtype=np.float64):
    x = np.linspace(0.0, 1.0, n)[:, None]
    mu = np.linspace(0.0, 1.0, m)[None, :]
    W = np.sin(10.0 * (mu + x)) / (np.cos(100.0 * (mu - x)) + 1.1)
    return W.astype(dtype)


def convdiff_coeffs(N, Pe):
    """(dims, coeffs) of the h^2-scaled 7-point convection-diffusion stencil."""
    h = 1.0 / (N + 1)
    a = Pe * h / 2.0
    return (N, N, N), (6.0, -1.0 - a, -1.0 + a, -1.0 - a, -1.0 + a, -1.0 - a, -1.0 + a)


def rhs(n, tag=0):
    return rng("b", n, tag).standard_normal(n)


def batch_qr_sizes(batch, n_lo=4096, n_hi=262144, m_lo=16, m_hi=128, tag=0):
    g = rng("sizes", batch, tag)
    ns = g.integers(n_lo, n_hi + 1, size=batch)
    ms = g.integers(m_lo, m_hi + 1, size=batch)
    return ns, ms


def batch_gmres_sizes(batch, N_lo=32, N_hi=96, pe_lo=1.0, pe_hi=100.0, tag=0):
    g = rng("sizes", batch, tag, 1)
    Ns = g.integers(N_lo, N_hi + 1, size=batch)
    Pes = g.uniform(pe_lo, pe_hi, size=batch)
    return Ns, Pes


def svd_matrix_torch(n, m, sigma_min, tag=0, device="cuda"):
    """Device-side draw of the same recipe as ``svd_matrix`` for sizes a host QR
    would take minutes on (fp64, column-major (n, m) tensor).  Uses torch's
    seeded device generator, so its values differ from ``svd_matrix``'s.
    The Q factor of the tall Gaussian G is formed by Cholesky QR
    (G^T G = C^T C, U = G C^-1): the same positive-diagonal QR factor, accurate
    to rounding because a tall Gaussian matrix is well conditioned.  Only
    matrix products run on the device; the m x m factorisations run on the host."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(ROOT_ENTROPY * 1000 + int(tag))
    G = torch.randn((n, m), generator=gen, dtype=torch.float64, device=device)
    gram = (G.T @ G).cpu().numpy()
    C = np.linalg.cholesky(gram).T                       # gram = C^T C, C upper
    Cinv = np.linalg.inv(C)
    U = G @ torch.from_numpy(Cinv).to(device)
    del G
    V, _ = np.linalg.qr(rng("V", m, tag).standard_normal((m, m)))
    sigma = np.logspace(0.0, np.log10(sigma_min), m)
    SVt = torch.from_numpy(np.ascontiguousarray((sigma[:, None] * V.T))).to(device)
    W = U @ SVt
    del U
    return W.t().contiguous().t()          # column-major copy
