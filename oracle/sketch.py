"""Sketching operators Theta (k x n) of Sec. 2.1 (oracle side; test infrastructure).

The paper relies on oblivious l2-subspace embeddings drawn from a seeded
generator (Sec. 2.1): Gaussian / Rademacher matrices and the (partial)
subsampled randomized Hadamard transform, P-SRHT.  It fixes the
distributions and scalings but not the bit-level layout; the readings taken
here (counter layout, uniform-to-normal transform, sign and row draws) are
listed in the design notes and are shared, as definitions, with the device
library, which implements them on its own.

Gaussian (Sec. 2.1; entries N(0, 1/k)):
    theta[j, l] = z(j, l) / sqrt(k), where z comes from one Philox4x32-10
    call at counter (floor(l/4), j, sketch_id, instance), key = seed, and
    Box-Muller on the word pairs (x0, x1) -> l%4 in {0, 1}, (x2, x3) ->
    l%4 in {2, 3}:  u1 = ((x_a >> 9) + 1/2) * 2**-23,  u2 = (x_b >> 8) * 2**-24
    (both exactly representable in float32 and fp64),
    rho = sqrt(-2 ln u1),  z_a = rho cos(2 pi u2),  z_b = rho sin(2 pi u2).

Gaussian with bf16 entries (a stored variant of the Gaussian sketch):
    theta[j, l] = bf16(z(j, l)) / sqrt(k), z as above in fp64, rounded once
    to the nearest bfloat16 (ties to even).  Still an i.i.d. sketch whose
    entries differ from the N(0, 1/k) ones by at most 2**-8 relative.

Rademacher (Sec. 2.1; entries +-1/sqrt(k) with equal probability):
    theta[j, l] = -1/sqrt(k) iff bit (l % 32) of word ((l % 128) // 32) of
    Philox(floor(l/128), j, sketch_id, instance) is set, else +1/sqrt(k)
    (one Philox call gives the signs of 128 consecutive columns of a row).

P-SRHT (Sec. 2.1): with s = 2**ceil(log2 n), n <= s < 2n,
    Theta = k**-1/2 * Rows_rho * H_s * D, restricted to its first n columns
    (equivalently: zero-pad x to length s).  H_s is the unnormalised
    Walsh-Hadamard matrix in Sylvester order, H[a, b] = (-1)**popcount(a & b).
    D = diag(d):  d_l = -1 iff bit (l % 32) of word ((l % 128) // 32) of
    Philox(floor(l/128), 0xFFFFFFFF, sketch_id, instance) is set.
    rho: k distinct rows of [0, s) drawn by a partial Fisher-Yates shuffle;
    draw t uses Philox(t, 0xFFFFFFFE, sketch_id, instance) and swaps position
    t with t + floor((x1 * 2**32 + x0) * (s - t) / 2**64); rows are kept in
    draw order.

Identity (test sketch): k = n, Theta = I.  With it RGS reduces to Gram-Schmidt.
"""

import math

import numpy as np

from .philox import philox4x32, seed_key

TAG_SIGNS = 0xFFFFFFFF
TAG_ROWS = 0xFFFFFFFE


# ----------------------------------------------------------------------------
# Gaussian
# ----------------------------------------------------------------------------

def gaussian_block(k, seed, sketch_id, instance, j0, j1, l0, l1):
    """Entries theta[j0:j1, l0:l1] of the Gaussian sketch, fp64."""
    key = seed_key(seed)
    js = np.arange(j0, j1, dtype=np.uint64)
    b0, b1 = l0 // 4, (l1 + 3) // 4
    blocks = np.arange(b0, b1, dtype=np.uint64)
    ctr = np.empty((js.size, blocks.size, 4), dtype=np.uint64)
    ctr[..., 0] = blocks[None, :]
    ctr[..., 1] = js[:, None]
    ctr[..., 2] = sketch_id
    ctr[..., 3] = instance
    x = philox4x32(ctr, key).astype(np.uint64)            # (J, B, 4)
    u1a = ((x[..., 0] >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23
    u2a = (x[..., 1] >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    u1b = ((x[..., 2] >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23
    u2b = (x[..., 3] >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    ra = np.sqrt(-2.0 * np.log(u1a))
    rb = np.sqrt(-2.0 * np.log(u1b))
    z = np.empty((js.size, blocks.size, 4), dtype=np.float64)
    z[..., 0] = ra * np.cos(2.0 * np.pi * u2a)
    z[..., 1] = ra * np.sin(2.0 * np.pi * u2a)
    z[..., 2] = rb * np.cos(2.0 * np.pi * u2b)
    z[..., 3] = rb * np.sin(2.0 * np.pi * u2b)
    z = z.reshape(js.size, -1)
    off = l0 - 4 * b0
    return z[:, off:off + (l1 - l0)] / math.sqrt(k)


def bf16_round_f64(x):
    """Round fp64 values to the nearest bfloat16 (ties to even) in one step,
    returned as fp64.  Finite values within the float32 normal range."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    u = x.view(np.uint64)
    # bfloat16 keeps 7 of the 52 fraction bits: round at bit 45
    lsb = (u >> np.uint64(45)) & np.uint64(1)
    r = ((u + np.uint64((1 << 44) - 1) + lsb) >> np.uint64(45)) << np.uint64(45)
    return r.view(np.float64).reshape(x.shape)


def gaussian_bf16_block(k, seed, sketch_id, instance, j0, j1, l0, l1):
    """Entries theta[j0:j1, l0:l1] of the Gaussian sketch with bf16 entries."""
    z = gaussian_block(1, seed, sketch_id, instance, j0, j1, l0, l1)   # k = 1: z itself, unscaled
    return bf16_round_f64(z) / math.sqrt(k)


# ----------------------------------------------------------------------------
# Rademacher
# ----------------------------------------------------------------------------

def rademacher_block(k, seed, sketch_id, instance, j0, j1, l0, l1):
    """Entries theta[j0:j1, l0:l1] of the Rademacher sketch, fp64."""
    key = seed_key(seed)
    js = np.arange(j0, j1, dtype=np.uint64)
    b0, b1 = l0 // 128, (l1 + 127) // 128
    blocks = np.arange(b0, b1, dtype=np.uint64)
    ctr = np.empty((js.size, blocks.size, 4), dtype=np.uint64)
    ctr[..., 0] = blocks[None, :]
    ctr[..., 1] = js[:, None]
    ctr[..., 2] = sketch_id
    ctr[..., 3] = instance
    words = philox4x32(ctr, key).astype(np.uint64)        # (J, B, 4)
    l = np.arange(l0, l1, dtype=np.uint64)
    w = words[:, (l // np.uint64(128) - np.uint64(b0)).astype(np.int64),
              ((l % np.uint64(128)) // np.uint64(32)).astype(np.int64)]
    bit = (w >> (l % np.uint64(32))[None, :]) & np.uint64(1)
    return np.where(bit == 1, -1.0, 1.0) / math.sqrt(k)


# ----------------------------------------------------------------------------
# SRHT pieces
# ----------------------------------------------------------------------------

def srht_size(n):
    """s = 2**ceil(log2 n): the padded Hadamard order of P-SRHT."""
    s = 1
    while s < n:
        s *= 2
    return s


def srht_signs(n, seed, sketch_id, instance):
    """The diagonal d of D (entries +-1, fp64) for rows 0..n-1."""
    key = seed_key(seed)
    nblk = (n + 127) // 128
    ctr = np.zeros((nblk, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nblk, dtype=np.uint64)
    ctr[:, 1] = TAG_SIGNS
    ctr[:, 2] = sketch_id
    ctr[:, 3] = instance
    words = philox4x32(ctr, key).reshape(-1).astype(np.uint64)   # 4 words / block
    l = np.arange(n, dtype=np.uint64)
    w = words[(l // np.uint64(128)) * np.uint64(4) + (l % np.uint64(128)) // np.uint64(32)]
    bit = (w >> (l % np.uint64(32))) & np.uint64(1)
    return np.where(bit == 1, -1.0, 1.0)


def srht_rows(s, k, seed, sketch_id, instance):
    """k distinct row indices of H_s drawn by a partial Fisher-Yates shuffle."""
    if k > s:
        raise ValueError("SRHT needs k <= s")
    key = seed_key(seed)
    ctr = np.zeros((k, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(k, dtype=np.uint64)
    ctr[:, 1] = TAG_ROWS
    ctr[:, 2] = sketch_id
    ctr[:, 3] = instance
    x = philox4x32(ctr, key)
    perm = {}                                   # sparse view of the shuffled array
    rows = np.empty(k, dtype=np.int64)
    for t in range(k):
        r64 = (int(x[t, 1]) << 32) | int(x[t, 0])
        idx = t + ((r64 * (s - t)) >> 64)
        a_t = perm.get(t, t)
        a_idx = perm.get(idx, idx)
        perm[t], perm[idx] = a_idx, a_t
        rows[t] = a_idx
    return rows


def fwht(x, dtype=np.float64):
    """Unnormalised Walsh-Hadamard transform in Sylvester order along axis 0.

    x: array of shape (s, ...) with s a power of two.  Returns H_s @ x,
    every butterfly computed in arithmetic ``dtype``.
    """
    y = np.array(x, dtype=dtype, copy=True)
    s = y.shape[0]
    if s & (s - 1):
        raise ValueError("length must be a power of two")
    h = 1
    while h < s:
        y = y.reshape((s // (2 * h), 2, h) + y.shape[1:])
        a = y[:, 0].copy()
        b = y[:, 1].copy()
        y[:, 0] = a + b
        y[:, 1] = a - b
        y = y.reshape((s,) + y.shape[3:])
        h *= 2
    return y


# ----------------------------------------------------------------------------
# Operator objects
# ----------------------------------------------------------------------------

class Sketch:
    """Common interface: ``apply(X, dtype)`` returns Theta @ X computed in
    arithmetic ``dtype`` (fp64 by default; float32 for the unique-precision
    model, where the entries are rounded to float32 once and every product
    and sum is a float32 operation)."""

    kind = None

    def __init__(self, n, k, seed=42, sketch_id=0, instance=0):
        self.n, self.k = int(n), int(k)
        self.seed, self.sketch_id, self.instance = int(seed), int(sketch_id), int(instance)

    def materialize(self, j0=0, j1=None, l0=0, l1=None):
        """Dense block Theta[j0:j1, l0:l1] (fp64)."""
        raise NotImplementedError

    def apply(self, X, dtype=np.float64):
        raise NotImplementedError


class Gaussian(Sketch):
    """Gaussian sketch, entries N(0, 1/k), generated block by block."""

    kind = "gaussian"
    BLOCK = 4096

    def __init__(self, n, k, seed=42, sketch_id=0, instance=0, cache_limit=2 ** 26):
        super().__init__(n, k, seed, sketch_id, instance)
        self._dense = None
        if self.k * self.n <= cache_limit:
            self._dense = self.materialize()

    def materialize(self, j0=0, j1=None, l0=0, l1=None):
        j1 = self.k if j1 is None else j1
        l1 = self.n if l1 is None else l1
        return gaussian_block(self.k, self.seed, self.sketch_id, self.instance, j0, j1, l0, l1)

    def apply(self, X, dtype=np.float64):
        X = np.asarray(X, dtype=dtype)
        vec = X.ndim == 1
        X2 = X.reshape(self.n, -1)
        if self._dense is not None:
            Y = self._dense.astype(dtype) @ X2
        else:
            Y = np.zeros((self.k, X2.shape[1]), dtype=dtype)
            for l0 in range(0, self.n, self.BLOCK):
                l1 = min(self.n, l0 + self.BLOCK)
                Y += self.materialize(0, self.k, l0, l1).astype(dtype) @ X2[l0:l1]
        return Y[:, 0] if vec else Y


class GaussianBF16(Gaussian):
    """Gaussian sketch with entries rounded to bfloat16."""

    kind = "gaussian_bf16"

    def materialize(self, j0=0, j1=None, l0=0, l1=None):
        j1 = self.k if j1 is None else j1
        l1 = self.n if l1 is None else l1
        return gaussian_bf16_block(self.k, self.seed, self.sketch_id, self.instance, j0, j1, l0, l1)


class Rademacher(Gaussian):
    """Rademacher sketch, entries +-1/sqrt(k), generated block by block."""

    kind = "rademacher"

    def materialize(self, j0=0, j1=None, l0=0, l1=None):
        j1 = self.k if j1 is None else j1
        l1 = self.n if l1 is None else l1
        return rademacher_block(self.k, self.seed, self.sketch_id, self.instance, j0, j1, l0, l1)


class SRHT(Sketch):
    """P-SRHT: k**-1/2 * Rows_rho * H_s * D on the zero-padded input."""

    kind = "srht"

    def __init__(self, n, k, seed=42, sketch_id=0, instance=0):
        super().__init__(n, k, seed, sketch_id, instance)
        self.s = srht_size(self.n)
        if self.k > self.s:
            raise ValueError("SRHT needs k <= s")
        self.d = srht_signs(self.n, seed, sketch_id, instance)
        self.rows = srht_rows(self.s, self.k, seed, sketch_id, instance)

    def apply(self, X, dtype=np.float64):
        X = np.asarray(X, dtype=dtype)
        vec = X.ndim == 1
        X2 = X.reshape(self.n, -1)
        pad = np.zeros((self.s, X2.shape[1]), dtype=dtype)
        pad[: self.n] = self.d.astype(dtype)[:, None] * X2      # sign flips: exact
        if dtype == np.float64:
            Y = fwht(pad)[self.rows] / math.sqrt(self.k)
        else:   # k**-1/2 rounded to the arithmetic type once, then one product per entry
            Y = fwht(pad, dtype)[self.rows] * dtype(1.0 / math.sqrt(self.k))
        return Y[:, 0] if vec else Y

    def materialize(self, j0=0, j1=None, l0=0, l1=None):
        j1 = self.k if j1 is None else j1
        l1 = self.n if l1 is None else l1
        r = self.rows[j0:j1][:, None]
        l = np.arange(l0, l1)[None, :]
        par = np.vectorize(lambda v: bin(int(v)).count("1") & 1)(r & l)
        return np.where(par == 1, -1.0, 1.0) * self.d[l0:l1][None, :] / math.sqrt(self.k)


class Identity(Sketch):
    """Theta = I (k = n): the test sketch under which RGS is Gram-Schmidt."""

    kind = "identity"

    def __init__(self, n, k=None, seed=0, sketch_id=0, instance=0):
        super().__init__(n, n if k is None else k, seed, sketch_id, instance)
        if self.k != self.n:
            raise ValueError("identity sketch needs k = n")

    def apply(self, X, dtype=np.float64):
        return np.array(X, dtype=dtype, copy=True)

    def materialize(self, j0=0, j1=None, l0=0, l1=None):
        j1 = self.k if j1 is None else j1
        l1 = self.n if l1 is None else l1
        return np.eye(self.k, self.n)[j0:j1, l0:l1]


def make(kind, n, k, seed=42, sketch_id=0, instance=0):
    """Factory by name: 'gaussian', 'gaussian_bf16', 'rademacher', 'srht' or 'identity'."""
    if kind == "gaussian":
        return Gaussian(n, k, seed, sketch_id, instance)
    if kind == "rademacher":
        return Rademacher(n, k, seed, sketch_id, instance)
    if kind == "gaussian_bf16":
        return GaussianBF16(n, k, seed, sketch_id, instance)
    if kind == "srht":
        return SRHT(n, k, seed, sketch_id, instance)
    if kind == "identity":
        return Identity(n, k, seed, sketch_id, instance)
    raise ValueError(kind)
