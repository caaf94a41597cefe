"""Philox4x32-10 counter-based generator (oracle side; test infrastructure).

The paper only asks for "a seeded random number generator" so that any block
of the sketching matrix can be regenerated without storage or communication
(Sec. 2.1, the paragraph on Rademacher and (P-)SRHT matrices; Sec. 2.4 on
distributed architectures).  The generator chosen for that role is Philox4x32
with 10 rounds, defined in J. Salmon, M. Moraes, R. Dror, D. Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11, Sec. 3:

* state: a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1),
  all 32-bit words;
* one round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (full 64-bit
  products), then the new counter is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
* multipliers M0 = 0xD2511F53, M1 = 0xCD9E8D57;
* the key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between
  rounds, so round r (0-based) uses key + r * Weyl.

Pinned against an independent implementation (rocRAND's header engine built
for the host) in ``tests/test_oracle_philox.py``.
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
ROUNDS = 10


def philox4x32(counter, key, rounds=ROUNDS):
    """Apply Philox4x32-``rounds`` to an array of counters.

    counter: integer array of shape (..., 4) holding 32-bit words (c0..c3).
    key:     pair (k0, k1) of 32-bit words, or an array of shape (..., 2).
    Returns a uint32 array of shape (..., 4).
    """
    c = np.asarray(counter, dtype=np.uint64) & MASK32
    k = np.asarray(key, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0 = k[..., 0]
    k1 = k[..., 1]
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & MASK32
            k1 = (k1 + np.uint64(W1)) & MASK32
        p0 = M0 * c0          # exact: both factors < 2**32
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    out = np.stack([c0, c1, c2, c3], axis=-1)
    return out.astype(np.uint32)


def seed_key(seed):
    """Split a 64-bit seed into the Philox key (low word, high word)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)
