"""Philox4x32-10 counter-based random numbers (oracle side).

Definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11, sec. 4.2): the state is a counter of four 32-bit words and
a key of two 32-bit words.  One round maps (c0, c1, c2, c3) to

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

with multipliers M0 = 0xD2511F53, M1 = 0xCD9E8D57.  Ten rounds are applied;
between consecutive rounds the key is advanced by the Weyl constants
(0x9E3779B9, 0xBB67AE85).

The TE-PAI draws use counter = (g_lo, g_hi, s, stream) and key =
(seed_lo, seed_hi), where g is the flat rotation index j*L_eff + k of the
Trotter circuit and s the global sample index; the 64-bit uniform is
(x1 << 32) | x0 of the output words.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

STREAM_GATES = 1


def philox4x32_10(ctr, key):
    """Philox4x32-10 on arrays (or scalars) of uint32 words; returns 4 arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & MASK32 for k in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = c0 * np.uint64(M0)          # < 2^64: exact in uint64
        p1 = c2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def uniform_u64(seed: int, sample, draw, stream: int = STREAM_GATES):
    """The 64-bit uniform for (seed, sample, flat draw index, stream)."""
    draw = np.asarray(draw, dtype=np.uint64)
    sample = np.asarray(sample, dtype=np.uint64)
    ctr = (draw & np.uint64(MASK32), draw >> np.uint64(32),
           sample & np.uint64(MASK32), np.full_like(draw, stream))
    key = (np.uint64(seed & MASK32), np.uint64((seed >> 32) & MASK32))
    x0, x1, _, _ = philox4x32_10(ctr, key)
    return (x1 << np.uint64(32)) | x0
