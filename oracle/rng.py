"""Counter-based random numbers for the path-tracing oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC 2011), restated from its published definition: a 128-bit counter
and a 64-bit key; each of the 10 rounds multiplies counter words 0 and 2 by the
constants M0 and M1 into 64-bit products, and the new counter is

    (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0));

the key is bumped by the Weyl constants W0, W1 before every round but the first.
A 32-bit output x maps to the uniform ((x >> 9) + 1/2) 2^-23 in (0, 1): its
numerator 2 (x >> 9) + 1 has at most 24 bits, so the value is exact in FP32 and
FP64 alike and both implementations draw identical numbers.
"""

from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32(ctr, key, rounds=10):
    """ctr (..., 4), key (..., 2): 32-bit words in any integer dtype -> (..., 4) uint64 words."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i].copy() for i in range(4))
    k0, k1 = key[..., 0].copy(), key[..., 1].copy()
    m0, m1, mask = np.uint64(M0), np.uint64(M1), np.uint64(MASK)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & mask
            k1 = (k1 + np.uint64(W1)) & mask
        p0 = m0 * c0
        p1 = m1 * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & mask, (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & mask)
    return np.stack([c0, c1, c2, c3], axis=-1)


def uniforms(words):
    """32-bit words -> uniforms ((x >> 9) + 1/2) 2^-23 in (0, 1), FP64 (exactly FP32 values)."""
    w = np.asarray(words, dtype=np.uint64)
    return ((w >> np.uint64(9)).astype(np.float64) + 0.5) * (2.0 ** -23)
