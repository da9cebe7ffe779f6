"""Counter-based Gaussian generator for the RSVD test matrix (test infrastructure).

Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3" (SC 2011): a 128-bit counter (four 32-bit words) is passed through ten rounds, each
multiplying words 0 and 2 by the constants 0xD2511F53 and 0xCD9E8D57 (64-bit products split in
high and low halves) and mixing the high halves with words 1 and 3 and the key; the 64-bit key
is bumped by the Weyl constants 0x9E3779B9, 0xBB67AE85 between rounds.

Gaussian values, as the device generator defines them: pair p (elements 2p, 2p+1) comes from the
counter (p mod 2^32, p div 2^32, stream, 0) under the key (seed mod 2^32, seed div 2^32); words
0, 1 give the 53-bit integer a = (w0 >> 5) 2^26 + (w1 >> 6) and u1 = (a + 1) 2^-53 in (0, 1];
words 2, 3 likewise give b and u2 = b 2^-53 in [0, 1); then Box-Muller:
sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorized over numpy uint64 arrays holding 32-bit words; returns four such arrays."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3))
    k0 = np.uint64(k0 & MASK)
    k1 = np.uint64(k1 & MASK)
    for _ in range(10):
        p0 = c0 * np.uint64(M0)            # < 2^64: exact in uint64
        p1 = c2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return c0, c1, c2, c3


def philox_scalar(ctr, key):
    """The same rounds on Python integers, one counter at a time (a second, plain rendering)."""
    c = list(ctr)
    k = list(key)
    for _ in range(10):
        a = M0 * c[0]
        b = M1 * c[2]
        c = [((b >> 32) ^ c[1] ^ k[0]) & MASK, b & MASK, ((a >> 32) ^ c[3] ^ k[1]) & MASK, a & MASK]
        k = [(k[0] + W0) & MASK, (k[1] + W1) & MASK]
    return tuple(c)


def gaussian(count, seed, stream=0):
    """count standard normal FP64 values (the device generator's sequence)."""
    npair = (count + 1) // 2
    p = np.arange(npair, dtype=np.uint64)
    w0, w1, w2, w3 = philox4x32_10(p & np.uint64(MASK), p >> np.uint64(32),
                                   np.full(npair, stream, dtype=np.uint64), np.zeros(npair, dtype=np.uint64),
                                   seed & MASK, (seed >> 32) & MASK)
    a = ((w0 >> np.uint64(5)) << np.uint64(26)) | (w1 >> np.uint64(6))
    b = ((w2 >> np.uint64(5)) << np.uint64(26)) | (w3 >> np.uint64(6))
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    rho = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    out = np.empty(2 * npair)
    out[0::2] = rho * np.cos(th)
    out[1::2] = rho * np.sin(th)
    return out[:count]
