"""Philox4x32-10 and Box-Muller normals (oracle side).

Philox4x32 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of a
multiply-high/low S-box network on a 4-word counter with a 2-word key that is
bumped by the Weyl constants between rounds.  Written here from that
definition in plain Python integers.

The paper draws the random boundary data as i.i.d. standard normals at each
grid point of the buffered patch boundary (randomized reduced-basis approach,
Section 3, and eq. elliptic_random).  Draw (node, sample, patch) uses counter
(node, sample, patch, 0) and key (seed low word, seed high word); the four
output words give two 53-bit uniforms u1, u2 in (0, 1], and the normal is
sqrt(-2 ln u1) cos(2 pi u2).
"""
from __future__ import annotations

import numpy as np

MASK = 0xFFFFFFFF
M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
TWO_PI = 6.283185307179586


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on python ints: returns the 4 output words."""
    c0, c1, c2, c3 = (int(x) & MASK for x in ctr)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox4x32_10_np(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over uint32 counter arrays (same definition, numpy uint64 products)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & MASK)
    k1 = np.uint64(int(k1) & MASK)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    mask = np.uint64(MASK)
    s32 = np.uint64(32)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & mask
            k1 = (k1 + np.uint64(W1)) & mask
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & mask
        hi1, lo1 = p1 >> s32, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform53(x0, x1):
    """(k + 1/2) * 2^-53 with k = (x0 >> 5) * 2^26 + (x1 >> 6); in (0, 1]."""
    x0 = np.asarray(x0, dtype=np.uint64)
    x1 = np.asarray(x1, dtype=np.uint64)
    k = (x0 >> np.uint64(5)) * np.uint64(1 << 26) + (x1 >> np.uint64(6))
    return (k.astype(np.float64) + 0.5) * (2.0 ** -53)


def normals(seed: int, patch: int, n_nodes: int, n_samples: int) -> np.ndarray:
    """Boundary sample matrix Omega (n_nodes x n_samples) of one patch."""
    node = np.arange(n_nodes, dtype=np.uint64)[:, None] * np.ones((1, n_samples), dtype=np.uint64)
    samp = np.ones((n_nodes, 1), dtype=np.uint64) * np.arange(n_samples, dtype=np.uint64)[None, :]
    pat = np.full((n_nodes, n_samples), patch, dtype=np.uint64)
    zero = np.zeros((n_nodes, n_samples), dtype=np.uint64)
    x0, x1, x2, x3 = philox4x32_10_np(node, samp, pat, zero, seed & MASK, (seed >> 32) & MASK)
    u1 = uniform53(x0, x1)
    u2 = uniform53(x2, x3)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(TWO_PI * u2)
