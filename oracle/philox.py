"""Philox4x32-10 and the N(2, 1) start vector drawn from it.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Philox4x32 with 10 rounds as published by Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC 2011): per round,
(hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (32 x 32 -> 64-bit products),
c = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0), then the key is bumped by the
Weyl constants before the next round.

The start vector of Algorithm 1 (q ~ N(2, 1)^m) is drawn with counter
(i, 0, 0, 0) and key (seed low 32 bits, seed high 32 bits) for entry i, from
the first two output words x0, x1: u_j = (x_j + 1) 2^-32 in (0, 1], and the
Box-Muller transform g = sqrt(-2 ln u0) cos(2 pi u1); q_i = 2 + g.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: (4, N) uint32-valued, key: (2,) or (2, N). Returns (4, N) uint64 words."""
    c = [np.asarray(x, dtype=np.uint64) & MASK for x in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK
    for r in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [(hi1 ^ c[1] ^ k0) & MASK, lo1, (hi0 ^ c[3] ^ k1) & MASK, lo0]
        if r < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return c


def start_vector(m: int, seed: int, mean: float = 2.0, std: float = 1.0) -> np.ndarray:
    """q_i = mean + std * sqrt(-2 ln u0) cos(2 pi u1) from Philox4x32-10 (float64)."""
    i = np.arange(m, dtype=np.uint64)
    zero = np.zeros(m, dtype=np.uint64)
    seed = int(seed)
    words = philox4x32_10([i & MASK, i >> np.uint64(32), zero, zero],
                          (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    two32 = 4294967296.0
    u0 = (words[0].astype(np.float64) + 1.0) / two32
    u1 = (words[1].astype(np.float64) + 1.0) / two32
    g = np.sqrt(-2.0 * np.log(u0)) * np.cos(6.283185307179586 * u1)
    return mean + std * g
