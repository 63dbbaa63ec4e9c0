"""Counter-based Gaussians for the per-level redraw -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) written from its
published definition: a round maps the counter (c0, c1, c2, c3) with key
(k0, k1) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
M0 = 0xD2511F53, M1 = 0xCD9E8D57, and the key is bumped by the Weyl
constants (0x9E3779B9, 0xBB67AE85) between rounds; ten rounds.  A Gaussian
block entry (i, j) uses counter (i, j, word, seed_hi) and key
(seed_lo, 0x2311); the first two output words give a 53-bit uniform u1, the
last two u2, each (m + 1/2) 2^-53, and the entry is
sqrt(-2 ln u1) cos(2 pi u2) (the Box-Muller transform).
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten rounds on arrays of 32-bit values held in uint64."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3))
    k0, k1 = np.uint64(k0), np.uint64(k1)
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & _MASK,
                          (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & _MASK)
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def gaussian(nrows: int, ncols: int, seed: int, word: int) -> np.ndarray:
    """nrows x ncols standard normal block (FP64) of the generator above."""
    i, j = np.meshgrid(np.arange(nrows, dtype=np.uint64), np.arange(ncols, dtype=np.uint64), indexing="ij")
    hi = np.full(i.shape, (seed >> 32) & 0xFFFFFFFF, dtype=np.uint64)
    w = np.full(i.shape, word & 0xFFFFFFFF, dtype=np.uint64)
    c0, c1, c2, c3 = philox4x32_10(i, j, w, hi, seed & 0xFFFFFFFF, 0x2311)
    m53 = np.uint64((1 << 53) - 1)
    a = ((c0 << np.uint64(21)) ^ (c1 >> np.uint64(11))) & m53
    b = ((c2 << np.uint64(21)) ^ (c3 >> np.uint64(11))) & m53
    u1 = (a.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = (b.astype(np.float64) + 0.5) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
