"""Seeded synthetic inputs (geometry, Gaussian test matrices, right-hand sides).

This module holds no arithmetic of the factorization itself: it only draws
random numbers and lays out point sets, so that the CPU reference and the HIP
path can be fed identical inputs.  Gaussian test matrices are standard normal,
as the sketching setting requires (Sec. 4, eq. rand_sample_setting).

Seed convention: base seed 2311_01451; +0 Omega, +1 Psi, +2 right-hand sides,
+3 geometry, +4 coefficient field, +100*i for problem i of a batch.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 2311_01451


def rng(offset: int = 0, base: int = BASE_SEED) -> np.random.Generator:
    return np.random.default_rng(base + offset)


def grid2d(n: int) -> np.ndarray:
    """Cell-centred n x n grid on [0,1]^2, h = 1/n; row i*n+j is ((j+1/2)h, (i+1/2)h)."""
    h = 1.0 / n
    c = (np.arange(n, dtype=np.float64) + 0.5) * h
    yy, xx = np.meshgrid(c, c, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel()], axis=1)


def jittered_grid2d(n: int, seed_offset: int = 3, amp: float = 0.3) -> np.ndarray:
    """Cell-centred grid with each coordinate jittered by U[-amp*h, amp*h]."""
    p = grid2d(n)
    h = 1.0 / n
    j = rng(seed_offset).uniform(-amp * h, amp * h, size=p.shape)
    return p + j


def grid3d_interior(n: int) -> np.ndarray:
    """Interior finite-difference nodes i*h, i=1..n, h = 1/(n+1), x fastest."""
    h = 1.0 / (n + 1)
    c = np.arange(1, n + 1, dtype=np.float64) * h
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)


def uniform_points(n: int, dim: int, seed_offset: int = 3) -> np.ndarray:
    return rng(seed_offset).uniform(0.0, 1.0, size=(n, dim))


def gaussian(nrows: int, ncols: int, seed_offset: int) -> np.ndarray:
    """Standard normal nrows x ncols FP64 matrix (row-major), PCG64 stream."""
    return rng(seed_offset).standard_normal((nrows, ncols))


def test_matrices(n: int, s: int, base_offset: int = 0):
    """(Omega, Psi), each n x s standard normal, in user point order."""
    return gaussian(n, s, base_offset + 0), gaussian(n, s, base_offset + 1)


def rhs(n: int, w: int, base_offset: int = 0) -> np.ndarray:
    return gaussian(n, w, base_offset + 2)


def smooth_log_coefficient(n_nodes: int, seed_offset: int = 4) -> np.ndarray:
    """exp(g) with g iid N(0,1) on an n^3 node grid, box-filtered [1,1,1]/3 per axis
    with edge replication.  Returned array is indexed [z, y, x]."""
    g = rng(seed_offset).standard_normal((n_nodes, n_nodes, n_nodes))
    for ax in range(3):
        gp = np.concatenate([np.take(g, [0], axis=ax), g, np.take(g, [-1], axis=ax)], axis=ax)
        sl = [slice(None)] * 3
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        c = [slice(None)] * 3
        a[ax] = slice(0, -2)
        b[ax] = slice(1, -1)
        c[ax] = slice(2, None)
        g = (gp[tuple(a)] + gp[tuple(b)] + gp[tuple(c)]) / 3.0
        del sl
    return np.exp(g)


def uneven_batch(count: int = 48, n_lo: int = 45, n_hi: int = 181, ranks=(32, 48, 64),
                 seed_offset: int = 7) -> list:
    """The many-problem workload: ``count`` jittered 2D grids with n_i x n_i
    points, n_i^2 log-uniform between n_lo^2 and n_hi^2 (about 2,000 to
    33,000 points), and ranks drawn uniformly from ``ranks``.  Problem i's
    geometry, samples and right-hand sides use seed offsets +100 i (jitter
    at 3 + 100 i).  Returns a list of dicts {i, n, k, geom_seed, seed}."""
    r = rng(seed_offset)
    out = []
    for i in range(count):
        n = int(round(np.exp(r.uniform(np.log(n_lo), np.log(n_hi)))))
        k = int(r.choice(np.asarray(ranks)))
        out.append({"i": i, "n": n, "k": k, "geom_seed": 3 + 100 * i, "seed": 100 * i})
    return out
