"""Synthetic black-box operators as explicit matrices -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

RSRS only ever sees these operators through products with A and A^T
(Sec. 4, eq. rand_sample_setting).  The oracle forms them explicitly (dense
NumPy arrays, or SciPy sparse for the 7-point operator) so that sketches,
residuals and error norms can be computed plainly.  Entries follow the
workloads used for measurement:

* ``log2d``: 2D Laplace-kernel volume operator on a grid with spacing h,
  A_ij = delta_ij + h^2 * (-log|x_i - x_j| / (2 pi)) for i != j and
  A_ii = 1 + h^2/2 (the kernel family of Sec. 3 and Experiment 1, with the
  diagonal fixed by the workload rather than by quadrature).
* ``inv_r3d``: A_ij = delta_ij + N^{-1} / (4 pi |x_i - x_j|), A_ii = 1.
* ``poisson7``: -div(a grad u) on interior FD nodes, 7-point stencil, face
  coefficient = mean of the two node values, Dirichlet nodes eliminated.
* ``log2d_skew``: ``log2d`` plus eps * (x_i - x_j)_0 / |x_i - x_j|^2, an
  antisymmetric part, so that A != A^T.
* ``log2d_first``: the first-kind log kernel of Experiment 1 on a cell-centred
  grid: A_ij = h^2 (-log|x_i - x_j| / (2 pi)) with no identity term, and the
  diagonal the average of the kernel over the point's own cell,
  A_ii = h^2 (-log h - c_sq) / (2 pi), c_sq = (1/h^2) int_cell log|y| dy / h
  (the mean of log|u| over the unit square centred at 0):
  c_sq = (log 2 - 3 + pi/2) / 2 - log 2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _pairwise(points: np.ndarray):
    p = np.asarray(points, dtype=np.float64)
    diff = p[:, None, :] - p[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=2))
    return diff, r


def log2d(points: np.ndarray, h: float) -> np.ndarray:
    _, r = _pairwise(points)
    n = r.shape[0]
    with np.errstate(divide="ignore"):
        a = (h * h) * (-np.log(r) / (2.0 * np.pi))
    a[np.arange(n), np.arange(n)] = 0.0
    a += np.eye(n)
    a[np.arange(n), np.arange(n)] = 1.0 + 0.5 * h * h
    return a


def log2d_skew(points: np.ndarray, h: float, eps: float) -> np.ndarray:
    diff, r = _pairwise(points)
    n = r.shape[0]
    a = log2d(points, h)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = diff[:, :, 0] / (r * r)
    s[np.arange(n), np.arange(n)] = 0.0
    return a + eps * s


LOG_MEAN_UNIT_SQUARE = 0.5 * (np.log(2.0) - 3.0 + 0.5 * np.pi) - np.log(2.0)


def log2d_first(points: np.ndarray, h: float) -> np.ndarray:
    _, r = _pairwise(points)
    n = r.shape[0]
    with np.errstate(divide="ignore"):
        a = (h * h) * (-np.log(r) / (2.0 * np.pi))
    a[np.arange(n), np.arange(n)] = (h * h) * (-np.log(h) - LOG_MEAN_UNIT_SQUARE) / (2.0 * np.pi)
    return a


def inv_r3d(points: np.ndarray) -> np.ndarray:
    _, r = _pairwise(points)
    n = r.shape[0]
    with np.errstate(divide="ignore"):
        a = (1.0 / n) / (4.0 * np.pi * r)
    a[np.arange(n), np.arange(n)] = 1.0
    return a


def poisson7(n: int, coef_nodes: np.ndarray) -> sp.csr_matrix:
    """7-point -div(a grad u) on the n^3 interior nodes of a grid with h=1/(n+1).

    ``coef_nodes`` is a on all (n+2)^3 nodes including the boundary, indexed
    [z, y, x].  Unknowns are ordered x fastest (as ``inputs.grid3d_interior``).
    """
    h = 1.0 / (n + 1)
    a = np.asarray(coef_nodes, dtype=np.float64)
    assert a.shape == (n + 2, n + 2, n + 2)
    idx = np.arange(n ** 3).reshape(n, n, n)   # [z, y, x] of interior nodes
    rows, cols, vals = [], [], []
    diag = np.zeros((n, n, n))
    inner = a[1:-1, 1:-1, 1:-1]
    for axis in range(3):
        for sgn in (-1, 1):
            sl = [slice(1, -1)] * 3
            sl[axis] = slice(1 + sgn, n + 1 + sgn)
            nb = a[tuple(sl)]
            face = 0.5 * (inner + nb) / (h * h)
            diag += face
            # off-diagonal coupling to interior neighbours only
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if sgn < 0:
                src[axis] = slice(1, n)
                dst[axis] = slice(0, n - 1)
            else:
                src[axis] = slice(0, n - 1)
                dst[axis] = slice(1, n)
            rows.append(idx[tuple(src)].ravel())
            cols.append(idx[tuple(dst)].ravel())
            vals.append(-face[tuple(src)].ravel())
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    m = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n ** 3, n ** 3))
    return m.tocsr()
