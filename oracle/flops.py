"""Algorithmic work model of one factorization -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The flop and byte counts of the method itself, box by box, as the cost
analysis of Sec. 4.5 prices each step of Algorithm 1 (dense N^3 work avoided;
counts in the plain LAPACK-style operations the oracle performs).  For a box
with b = |B_a|, n = |N_a|, l = b + n, k_B = min(k, b), r = b - k_B and s
samples, the general (two-sided) step costs

  2 (4 s l^2 - 4/3 l^3)   thin QR with Q of the two s x l test-matrix panels
  8 b s l                 the two projections Y_B Q Q^T, Z_B Q Q^T
  4 s b k                 column-pivoted QR of the b x s sketch, k steps
  8 r k s                 sparsification of Y, Z, Omega, Psi
  4 r s l                 the two extractions (reusing Q)
  2/3 r^3                 LU of X_RR
  4 r^2 (k + n)           the multipliers K_U, K_L
  8 r (k + n) s           elimination of Y, Z, Omega, Psi

and moves (element size e bytes) e s (2l + 2b + 2n) read, e s (4b + 2n)
written and e (r k + r^2 + 2 r (k + n)) stored.  With per-box column
subsets the QR, projection, ID and extraction terms and the 2l + 2b read
panels count s_B = min(s, l + k + p) columns instead of s.  The symmetric variant keeps
one sketch side: every two-sided term is halved except the ID and the LU.
The root costs a thin QR with Q of the s x |B_t| panel, the product with Y,
a triangular solve and an LU.  Solves cost 2 flops per stored entry and
right-hand side; one batch reads every stored entry once.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import tree as otree


@dataclass
class BoxWork:
    b: int
    n: int
    k: int
    r: int
    flops: float
    bytes_moved: float
    stored: int


def box_work(b: int, n: int, k: int, s: int, symmetric: bool = False, esize: int = 8,
             sB: int | None = None) -> BoxWork:
    """Work of one processed box (cost terms of Sec. 4.5 for the steps of
    Algorithm 1); see the module docstring for the terms.  ``sB``: the
    columns the box's nullification, ID and extraction use (default s)."""
    kb = min(k, b)
    r = b - kb
    l = b + n
    h = 0.5 if symmetric else 1.0
    c = s if sB is None else sB
    f = (h * 2.0 * (4.0 * c * l * l - (4.0 / 3.0) * l ** 3)
         + h * 8.0 * b * c * l
         + 4.0 * c * b * kb
         + h * 8.0 * r * kb * s
         + h * 4.0 * r * c * l
         + (2.0 / 3.0) * r ** 3
         + h * 4.0 * r * r * (kb + n)
         + h * 8.0 * r * (kb + n) * s)
    stored = r * kb + r * r + (1 if symmetric else 2) * r * (kb + n)
    moved = (h * esize * (c * (2 * l + 2 * b) + s * 2 * n)
             + h * esize * s * (4 * b + 2 * n)
             + esize * stored)
    return BoxWork(b=b, n=n, k=kb, r=r, flops=f, bytes_moved=moved, stored=stored)


def root_work(nt: int, s: int) -> float:
    """Root of Algorithm 1: A_t = Y_Bt pinv(Omega_Bt) by a thin QR with Q of
    the s x nt panel, the product Y_Bt Q, a triangular solve with nt right
    sides, then an LU."""
    return (4.0 * s * nt * nt - (4.0 / 3.0) * nt ** 3) + 2.0 * s * nt * nt + nt ** 3 + (2.0 / 3.0) * nt ** 3


@dataclass
class FactorWork:
    boxes: list            # BoxWork in processing order
    root: int
    flops: float           # boxes + root
    bytes_moved: float
    stored_entries: int    # boxes + root block


def factor_work(tree: otree.Tree, k: int, s: int, symmetric: bool = False,
                esize: int = 8, col_subset: bool = False, p: int | None = None) -> FactorWork:
    """Work of a fixed-rank factorization of ``tree`` with s samples: every
    processed box of the schedule (active counts from the count model of
    Sec. 4.5 under the box order of ``oracle.tree.schedule``) plus the root
    (which uses all s columns).  ``col_subset``: boxes use s_B = min(s, l +
    k + p) columns (p defaults to k), as ``oracle.rsrs.factor`` does."""
    if p is None:
        p = k
    sch = otree.schedule(tree, k)
    out = []
    for classes in sch.order:
        for cls in classes:
            for bx in cls:
                b = int(sch.b_count[bx])
                n = int(sch.l_count[bx]) - b
                sB = min(s, int(sch.l_count[bx]) + k + p) if col_subset else s
                out.append(box_work(b, n, k, s, symmetric, esize, sB))
    nt = int(sch.root_count)
    flops = sum(w.flops for w in out) + root_work(nt, s)
    stored = sum(w.stored for w in out) + nt * nt
    moved = sum(w.bytes_moved for w in out) + esize * (2 * nt * s + nt * nt)
    return FactorWork(boxes=out, root=nt, flops=flops, bytes_moved=moved, stored_entries=stored)


def solve_work(fw: FactorWork, nrhs: int, esize: int = 8):
    """(flops, bytes) of one solve of nrhs columns: 2 flops per stored entry
    and column; every stored entry read once per batch (eq. Ainvfact)."""
    return 2.0 * fw.stored_entries * nrhs, float(esize * fw.stored_entries)
