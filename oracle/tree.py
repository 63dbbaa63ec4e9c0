"""Hierarchical partition of the points (Sec. 3, opening paragraphs) -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper fixes the tree only in words: the root box holds all points, a box
is split into 2^d children while it holds more than ``m`` points, adaptive
trees are 2:1 balanced, boxes are adjacent when they share a face, edge or
corner, and the active set shrinks as redundant indices are eliminated
(eq. active, BNactive).  The readings taken here:

* Root box: the cube [lo, lo+side)^d given by the caller.  Coordinates are
  quantized to Q=20 bits per axis, q = clamp(floor(((x-lo)/side) * 2^Q)),
  evaluated in IEEE FP64 in exactly that order; a box at level l owns the
  points whose q >> (Q-l) equals its integer coordinates, so a point on a
  split plane belongs to the upper child.  Empty children are never created.
* 2:1 balance: repeatedly split every leaf whose closed box touches a leaf two
  or more levels finer, until no leaf does.
* Box ids: boxes sorted by (level, Morton code of their coordinates), Morton
  code interleaving axis 0 into the lowest bit.  Points are renumbered into
  "tree order": leaves in Morton order of their first fine cell, points inside
  a leaf by ascending user index; every box then owns a contiguous range.
* Neighbours at level l: the level-l boxes and the leaves of coarser levels
  (together they partition the active points while level l is processed)
  whose closed box meets the closed box of B, B excluded, sorted by box id.
* Box order inside a level (the paper leaves it open and runs boxes one after
  another): boxes whose closed neighbourhoods {B} u N(B) are disjoint touch
  disjoint rows of Y, Z, Omega, Psi, so their updates commute exactly.  The
  processed boxes of a level are coloured greedily, visiting them by
  (sum_a (c_a mod 3) 3^a, box id) and giving each the smallest colour not held
  by a box whose closed neighbourhood meets its own; colours run in ascending
  order, boxes inside a colour by box id.
* A box is processed (compressed) when its active count b exceeds k; otherwise
  every one of its points stays active (fixed rank k, k_B = min(k, b)).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

QBITS = 20


def quantize(points: np.ndarray, lo, side: float, qbits: int = QBITS) -> np.ndarray:
    """Integer cell coordinates at the finest level (see module docstring)."""
    pts = np.asarray(points, dtype=np.float64)
    d = pts.shape[1]
    lo = np.asarray(lo, dtype=np.float64)[:d]
    scale = float(2 ** qbits)
    t = (pts - lo[None, :]) / float(side)
    t = t * scale
    q = np.floor(t)
    q = np.clip(q, 0.0, scale - 1.0)
    return q.astype(np.int64)


def morton(coords: np.ndarray, d: int, nbits: int = QBITS) -> np.ndarray:
    """Bit-interleaved code of integer coordinates, axis 0 in the lowest bit."""
    c = np.asarray(coords, dtype=np.int64).reshape(-1, d)
    code = np.zeros(c.shape[0], dtype=np.int64)
    for bit in range(nbits):
        for a in range(d):
            code |= ((c[:, a] >> bit) & 1) << (bit * d + a)
    return code


@dataclass
class Tree:
    dim: int
    leaf_size: int
    qbits: int
    n: int
    level: np.ndarray        # [nbox]
    coords: np.ndarray       # [nbox, dim]
    parent: np.ndarray       # [nbox], -1 for the root
    children: list           # list of sorted child-id arrays
    is_leaf: np.ndarray      # [nbox] bool
    pt_begin: np.ndarray     # [nbox] tree-order range
    pt_end: np.ndarray
    perm: np.ndarray         # [n] tree position -> user index
    nlevels: int             # depth L (max level)
    level_boxes: list = field(default_factory=list)   # box ids per level

    @property
    def nbox(self) -> int:
        return int(self.level.shape[0])

    def box_lo_hi(self, b: int):
        """Closed extent of box b in finest-level integer units."""
        w = 1 << (self.qbits - int(self.level[b]))
        lo = self.coords[b] * w
        return lo, lo + w


def _split(q: np.ndarray, pts_idx: np.ndarray, level: int, qbits: int):
    """Non-empty children of a box at ``level`` holding user points ``pts_idx``."""
    sub = q[pts_idx] >> (qbits - level - 1)
    keys, inv = np.unique(sub, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    out = []
    for i in range(keys.shape[0]):
        out.append((tuple(int(v) for v in keys[i]), pts_idx[inv == i]))
    return out


def _adjacent(lo1, hi1, lo2, hi2) -> bool:
    return bool(np.all(lo1 <= hi2) and np.all(lo2 <= hi1))


def build_tree(points, leaf_size: int, lo=None, side: float = 1.0,
               qbits: int = QBITS) -> Tree:
    """Adaptive 2:1-balanced tree over ``points`` (N x d), Sec. 3."""
    pts = np.asarray(points, dtype=np.float64)
    n, d = pts.shape
    if d not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if lo is None:
        lo = np.zeros(d)
    q = quantize(pts, lo, side, qbits)

    # boxes: dict (level, coords) -> user point indices; children known by key
    boxes = {(0, (0,) * d): np.arange(n, dtype=np.int64)}
    split = set()
    frontier = [(0, (0,) * d)]
    while frontier:
        nxt = []
        for key in frontier:
            lev, c = key
            idx = boxes[key]
            if idx.shape[0] > leaf_size and lev < qbits:
                split.add(key)
                for cc, cidx in _split(q, idx, lev, qbits):
                    ck = (lev + 1, cc)
                    boxes[ck] = cidx
                    nxt.append(ck)
        frontier = nxt

    # 2:1 balance
    def extent(key):
        lev, c = key
        w = 1 << (qbits - lev)
        lo_ = np.array(c, dtype=np.int64) * w
        return lo_, lo_ + w

    while True:
        leaves = [k for k in boxes if k not in split]
        if not leaves:
            break
        lev = np.array([k[0] for k in leaves], dtype=np.int64)
        ext = [extent(k) for k in leaves]
        los = np.stack([e[0] for e in ext])
        his = np.stack([e[1] for e in ext])
        marked = []
        for i, key in enumerate(leaves):
            finer = lev >= lev[i] + 2
            if not finer.any():
                continue
            touch = np.all(los[finer] <= his[i][None, :], axis=1) & \
                np.all(los[i][None, :] <= his[finer], axis=1)
            if touch.any() and key[0] < qbits:
                marked.append(key)
        if not marked:
            break
        for key in marked:
            split.add(key)
            for cc, cidx in _split(q, boxes[key], key[0], qbits):
                boxes[(key[0] + 1, cc)] = cidx

    keys = list(boxes.keys())
    levs = np.array([k[0] for k in keys], dtype=np.int64)
    crd = np.array([k[1] for k in keys], dtype=np.int64).reshape(-1, d)
    mc = morton(crd, d, qbits)
    order = np.lexsort((mc, levs))
    keys = [keys[i] for i in order]
    levs = levs[order]
    crd = crd[order]
    idmap = {k: i for i, k in enumerate(keys)}
    nbox = len(keys)
    parent = np.full(nbox, -1, dtype=np.int64)
    children = [[] for _ in range(nbox)]
    for i, (lev, c) in enumerate(keys):
        if lev > 0:
            pk = (lev - 1, tuple(v >> 1 for v in c))
            parent[i] = idmap[pk]
            children[idmap[pk]].append(i)
    children = [np.array(sorted(ch), dtype=np.int64) for ch in children]
    is_leaf = np.array([k not in split for k in keys])

    # tree order of points: leaves by Morton code of their first fine cell
    leaf_ids = np.nonzero(is_leaf)[0]
    fine_key = np.array([int(mc[order][i]) << (d * (qbits - int(levs[i]))) for i in leaf_ids],
                        dtype=np.int64)
    leaf_sorted = leaf_ids[np.argsort(fine_key, kind="stable")]
    perm_parts = []
    pt_begin = np.zeros(nbox, dtype=np.int64)
    pt_end = np.zeros(nbox, dtype=np.int64)
    pos = 0
    for b in leaf_sorted:
        idx = np.sort(boxes[keys[b]])
        pt_begin[b] = pos
        pos += idx.shape[0]
        pt_end[b] = pos
        perm_parts.append(idx)
    perm = np.concatenate(perm_parts) if perm_parts else np.zeros(0, dtype=np.int64)
    # ranges of tree boxes: union of their children (children are contiguous)
    for b in range(nbox - 1, -1, -1):
        if not is_leaf[b]:
            ch = children[b]
            pt_begin[b] = pt_begin[ch].min()
            pt_end[b] = pt_end[ch].max()
    L = int(levs.max()) if nbox else 0
    level_boxes = [np.nonzero(levs == lv)[0] for lv in range(L + 1)]
    return Tree(dim=d, leaf_size=leaf_size, qbits=qbits, n=n, level=levs, coords=crd,
                parent=parent, children=children, is_leaf=is_leaf, pt_begin=pt_begin,
                pt_end=pt_end, perm=perm, nlevels=L, level_boxes=level_boxes)


def representatives(tree: Tree, lev: int) -> np.ndarray:
    """Boxes that partition the active points while level ``lev`` is processed:
    the level-``lev`` boxes and the leaves of coarser levels."""
    sel = (tree.level == lev) | (tree.is_leaf & (tree.level < lev))
    return np.nonzero(sel)[0]


def neighbours(tree: Tree, lev: int) -> dict:
    """N(B) for every level-``lev`` box B: adjacent representatives, by box id."""
    reps = representatives(tree, lev)
    w = np.array([1 << (tree.qbits - int(tree.level[r])) for r in reps], dtype=np.int64)
    los = tree.coords[reps] * w[:, None]
    his = los + w[:, None]
    out = {}
    for b in tree.level_boxes[lev] if lev < len(tree.level_boxes) else []:
        lo, hi = tree.box_lo_hi(int(b))
        touch = np.all(los <= hi[None, :], axis=1) & np.all(lo[None, :] <= his, axis=1)
        nb = reps[touch]
        out[int(b)] = np.sort(nb[nb != b])
    return out


@dataclass
class Schedule:
    """Box order and the active-count model for a given rank k."""
    k: int
    order: list              # per level L..1: list of colour classes (lists of box ids)
    colour: np.ndarray       # [nbox], -1 when not processed
    processed: np.ndarray    # [nbox] bool
    nbrs: dict               # level -> {box: neighbour ids}
    b_count: np.ndarray      # active count of each box when its level is processed
    l_count: np.ndarray      # b + n at processing time (0 if not processed)
    root_count: int
    levels: list             # processed order of levels (L..1)


def schedule(tree: Tree, k: int) -> Schedule:
    """Colour-major box order and active counts for fixed rank k (Algorithm 1,
    eq. BNactive; count model of Sec. 4.5 with the order fixed here)."""
    nbox = tree.nbox
    remaining = np.zeros(nbox, dtype=np.int64)      # active count after own level
    b_count = np.zeros(nbox, dtype=np.int64)
    l_count = np.zeros(nbox, dtype=np.int64)
    colour = np.full(nbox, -1, dtype=np.int64)
    processed = np.zeros(nbox, dtype=bool)
    order = []
    nbrs_all = {}
    levels = list(range(tree.nlevels, 0, -1))
    for lev in levels:
        boxes = tree.level_boxes[lev]
        for b in boxes:
            if tree.is_leaf[b]:
                b_count[b] = tree.pt_end[b] - tree.pt_begin[b]
            else:
                b_count[b] = remaining[tree.children[b]].sum()
        nb = neighbours(tree, lev)
        nbrs_all[lev] = nb
        proc = [int(b) for b in boxes if b_count[b] > k]
        for b in boxes:
            processed[b] = b_count[b] > k
        # greedy colouring of the processed boxes
        closed = {b: set(nb[b].tolist()) | {b} for b in proc}
        pat = []
        for b in proc:
            c = tree.coords[b]
            pat.append(int(sum(int(c[a] % 3) * 3 ** a for a in range(tree.dim))))
        visit = sorted(range(len(proc)), key=lambda i: (pat[i], proc[i]))
        ncol = 0
        coloured = []
        for i in visit:
            b = proc[i]
            used = set()
            for b2 in coloured:
                if closed[b] & closed[b2]:
                    used.add(int(colour[b2]))
            c = 0
            while c in used:
                c += 1
            colour[b] = c
            ncol = max(ncol, c + 1)
            coloured.append(b)
        classes = [sorted(b for b in proc if colour[b] == c) for c in range(ncol)]
        # active count of representatives while this level runs
        act = {}
        for r in representatives(tree, lev):
            r = int(r)
            if tree.level[r] == lev:
                act[r] = int(b_count[r])
            else:
                act[r] = int(tree.pt_end[r] - tree.pt_begin[r])
        for cls in classes:
            for b in cls:
                l_count[b] = b_count[b] + sum(act[x] for x in nb[b].tolist())
            for b in cls:
                act[b] = k
        for b in boxes:
            remaining[b] = k if processed[b] else b_count[b]
        order.append(classes)
    # root: active points left after level 1 (or everything when L = 0)
    if tree.nlevels == 0:
        root_count = tree.n
    else:
        root_count = int(sum(remaining[b] for b in tree.level_boxes[1]))
        root_count += int(sum(tree.pt_end[b] - tree.pt_begin[b]
                              for b in range(nbox) if tree.is_leaf[b] and tree.level[b] == 0))
    return Schedule(k=k, order=order, colour=colour, processed=processed, nbrs=nbrs_all,
                    b_count=b_count, l_count=l_count, root_count=root_count, levels=levels)


def samples_required(tree: Tree, k: int, p: int) -> int:
    """Smallest s for which every null space of Algorithm 1 has k+p columns
    (eq. s_L, s_B; the non-uniform count of Sec. 4.5) and the root extraction
    has a right inverse: max(max_B (|B_a|+|N_a|) + k + p, |B_t|)."""
    sch = schedule(tree, k)
    lmax = int(sch.l_count.max()) if sch.processed.any() else 0
    need = lmax + k + p if sch.processed.any() else 0
    return int(max(need, sch.root_count))
