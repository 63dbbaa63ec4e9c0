"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and the host tree / neighbour / schedule code is bit-identical
to the oracle's (Sec. 3 readings; Algorithm 1 box order)."""
import os
import re

import numpy as np
import pytest

from oracle import tree as ot
from paper_2311_01451_amd import inputs, rsrs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "rsrs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(rsrs_[a-z0-9_]+)\s*\(", src))
    return sorted(n for n in names if not n.endswith("_fn"))


def test_library_exports_every_declared_symbol():
    L = rsrs.lib()
    declared = header_functions()
    assert "rsrs_factor" in declared and "rsrs_solve" in declared
    for name in declared:
        assert hasattr(L, name), name
    assert set(rsrs.EXPORTS) == set(declared)


def _compare(pts, m, k, lo=None, side=1.0):
    to = ot.build_tree(pts, m, lo=lo, side=side)
    tc = rsrs.rsrs_build_tree(pts, m, root_lo=lo, root_side=side)
    ci = tc.info()
    for key in ("level", "coords", "parent", "is_leaf", "pt_begin", "pt_end", "perm"):
        assert np.array_equal(ci[key], getattr(to, key)), key
    assert ci["nlevels"] == to.nlevels
    for lev in range(1, to.nlevels + 1):
        a, b = ot.neighbours(to, lev), tc.neighbours(lev)
        assert set(a) == set(b)
        for x in a:
            assert np.array_equal(a[x], b[x])
    sch = ot.schedule(to, k)
    col, bc, lc, rc = tc.schedule(k)
    assert np.array_equal(sch.colour, col)
    assert np.array_equal(sch.b_count, bc)
    assert np.array_equal(sch.l_count, lc)
    assert rc == sch.root_count
    assert tc.samples_required(k, k) == ot.samples_required(to, k, k)


def test_tree_bit_exact_uniform_2d():
    _compare(inputs.grid2d(64), 64, 32)
    _compare(inputs.grid2d(256), 64, 64)


def test_tree_bit_exact_adaptive_2d():
    rng = np.random.default_rng(5)
    pts = np.concatenate([rng.uniform(0, 1, (3000, 2)), 0.5 + 0.01 * rng.standard_normal((3000, 2))])
    _compare(np.clip(pts, 0, 0.999999), 12, 6)


def test_tree_bit_exact_3d():
    _compare(inputs.uniform_points(32768, 3), 64, 128, lo=[0, 0, 0])
    h = 1.0 / 49
    _compare(inputs.grid3d_interior(48), 64, 96, lo=[h / 2] * 3, side=64 * h)


def test_paper_sample_counts_native():
    """Experiment 1 sample counts (1520 at k=40, 2280 at k=60) from the C++ code."""
    for n, k in ((284, 40), (401, 60)):
        t = rsrs.rsrs_build_tree(inputs.grid2d(n), 4 * k)
        assert t.samples_required(k, k) == 37 * k + k


def test_invalid_arguments_are_reported():
    with pytest.raises(rsrs.RSRSError) as e:
        rsrs.rsrs_build_tree(np.zeros((4, 2)), 0)
    assert e.value.status == 1
    with pytest.raises(rsrs.RSRSError):
        rsrs.rsrs_build_tree(np.full((4, 2), np.nan), 4)


@pytest.mark.parametrize("symmetric", [0, 1])
def test_work_model_native_equals_oracle(symmetric):
    """rsrs_work_model (the algorithmic counts behind the benchmark's
    TFLOP/s figures) equals the oracle's work model (cost terms of Sec. 4.5)
    on the 64^2 and 256^2 grids and an adaptive 3D tree."""
    from oracle import flops as ofl
    cases = [(inputs.grid2d(64), 64, 32, None), (inputs.grid2d(256), 64, 64, None),
             (inputs.uniform_points(4096, 3), 64, 32, [0, 0, 0])]
    for pts, m, k, lo in cases:
        to = ot.build_tree(pts, m, lo=lo)
        tc = rsrs.rsrs_build_tree(pts, m, root_lo=lo)
        s = tc.samples_required(k, k)
        for esize, cs in ((8, False), (4, False), (8, True)):
            w = rsrs.rsrs_work_model(tc, k, s, bool(symmetric), esize, col_subset=cs)
            o = ofl.factor_work(to, k, s, symmetric=bool(symmetric), esize=esize, col_subset=cs)
            assert abs(w["flops"] - o.flops) <= 1e-12 * o.flops
            assert abs(w["bytes"] - o.bytes_moved) <= 1e-12 * o.bytes_moved
            assert w["stored_entries"] == o.stored_entries
        # column subsets price fewer flops whenever some box has l + k + p < s
        full = ofl.factor_work(to, k, s, symmetric=bool(symmetric))
        sub = ofl.factor_work(to, k, s, symmetric=bool(symmetric), col_subset=True)
        assert sub.flops < full.flops and sub.stored_entries == full.stored_entries
