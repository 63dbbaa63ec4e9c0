"""GPU: the GEMM tile autotuner.

The table is measured once (196 launch classes), written to a cache file and
loaded back from it without timing anything.  Every tile shape accumulates
each output entry over the same K slices in the same order, so factorizations
and solves must be bit for bit the same whichever shape the launches take:
checked by forcing each shape in turn, and with the measured table, against
the built-in rule, in FP64 (general variant) and on the mixed path
(symmetric variant).
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2311_01451_amd import inputs, rsrs  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _factor_and_solve(mixed):
    n, k = 64, 32
    pts = inputs.grid2d(n)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
    tc = rsrs.rsrs_build_tree(pts, 64)
    s = tc.samples_required(k, k)
    if mixed:
        smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=rsrs.RSRS_F32, symmetric=True)
        F = rsrs.rsrs_factor(tc, smp, k, precision=rsrs.RSRS_PREC_F32_MIXED, symmetric=True)
    else:
        smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=rsrs.RSRS_F64)
        F = rsrs.rsrs_factor(tc, smp, k)
    f = torch.tensor(inputs.rhs(n * n, 16), dtype=torch.float64, device="cuda")
    u = F.solve(f).cpu().numpy()
    blocks = [F.box(i) for i in range(F.info()["nboxes"])]
    return blocks, u


def _same(a, b):
    ba, ua = a
    bb, ub = b
    assert len(ba) == len(bb)
    for x, y in zip(ba, bb):
        for key in ("S", "R", "T", "XRR", "KU", "KL"):
            assert np.array_equal(x[key], y[key]), key
    assert np.array_equal(ua, ub)


def test_autotune_table_and_cache(tmp_path):
    need_gpu()
    path = str(tmp_path / "tiles.txt")
    a = time.perf_counter()
    r1 = rsrs.rsrs_gemm_autotune(path)
    t1 = time.perf_counter() - a
    lines = [x for x in open(path) if not x.startswith("#")]
    assert r1["classes"] == 196 and len(lines) == 196
    shapes = [int(x.split()[4]) for x in lines]
    assert set(shapes) <= {0, 1, 2}
    a = time.perf_counter()
    r2 = rsrs.rsrs_gemm_autotune(path)
    t2 = time.perf_counter() - a
    print(f"[autotune] measured in {t1:.2f} s, loaded in {t2 * 1e3:.1f} ms; "
          f"{r1['changed']} of {r1['classes']} classes differ from the built-in rule; "
          f"shape counts {[shapes.count(v) for v in (0, 1, 2)]}", flush=True)
    assert r2 == r1
    rsrs.rsrs_gemm_tile_override(-2)


@pytest.mark.parametrize("mixed", [False, True])
def test_tile_shapes_do_not_change_results(mixed, tmp_path):
    need_gpu()
    rsrs.rsrs_gemm_tile_override(-2)
    ref = _factor_and_solve(mixed)
    try:
        for shp in (0, 1, 2):
            rsrs.rsrs_gemm_tile_override(shp)
            _same(ref, _factor_and_solve(mixed))
            print(f"[autotune] mixed={mixed}: shape {shp} gives the same factor and solution bit for bit",
                  flush=True)
        rsrs.rsrs_gemm_tile_override(-1)
        rsrs.rsrs_gemm_autotune(str(tmp_path / "tiles.txt"))
        _same(ref, _factor_and_solve(mixed))
    finally:
        rsrs.rsrs_gemm_tile_override(-2)
    with pytest.raises(rsrs.RSRSError) as e:
        rsrs.rsrs_gemm_tile_override(3)
    assert e.value.status == 1


def test_workload_tuning_keeps_results():
    """Tuning on the workload itself (the factorization of the 64 x 64 grid at
    k = 32 run under each tile shape, every launch timed by its shape
    signature): the tuned factorization is bit for bit the untuned one."""
    need_gpu()
    rsrs.rsrs_gemm_tile_override(-2)
    try:
        for mixed in (False, True):
            ref = _factor_and_solve(mixed)
            tc = rsrs.rsrs_build_tree(inputs.grid2d(64), 64)
            s = tc.samples_required(32, 32)
            prec = rsrs.RSRS_PREC_F32_MIXED if mixed else rsrs.RSRS_PREC_F64
            a = time.perf_counter()
            r = rsrs.rsrs_gemm_autotune_workload(tc, 32, s, precision=prec, symmetric=mixed)
            print(f"[autotune workload] mixed={mixed}: {r['signatures']} signatures, {r['changed']} moved, "
                  f"{time.perf_counter() - a:.2f} s", flush=True)
            assert r["signatures"] > 0
            _same(ref, _factor_and_solve(mixed))
    finally:
        rsrs.rsrs_gemm_tile_override(-2)
