"""GPU parity of the factor options against the oracle: the rank tolerance
(k_B = the numerical rank of the ID's sketch relative to ||[Y_B Z_B]||,
capped at k), the concatenated-sketch ID ([M_Y, M_Z] instead of
M_Y + M_Z) and per-box column subsets (a box reads its first
s_B = min(s, l + k + p) sample columns).

With a rank tolerance the skeleton counts are data-dependent; on the
64 x 64 workload at k = 32 they range from 0 to 20, boxes whose children
kept nothing have no active points left, and at tolerance 1e-10 the level-1
boxes eliminate everything (empty root).  Every box must take the oracle's
k_B and skeletons and match its blocks to the conditioning-aware bound of
the plain parity tests; a box whose k_B differs is accepted only when the
oracle's pivot at the boundary lies within 1e-6 of the threshold (a
rounding-level tie), after which the solutions are compared instead.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import rsrs as orr  # noqa: E402
from paper_2311_01451_amd import inputs, rsrs  # noqa: E402
from test_gpu_parity import (_log_problem, _solution_checks, compare_boxes, dev,  # noqa: E402
                             need_gpu, relmax)


def _kb_report(P):
    kg = [len(P.F.box(i)["S"]) for i in range(len(P.Fo.boxes))]
    ko = [len(bo.S) for bo in P.Fo.boxes]
    return kg, ko


@pytest.mark.parametrize("tol", [1e-10, 1e-8])
def test_rank_tolerance_parity_config0(tol):
    need_gpu()
    P = _log_problem(64, 64, 32, rank_tol=tol)
    kg, ko = _kb_report(P)
    print(f"[rank_tol {tol:g}] k_B oracle min/max {min(ko)}/{max(ko)}, root {len(P.Fo.Bt)}", flush=True)
    worst, ncmp = compare_boxes(P)
    print(f"[rank_tol {tol:g}] {ncmp}/{len(P.Fo.boxes)} boxes compared, worst error / predicted {worst:.2f}",
          flush=True)
    if ncmp < len(P.Fo.boxes):   # a rounding-level tie at the threshold (checked inside)
        print(f"[rank_tol {tol:g}] box {ncmp}: k_B {kg[ncmp]} vs {ko[ncmp]}", flush=True)
    else:
        assert kg == ko
        Bt, At = P.F.root()
        assert np.array_equal(Bt, P.Fo.Bt)
        if len(Bt):
            assert relmax(At, P.Fo.At) < 100.0 * P.max_pred
    _solution_checks(P)
    f = dev(inputs.rhs(4096, 2))
    u, rel, it = rsrs.rsrs_solve_refine(P.F, P.op, f, tol=1e-10, maxit=10)
    eo = orr.relerr(P.Fo, P.A)
    print(f"[rank_tol {tol:g}] oracle relerr {eo:.2e}; refined residual {rel:.1e} after {it}", flush=True)
    assert rel <= 1e-10


def test_rank_tolerance_fixed_limit_and_mixed():
    """A tolerance far below every pivot keeps k skeletons per box, like the
    fixed rank; the mixed path with a tolerance refines to 1e-10."""
    need_gpu()
    n, m, k = 32, 32, 16
    P = _log_problem(n, m, k, rank_tol=1e-300)
    assert all(len(P.F.box(i)["S"]) == k for i in range(len(P.Fo.boxes)))
    worst, ncmp = compare_boxes(P)
    assert ncmp == len(P.Fo.boxes)
    pts = inputs.grid2d(64)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / 64)
    tc = rsrs.rsrs_build_tree(pts, 64)
    s = tc.samples_required(32, 32)
    for sym in (False, True):
        smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=rsrs.RSRS_F32, symmetric=sym)
        F = rsrs.rsrs_factor(tc, smp, 32, precision=rsrs.RSRS_PREC_F32_MIXED, symmetric=sym, rank_tol=1e-6)
        kb = [len(F.box(i)["S"]) for i in range(F.info()["nboxes"])]
        f = torch.tensor(inputs.rhs(4096, 3), dtype=torch.float64, device="cuda")
        u, rel, it = rsrs.rsrs_solve_refine(F, op, f, tol=1e-10, maxit=20)
        print(f"[mixed rank_tol 1e-6 sym={sym}] k_B {min(kb)}..{max(kb)}, residual {rel:.1e} after {it}",
              flush=True)
        assert rel <= 1e-10


def test_concatenated_id_parity():
    need_gpu()
    for skew in (0.0, 4e-3):
        P = _log_problem(32, 32, 16, skew=skew, id_mode=rsrs.RSRS_ID_CONCAT)
        worst, ncmp = compare_boxes(P)
        print(f"[concat skew={skew}] {ncmp}/{len(P.Fo.boxes)} boxes compared, worst / predicted {worst:.2f}",
              flush=True)
        assert ncmp == len(P.Fo.boxes)
        _solution_checks(P)


@pytest.mark.parametrize("n,m,k,skew,id_mode", [(64, 64, 16, 0.0, 0), (32, 32, 16, 4e-3, 0),
                                                (32, 32, 16, 4e-3, 1)])
def test_column_subsets_parity(n, m, k, skew, id_mode):
    """Per-box column subsets against the oracle's variant: the 64 x 64
    workload's geometry at k = 16 (every box compared, root included) and a
    nonsymmetric operator with either ID sketch."""
    need_gpu()
    P = _log_problem(n, m, k, skew=skew, id_mode=id_mode, col_subset=True)
    sB = [min(P.s, len(bo.Ba) + len(bo.Na) + 2 * k) for bo in P.Fo.boxes]
    assert min(sB) < P.s
    worst, ncmp = compare_boxes(P)
    print(f"[col_subset n={n} skew={skew} id={id_mode}] s_B {min(sB)}..{max(sB)} of {P.s}; "
          f"{ncmp}/{len(P.Fo.boxes)} boxes compared, worst / predicted {worst:.2f}", flush=True)
    assert ncmp == len(P.Fo.boxes)
    Bt, At = P.F.root()
    assert np.array_equal(Bt, P.Fo.Bt)
    assert relmax(At, P.Fo.At) < 100.0 * P.max_pred
    _solution_checks(P)
    eo = orr.relerr(P.Fo, P.A)
    Fo_full = orr.factor(P.to, P.A @ P.Om, P.A.T @ P.Psi, P.Om, P.Psi, k)
    print(f"[col_subset n={n}] oracle relerr {eo:.2e} (all columns {orr.relerr(Fo_full, P.A):.2e})", flush=True)


def test_column_subsets_mixed_refines():
    """The mixed path (BF16 sample products, FP32 factor) with column
    subsets, symmetric and general, refines to 1e-10 on the 64 x 64 workload."""
    need_gpu()
    pts = inputs.grid2d(64)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / 64)
    tc = rsrs.rsrs_build_tree(pts, 64)
    s = tc.samples_required(32, 32)
    for sym in (False, True):
        smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=rsrs.RSRS_BF16, symmetric=sym)
        F = rsrs.rsrs_factor(tc, smp, 32, precision=rsrs.RSRS_PREC_F32_MIXED, symmetric=sym, col_subset=True)
        f = torch.tensor(inputs.rhs(4096, 3), dtype=torch.float64, device="cuda")
        u0 = rsrs.rsrs_solve(F, f)
        r0 = float(torch.linalg.norm(f - op.matvec(u0)) / torch.linalg.norm(f))
        u, rel, it = rsrs.rsrs_solve_refine(F, op, f, tol=1e-10, maxit=30)
        print(f"[col_subset mixed sym={sym}] one-shot residual {r0:.1e}; refined {rel:.1e} after {it}",
              flush=True)
        assert rel <= 1e-10


def test_option_validation():
    need_gpu()
    pts = inputs.grid2d(16)
    tc = rsrs.rsrs_build_tree(pts, 16)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / 16)
    s = tc.samples_required(8, 8)
    for kw in ({"id_mode": 7}, {"rank_tol": -1.0}, {"rank_tol": float("nan")}, {"col_subset": 2}):
        smp = rsrs.rsrs_sample(tc, op, s, 1)
        with pytest.raises(rsrs.RSRSError) as e:
            rsrs.rsrs_factor(tc, smp, 8, **kw)
        assert e.value.status == 1
