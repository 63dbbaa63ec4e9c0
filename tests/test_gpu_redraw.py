"""GPU: per-level redrawing of the samples (rsrs_factor_redraw) against the
oracle's redraw.

Both sides draw every Gaussian block from Philox-4x32-10 (the GPU's
generator, and the oracle's own implementation of the published
definition): the first samples in user order with words 0 and 1, the r-th
redraw in tree order with words 2r and 2r + 1.  The GPU computes its
Gaussians with device log/cos, the oracle with NumPy's, so the two sides'
inputs agree to rounding and every block is compared with the
conditioning-aware tolerance of the plain parity tests.  The mixed path with
redraws must refine to 1e-10.
"""
from types import SimpleNamespace

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import operators as oop  # noqa: E402
from oracle import philox  # noqa: E402
from oracle import rsrs as orr  # noqa: E402
from oracle import tree as ot  # noqa: E402
from paper_2311_01451_amd import inputs, rsrs  # noqa: E402
from test_gpu_parity import _solution_checks, compare_boxes, dev, need_gpu  # noqa: E402

SEED = 0x5EED_0000_2311


@pytest.mark.parametrize("n,m,k,skew,symmetric", [(32, 32, 12, 0.0, True), (32, 32, 12, 4e-3, False),
                                                  (64, 64, 16, 0.0, True)])
def test_redraw_parity_with_oracle(n, m, k, skew, symmetric):
    need_gpu()
    pts = inputs.grid2d(n)
    N = n * n
    kind = rsrs.RSRS_OP_LOG2D if skew == 0.0 else rsrs.RSRS_OP_LOG2D_SKEW
    A = oop.log2d(pts, 1.0 / n) if skew == 0.0 else oop.log2d_skew(pts, 1.0 / n, skew)
    op = rsrs.rsrs_op_create_kernel(kind, pts, 1.0 / n, skew)
    tc = rsrs.rsrs_build_tree(pts, m)
    s = tc.samples_required(k, k)
    print(f"[redraw] N={N} k={k} skew={skew} symmetric={symmetric} s={s}", flush=True)
    F = rsrs.rsrs_factor_redraw(tc, op, s, SEED, k, symmetric=symmetric)
    Om = philox.gaussian(N, s, SEED, 0)
    rd = {"matvec": lambda X: A @ X, "rmatvec": lambda X: A.T @ X, "seed": SEED}
    if symmetric:
        Fo = orr.factor(ot.build_tree(pts, m), A @ Om, None, Om, None, k, symmetric=True, redraw=rd)
    else:
        Psi = philox.gaussian(N, s, SEED, 1)
        Fo = orr.factor(ot.build_tree(pts, m), A @ Om, A.T @ Psi, Om, Psi, k, redraw=rd)
    levels = sorted({bo.level for bo in Fo.boxes})
    assert len(levels) >= 2   # at least one redraw happened
    P = SimpleNamespace(pts=pts, A=A, k=k, rank_tol=0.0, F=F, Fo=Fo, all_matched=False)
    worst, ncmp = compare_boxes(P)
    print(f"[redraw] {ncmp}/{len(Fo.boxes)} boxes compared, worst error / predicted {worst:.2f}", flush=True)
    if ncmp == len(Fo.boxes):
        Bt, At = F.root()
        assert np.array_equal(Bt, Fo.Bt)
    _solution_checks(P)
    e_red = orr.relerr(Fo, A)
    if symmetric:
        F0 = orr.factor(ot.build_tree(pts, m), A @ Om, None, Om, None, k, symmetric=True)
    else:
        F0 = orr.factor(ot.build_tree(pts, m), A @ Om, A.T @ Psi, Om, Psi, k)
    print(f"[redraw] oracle relerr {e_red:.2e} with redraws, {orr.relerr(F0, A):.2e} without", flush=True)


def test_redraw_mixed_refines():
    need_gpu()
    n, k = 64, 32
    pts = inputs.grid2d(n)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
    tc = rsrs.rsrs_build_tree(pts, 64)
    s = tc.samples_required(k, k)
    f = torch.tensor(inputs.rhs(n * n, 3), dtype=torch.float64, device="cuda")
    for sym in (True, False):
        F = rsrs.rsrs_factor_redraw(tc, op, s, 7, k, precision=rsrs.RSRS_PREC_F32_MIXED, symmetric=sym)
        u, rel, it = rsrs.rsrs_solve_refine(F, op, f, tol=1e-10, maxit=30)
        print(f"[redraw mixed sym={sym}] refined {rel:.1e} after {it}", flush=True)
        assert rel <= 1e-10
    with pytest.raises(rsrs.RSRSError) as e:   # FP64 factor from FP32 samples
        rsrs.rsrs_factor_redraw(tc, op, s, 7, k, precision=rsrs.RSRS_PREC_F64, dtype=rsrs.RSRS_F32)
    assert e.value.status == 1
