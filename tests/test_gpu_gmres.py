"""GPU: GMRES preconditioned by the factorization (rsrs_solve_gmres), the
paper's use of the factorization as a preconditioner (Sec. 5).

* First-kind log kernel (no identity term, cell-averaged diagonal) with a
  rank far too low (k = 4): the refinement iteration diverges, GMRES reaches
  1e-10; the solution is checked against a dense solve within cond(A) 1e-10
  and the iteration count against the oracle's GMRES on the same factor
  inputs (same Omega, Psi; within a few steps).
* Several columns at once (one of them zero), a short restart length, and
  the mixed-precision factor as preconditioner of the FP64 problem.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import operators as oop  # noqa: E402
from oracle import rsrs as orr  # noqa: E402
from oracle import tree as ot  # noqa: E402
from paper_2311_01451_amd import inputs, rsrs  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_gmres_first_kind_where_refinement_diverges():
    need_gpu()
    n, m, k = 32, 32, 4
    pts = inputs.grid2d(n)
    h = 1.0 / n
    A = oop.log2d_first(pts, h)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D_FIRST, pts, h)
    tc = rsrs.rsrs_build_tree(pts, m)
    s = tc.samples_required(k, k)
    Om, Psi = inputs.test_matrices(n * n, s)
    dOm, dPsi = dev(Om), dev(Psi)
    smp = rsrs.rsrs_samples_wrap(tc, op.matvec(dOm), op.matvec(dPsi, transpose=True), dOm, dPsi)
    F = rsrs.rsrs_factor(tc, smp, k)
    # the operator itself against its definition
    X = np.random.default_rng(3).standard_normal((n * n, 2))
    assert np.abs(op.matvec(dev(X)).cpu().numpy() - A @ X).max() < 1e-13 * np.abs(A @ X).max()
    f = inputs.rhs(n * n, 3)
    df = dev(f)
    _, rel_ref, _ = rsrs.rsrs_solve_refine(F, op, df, tol=1e-10, maxit=12)
    print(f"[gmres] refinement after 12 steps: residual {rel_ref:.1e}", flush=True)
    assert rel_ref > 1.0
    u, rel, it = rsrs.rsrs_solve_gmres(F, op, df, tol=1e-10, restart=30, maxit=300)
    res = f - A @ u.cpu().numpy()
    host = float((np.linalg.norm(res, axis=0) / np.linalg.norm(f, axis=0)).max())
    xs = np.linalg.solve(A, f)
    err = float(np.linalg.norm(u.cpu().numpy() - xs) / np.linalg.norm(xs))
    Fo = orr.factor(ot.build_tree(pts, m), A @ Om, A.T @ Psi, Om, Psi, k)
    _, its_o, _ = orr.gmres(Fo, lambda v: A @ v, f[:, 0], tol=1e-10, restart=30, maxit=300)
    print(f"[gmres] GPU: residual {rel:.1e} (host {host:.1e}) after {it} steps, oracle {its_o[0]} steps; "
          f"error vs dense solve {err:.1e}", flush=True)
    assert rel <= 1e-10 and host <= 2e-10
    assert err <= 10 * np.linalg.cond(A) * 1e-10
    assert abs(it - its_o[0]) <= max(5, 0.1 * its_o[0])


def test_gmres_columns_restart_and_mixed_preconditioner():
    need_gpu()
    n, k = 64, 16
    pts = inputs.grid2d(n)
    h = 1.0 / n
    A = oop.log2d_first(pts, h)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D_FIRST, pts, h)
    tc = rsrs.rsrs_build_tree(pts, 64)
    s = tc.samples_required(k, k)
    rng = np.random.default_rng(21)
    f = rng.standard_normal((n * n, 5))
    f[:, 2] = 0.0
    df = dev(f)
    for prec, dt in ((rsrs.RSRS_PREC_F64, rsrs.RSRS_F64), (rsrs.RSRS_PREC_F32_MIXED, rsrs.RSRS_F32)):
        smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=dt)
        F = rsrs.rsrs_factor(tc, smp, k, precision=prec)
        for restart in (30, 4):
            u, rel, it = rsrs.rsrs_solve_gmres(F, op, df, tol=1e-10, restart=restart, maxit=400)
            un = u.cpu().numpy()
            assert np.all(un[:, 2] == 0.0)
            nz = [0, 1, 3, 4]
            res = f[:, nz] - A @ un[:, nz]
            host = float((np.linalg.norm(res, axis=0) / np.linalg.norm(f[:, nz], axis=0)).max())
            print(f"[gmres] precision {prec} restart {restart}: residual {rel:.1e} (host {host:.1e}) "
                  f"after {it} steps", flush=True)
            assert rel <= 1e-10 and host <= 2e-10


def test_gmres_rejects_bad_arguments():
    need_gpu()
    pts = inputs.grid2d(16)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / 16)
    tc = rsrs.rsrs_build_tree(pts, 16)
    smp = rsrs.rsrs_sample(tc, op, tc.samples_required(8, 8), 1)
    F = rsrs.rsrs_factor(tc, smp, 8)
    f = torch.zeros((256, 2), dtype=torch.float64, device="cuda")
    for kw in ({"restart": 0}, {"restart": 65}, {"tol": 0.0}, {"maxit": 0}):
        with pytest.raises(rsrs.RSRSError) as e:
            rsrs.rsrs_solve_gmres(F, op, f, **kw)
        assert e.value.status == 1
