"""GPU: the symmetric variant (A = A^T, U = L^T) against the oracle's
symmetric variant, on the same seeded Omega.

Per-box blocks are compared with the conditioning-aware tolerance of the
general parity tests; the GPU factor must be exactly symmetric (K_L = K_U^T
and X_RR = X_RR^T bit for bit), its solution within the solve-error bound of
the oracle's, and the mixed-precision symmetric path (BF16 sample products)
must refine to the FP64 bar.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import operators as oop  # noqa: E402
from oracle import rsrs as orr  # noqa: E402
from oracle import tree as ot  # noqa: E402
from paper_2311_01451_amd import inputs, rsrs  # noqa: E402
from test_gpu_parity import compare_boxes, solve_tolerance  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


class SymProblem:
    def __init__(self, pts, A, m, k):
        print(f"[symmetric] N={len(pts)} m={m} k={k}", flush=True)
        self.A = A
        N = len(pts)
        self.tc = rsrs.rsrs_build_tree(pts, m)
        s = self.tc.samples_required(k, k)
        Om, _ = inputs.test_matrices(N, s)
        dOm = dev(Om)
        smp = rsrs.rsrs_samples_wrap(self.tc, dev(A) @ dOm, None, dOm, None)
        self.F = rsrs.rsrs_factor(self.tc, smp, k, symmetric=True)
        self.Fo = orr.factor(ot.build_tree(pts, m), A @ Om, None, Om, None, k, symmetric=True)


@pytest.mark.parametrize("n,m,k", [(32, 32, 16), (32, 16, 8)])
def test_symmetric_parity_with_oracle(n, m, k):
    need_gpu()
    pts = inputs.grid2d(n)
    P = SymProblem(pts, oop.log2d(pts, 1.0 / n), m, k)
    worst, nb = compare_boxes(P)
    print(f"[symmetric] {nb} boxes compared, worst error / predicted {worst:.2f}", flush=True)
    for i in range(P.F.info()["nboxes"]):
        b = P.F.box(i)
        assert np.array_equal(b["KL"], b["KU"].T)
        assert np.array_equal(b["XRR"], b["XRR"].T)
    f = inputs.rhs(n * n, 3)
    u = P.F.solve(dev(f)).cpu().numpy()
    uo = orr.solve(P.Fo, f)
    err = float(np.abs(u - uo).max() / np.abs(uo).max())
    tol = solve_tolerance(P)
    print(f"[symmetric] solution error {err:.2e} (tol {tol:.2e})", flush=True)
    assert err <= tol
    ut = P.F.solve(dev(f), transpose=True).cpu().numpy()
    assert np.abs(ut - u).max() <= 1e-12 * np.abs(u).max()


def test_symmetric_mixed_bf16_refines_and_batches():
    need_gpu()
    n, m, k = 64, 64, 32
    pts = inputs.grid2d(n)
    A = oop.log2d(pts, 1.0 / n)
    tc = rsrs.rsrs_build_tree(pts, m)
    s = tc.samples_required(k, k)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
    mk = lambda: rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=rsrs.RSRS_BF16, symmetric=True)
    F = rsrs.rsrs_factor(tc, mk(), k, precision=rsrs.RSRS_PREC_F32_MIXED, symmetric=True)
    f = inputs.rhs(n * n, 8)
    u, rel, it = rsrs.rsrs_solve_refine(F, op, dev(f), tol=1e-10, maxit=30)
    r = f - A @ u.cpu().numpy()
    host = float(np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)))
    print(f"[symmetric mixed] refined {rel:.2e} after {it} (host {host:.2e})", flush=True)
    assert rel <= 1e-10 and host <= 1.5e-10
    # batched with another problem: bit for bit the same factor
    pts2 = inputs.jittered_grid2d(40, seed_offset=9)
    tc2 = rsrs.rsrs_build_tree(pts2, 64)
    op2 = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts2, 1.0 / 40)
    smp2 = rsrs.rsrs_sample(tc2, op2, tc2.samples_required(24, 24), 3, dtype=rsrs.RSRS_BF16,
                            symmetric=True)
    Fb = rsrs.rsrs_factor_batched([tc, tc2], [mk(), smp2], [k, 24], precision=rsrs.RSRS_PREC_F32_MIXED,
                                  symmetric=True)
    ua = F.solve(dev(f)).cpu().numpy()
    ub = Fb[0].solve(dev(f)).cpu().numpy()
    assert np.array_equal(ua, ub)


def test_symmetric_samples_need_the_symmetric_variant():
    need_gpu()
    pts = inputs.grid2d(16)
    A = oop.log2d(pts, 1.0 / 16)
    tc = rsrs.rsrs_build_tree(pts, 16)
    s = tc.samples_required(8, 8)
    Om, _ = inputs.test_matrices(256, s)
    smp = rsrs.rsrs_samples_wrap(tc, dev(A @ Om), None, dev(Om), None)
    with pytest.raises(rsrs.RSRSError) as e:
        rsrs.rsrs_factor(tc, smp, 8)
    assert e.value.status == 1


def test_symmetric_equals_general_with_equal_samples():
    """Sec. 2.2 on the GPU: the general factorization fed Psi = Omega and
    Z = Y must reproduce the symmetric variant.  First-class boxes see
    M_Y + M_Z = 2 M_Y and must pick the same skeletons with the same T to
    rounding; afterwards the paths differ only through the asymmetry of the
    general X_RR (of the order of the approximation error), so the two
    solutions must agree to within that error."""
    need_gpu()
    n, m, k = 32, 32, 12
    N = n * n
    pts = inputs.grid2d(n)
    A = oop.log2d(pts, 1.0 / n)
    tc = rsrs.rsrs_build_tree(pts, m)
    s = tc.samples_required(k, k)
    Om, _ = inputs.test_matrices(N, s)
    Y = A @ Om
    Fs = rsrs.rsrs_factor(tc, rsrs.rsrs_samples_wrap(tc, dev(Y), None, dev(Om), None), k, symmetric=True)
    Fg = rsrs.rsrs_factor(tc, rsrs.rsrs_samples_wrap(tc, dev(Y), dev(Y), dev(Om), dev(Om)), k)
    nb = Fs.info()["nboxes"]
    same = 0
    first = None
    for i in range(nb):
        a, g = Fs.box(i), Fg.box(i)
        key = (a["level"], a["colour"])
        first = key if first is None else first
        match = np.array_equal(a["S"], g["S"]) and np.array_equal(a["R"], g["R"])
        if key == first:
            assert match, i
            if a["T"].size:
                d = np.abs(a["T"] - g["T"]).max() / np.abs(a["T"]).max()
                assert d < 1e-12, (i, d)
        same += match
    print(f"[symmetric vs general] {same}/{nb} boxes with equal skeletons", flush=True)
    Aap = Fs.apply(dev(np.eye(N))).cpu().numpy()
    e = float(np.linalg.norm(A - Aap, 2) / np.linalg.norm(A, 2))
    f = inputs.rhs(N, 3)
    us = Fs.solve(dev(f)).cpu().numpy()
    ug = Fg.solve(dev(f)).cpu().numpy()
    d = float(np.abs(us - ug).max() / np.abs(us).max())
    print(f"[symmetric vs general] solutions differ by {d:.2e}, relerr {e:.2e}", flush=True)
    assert d < e
