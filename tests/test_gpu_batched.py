"""GPU: many independent problems factored together (rsrs_factor_batched).

Each problem of a batch must get exactly the factor that rsrs_factor computes
for it alone: the batch only merges the launches of class t of every problem,
and every output tile of the batched kernels is computed by the same sequence
of instructions either way, so the stored blocks are compared bit for bit.
The uneven many-problem workload (jittered 2D grids of log-uniform size, each
problem its own rank, FP32 mixed precision) is then checked through the
method's own guarantee: every solution reaches the residual bar after
refinement with its FP64 operator, and agrees with a dense solve.
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


def dev(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _problem(n, m, k, i, mixed):
    pts = inputs.jittered_grid2d(n, seed_offset=3 + 100 * i)
    A = oop.log2d(pts, 1.0 / n)
    tc = rsrs.rsrs_build_tree(pts, m)
    s = tc.samples_required(k, k)
    Om, Psi = inputs.test_matrices(n * n, s, 100 * i)
    if mixed:
        Om = Om.astype(np.float32).astype(np.float64)
        Psi = Psi.astype(np.float32).astype(np.float64)
    return dict(pts=pts, A=A, tc=tc, s=s, k=k, m=m, Om=Om, Psi=Psi, Y=A @ Om, Z=A.T @ Psi)


def _samples(P, mixed):
    dt = torch.float32 if mixed else torch.float64
    return rsrs.rsrs_samples_wrap(P["tc"], dev(P["Y"], dt), dev(P["Z"], dt), dev(P["Om"], dt),
                                  dev(P["Psi"], dt))


@pytest.mark.parametrize("mixed", [False, True])
def test_batched_equals_individual_bitwise(mixed):
    need_gpu()
    spec = [(24, 16, 8), (37, 32, 12), (30, 16, 16), (18, 32, 8), (41, 64, 16)]
    probs = [_problem(n, m, k, i, mixed) for i, (n, m, k) in enumerate(spec)]
    prec = rsrs.RSRS_PREC_F32_MIXED if mixed else rsrs.RSRS_PREC_F64
    print(f"[batched] mixed={mixed} sizes={[n * n for n, _, _ in spec]}", flush=True)
    single = [rsrs.rsrs_factor(P["tc"], _samples(P, mixed), P["k"], precision=prec) for P in probs]
    batch = rsrs.rsrs_factor_batched([P["tc"] for P in probs], [_samples(P, mixed) for P in probs],
                                     [P["k"] for P in probs], precision=prec)
    torch.cuda.synchronize()
    for i, (F1, F2) in enumerate(zip(single, batch)):
        i1, i2 = F1.info(), F2.info()
        assert i1["nboxes"] == i2["nboxes"] and i1["stored_values"] == i2["stored_values"]
        for b in range(i1["nboxes"]):
            x1, x2 = F1.box(b), F2.box(b)
            for key in ("Ba", "Na", "S", "R", "T", "XRR", "KU", "KL"):
                assert np.array_equal(x1[key], x2[key]), (i, b, key)
        assert np.array_equal(F1.root()[1], F2.root()[1])
        f = inputs.rhs(probs[i]["A"].shape[0], 2)
        u1 = F1.solve(dev(f)).cpu().numpy()
        u2 = F2.solve(dev(f)).cpu().numpy()
        assert np.array_equal(u1, u2)


def test_batched_fp64_matches_oracle():
    need_gpu()
    spec = [(24, 16, 8), (33, 32, 12), (20, 16, 16)]
    probs = [_problem(n, m, k, i, False) for i, (n, m, k) in enumerate(spec)]
    Fs = rsrs.rsrs_factor_batched([P["tc"] for P in probs], [_samples(P, False) for P in probs],
                                  [P["k"] for P in probs])
    for P, F in zip(probs, Fs):
        Fo = orr.factor(ot.build_tree(P["pts"], P["m"]), P["Y"], P["Z"], P["Om"], P["Psi"], P["k"])
        f = inputs.rhs(P["A"].shape[0], 2)
        u = F.solve(dev(f)).cpu().numpy()
        uo = orr.solve(Fo, f)
        eps = orr.relerr(Fo, P["A"])
        cond = np.linalg.cond(P["A"])
        tol = 4.0 * eps * cond / (1.0 - eps * cond) + 1e-12
        err = float(np.abs(u - uo).max() / np.abs(uo).max())
        print(f"[batched oracle] N={P['A'].shape[0]} k={P['k']} err {err:.2e} tol {tol:.2e}", flush=True)
        assert err <= tol


def test_batched_errors():
    need_gpu()
    P = _problem(16, 16, 8, 0, False)
    Q = _problem(20, 16, 8, 1, False)
    smp = _samples(P, False)
    with pytest.raises(rsrs.RSRSError) as e:   # the same samples twice
        rsrs.rsrs_factor_batched([P["tc"], P["tc"]], [smp, smp], [8, 8])
    assert e.value.status == 1
    # a problem with too few samples is named, and nothing is factored
    Om, Psi = inputs.test_matrices(400, Q["s"] - 1, 7)
    bad = rsrs.rsrs_samples_wrap(Q["tc"], dev(Q["A"] @ Om), dev(Q["A"].T @ Psi), dev(Om), dev(Psi))
    with pytest.raises(rsrs.RSRSError) as e:
        rsrs.rsrs_factor_batched([P["tc"], Q["tc"]], [_samples(P, False), bad], [8, 8])
    assert e.value.status == 2 and "problem 1" in str(e.value) and e.value.required_s == Q["s"]


def test_uneven_mixed_batch_refines():
    """Sixteen jittered log-kernel problems, N log-uniform in [2048, 16384],
    k in {32, 48, 64}, s = s_required, mixed precision, one batched factorization,
    refinement to 1e-6 with each problem's FP64 operator."""
    need_gpu()
    rng = np.random.default_rng(inputs.BASE_SEED + 7)
    probs = []
    for i in range(16):
        n = int(round(np.exp(rng.uniform(np.log(np.sqrt(2048)), np.log(np.sqrt(16384))))))
        k = int(rng.choice([32, 48, 64]))
        pts = inputs.jittered_grid2d(n, seed_offset=3 + 100 * i)
        tc = rsrs.rsrs_build_tree(pts, 64)
        s = tc.samples_required(k, k)
        op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
        smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED + 100 * i, dtype=rsrs.RSRS_F32)
        probs.append(dict(n=n, k=k, pts=pts, tc=tc, s=s, op=op, smp=smp))
    print("[uneven] N =", [P["n"] ** 2 for P in probs], "k =", [P["k"] for P in probs], flush=True)
    Fs = rsrs.rsrs_factor_batched([P["tc"] for P in probs], [P["smp"] for P in probs],
                                  [P["k"] for P in probs], precision=rsrs.RSRS_PREC_F32_MIXED)
    for i, (P, F) in enumerate(zip(probs, Fs)):
        N = P["n"] ** 2
        f = inputs.rhs(N, 4, 100 * i)
        u, rel, it = rsrs.rsrs_solve_refine(F, P["op"], dev(f), tol=1e-6, maxit=30)
        assert rel <= 1e-6, (i, rel)
        if i % 5 == 0:   # dense check on some of them
            A = oop.log2d(P["pts"], 1.0 / P["n"])
            r = f - A @ u.cpu().numpy()
            assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)) <= 1.5e-6
        print(f"[uneven] problem {i}: N={N} k={P['k']} s={P['s']} residual {rel:.2e} after {it}",
              flush=True)
