"""GPU: the many-problem workload at its stated size.

48 jittered 2D grids with the log kernel of the 64 x 64 workload, N = n^2
log-uniform from about 2,000 to 33,000 points, ranks drawn from {32, 48, 64},
leaves of 64 points, s = s_required of each problem (p = k), all factored by
one rsrs_factor_batched call.

* Mixed precision (FP32 samples and products, FP64 pivots): four problems
  (the two smallest, the largest and one in the middle) are factored again on
  their own from the same samples and must give bit-identical factors (the
  batch only merges launches); every problem then refines to 1e-6 through
  its own FP64 operator, and the smallest three also against a dense solve.
* FP64: the whole batch again, the two smallest problems sampled from
  host-drawn test matrices, and those two compared with the oracle box by
  box, then by their solutions (the parity bar of the single-problem tests).
"""
import time
from types import SimpleNamespace

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import operators as oop  # noqa: E402
from oracle import rsrs as orr  # noqa: E402
from oracle import tree as ot  # noqa: E402
from paper_2311_01451_amd import inputs, rsrs  # noqa: E402
from test_gpu_parity import _solution_checks, compare_boxes  # noqa: E402

LEAF = 64


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _setup():
    specs = inputs.uneven_batch()
    for P in specs:
        P["pts"] = inputs.jittered_grid2d(P["n"], seed_offset=P["geom_seed"])
        P["tc"] = rsrs.rsrs_build_tree(P["pts"], LEAF)
        P["s"] = P["tc"].samples_required(P["k"], P["k"])
    return specs


def _op(P):
    return rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, P["pts"], 1.0 / P["n"])


def _sample(P, dtype):
    op = _op(P)
    smp = rsrs.rsrs_sample(P["tc"], op, P["s"], inputs.BASE_SEED + P["seed"], dtype=dtype)
    torch.cuda.synchronize()
    del op   # the dense kernel matrices go; a fresh operator serves the residuals
    return smp


def test_config3_mixed_batch_full_size():
    need_gpu()
    specs = _setup()
    Ns = [P["n"] ** 2 for P in specs]
    print(f"[config3] {len(specs)} problems, N {min(Ns)}..{max(Ns)} (total {sum(Ns)}), "
          f"k counts {[sum(P['k'] == k for P in specs) for k in (32, 48, 64)]}", flush=True)
    smps = [_sample(P, rsrs.RSRS_F32) for P in specs]
    print("[config3] sampled", flush=True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    Fs = rsrs.rsrs_factor_batched([P["tc"] for P in specs], smps, [P["k"] for P in specs],
                                  precision=rsrs.RSRS_PREC_F32_MIXED)
    torch.cuda.synchronize()
    print(f"[config3] batched factor {time.perf_counter() - a:.3f} s", flush=True)
    del smps
    order = np.argsort(Ns)
    check = [int(order[0]), int(order[1]), int(order[len(order) // 2]), int(order[-1])]
    for i in check:
        P = specs[i]
        F1 = rsrs.rsrs_factor(P["tc"], _sample(P, rsrs.RSRS_F32), P["k"], precision=rsrs.RSRS_PREC_F32_MIXED)
        nb = F1.info()["nboxes"]
        assert nb == Fs[i].info()["nboxes"]
        for q in range(0, nb, max(1, nb // 8)):
            x, y = F1.box(q), Fs[i].box(q)
            for key in ("S", "T", "XRR", "KU", "KL"):
                assert np.array_equal(x[key], y[key]), (i, q, key)
        f = dev(inputs.rhs(Ns[i], 2, P["seed"]))
        assert torch.equal(F1.solve(f), Fs[i].solve(f)), i
        print(f"[config3] problem {i} (N={Ns[i]}, k={P['k']}): batched factor equals the lone one bit for bit",
              flush=True)
        del F1
    worst = 0.0
    for i, (P, F) in enumerate(zip(specs, Fs)):
        op = _op(P)
        f = inputs.rhs(Ns[i], 16, P["seed"])
        u, rel, it = rsrs.rsrs_solve_refine(F, op, dev(f), tol=1e-6, maxit=30)
        assert rel <= 1e-6, (i, rel)
        worst = max(worst, rel)
        if i in (int(order[0]), int(order[1]), int(order[2])):
            A = oop.log2d(P["pts"], 1.0 / P["n"])
            r = f - A @ u.cpu().numpy()
            host = float(np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)))
            assert host <= 1.5e-6, (i, host)
        print(f"[config3] problem {i}: N={Ns[i]} k={P['k']} s={P['s']} residual {rel:.1e} after {it}",
              flush=True)
        del op
    print(f"[config3] all {len(specs)} problems refined to 1e-6 (worst {worst:.1e})", flush=True)


def test_config3_fp64_batch_oracle_subset():
    need_gpu()
    specs = _setup()
    Ns = [P["n"] ** 2 for P in specs]
    order = np.argsort(Ns)
    subset = [int(order[0]), int(order[1])]
    smps = []
    for i, P in enumerate(specs):
        if i in subset:
            P["A"] = oop.log2d(P["pts"], 1.0 / P["n"])
            Om, Psi = inputs.test_matrices(Ns[i], P["s"], P["seed"])
            P["Om"], P["Psi"] = Om, Psi
            smps.append(rsrs.rsrs_samples_wrap(P["tc"], dev(P["A"] @ Om), dev(P["A"].T @ Psi), dev(Om), dev(Psi)))
        else:
            smps.append(_sample(P, rsrs.RSRS_F64))
    print("[config3 fp64] sampled", flush=True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    Fs = rsrs.rsrs_factor_batched([P["tc"] for P in specs], smps, [P["k"] for P in specs])
    torch.cuda.synchronize()
    print(f"[config3 fp64] batched factor {time.perf_counter() - a:.3f} s", flush=True)
    del smps
    for i in subset:
        P = specs[i]
        Fo = orr.factor(ot.build_tree(P["pts"], LEAF), P["A"] @ P["Om"], P["A"].T @ P["Psi"], P["Om"], P["Psi"],
                        P["k"])
        Q = SimpleNamespace(pts=P["pts"], A=P["A"], k=P["k"], rank_tol=0.0, F=Fs[i], Fo=Fo, all_matched=False)
        worst, ncmp = compare_boxes(Q)
        print(f"[config3 fp64] problem {i} (N={Ns[i]}, k={P['k']}): {ncmp}/{len(Fo.boxes)} boxes compared, "
              f"worst / predicted {worst:.2f}", flush=True)
        _solution_checks(Q)
    op = _op(specs[int(order[-1])])
    f = dev(inputs.rhs(Ns[int(order[-1])], 4, 7))
    u, rel, it = rsrs.rsrs_solve_refine(Fs[int(order[-1])], op, f, tol=1e-10, maxit=10)
    print(f"[config3 fp64] largest problem refined to {rel:.1e} after {it}", flush=True)
    assert rel <= 1e-10
