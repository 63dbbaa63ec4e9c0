"""GPU: the continuous-batching server (rsrs_server_*).

* Results in the mix equal results alone: every solve request, batched by the
  server with other requests of different widths (and interleaved with
  requests for another factor), is compared with rsrs_solve of that request
  alone; the columns of a batch are computed independently by the same
  kernels, so the FP64 results must agree to the last bit and the mixed ones
  within FP32 rounding of the same arithmetic (stated bound 1e-6 relative).
* Factor requests are admitted by the HBM budget: the bytes charged never
  exceed it, a request larger than the budget is refused at once, and each
  factor made by the server equals rsrs_factor on the same seed.
* Work overlaps: solves on a resident factor complete while a large
  factorization submitted before them is still running.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2311_01451_amd import inputs, rsrs  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _factor(n, k, mixed, seed_off=0, m=64):
    pts = inputs.jittered_grid2d(n, seed_offset=3 + seed_off)
    tc = rsrs.rsrs_build_tree(pts, m)
    s = tc.samples_required(k, k)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
    dt = rsrs.RSRS_F32 if mixed else rsrs.RSRS_F64
    prec = rsrs.RSRS_PREC_F32_MIXED if mixed else rsrs.RSRS_PREC_F64
    smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED + seed_off, dtype=dt)
    F = rsrs.rsrs_factor(tc, smp, k, precision=prec)
    return dict(pts=pts, tc=tc, s=s, op=op, F=F, N=n * n, k=k, prec=prec)


def test_results_in_the_mix_equal_results_alone():
    need_gpu()
    A = _factor(48, 32, mixed=False, seed_off=1)
    B = _factor(40, 32, mixed=True, seed_off=2)
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(40):
        P = A if i % 3 else B
        w = int(rng.choice([1, 4, 16, 64, 256]))
        f = dev(rng.standard_normal((P["N"], w)))
        reqs.append((P, f, P["F"].solve(f)))   # the request alone
    torch.cuda.synchronize()
    sv = rsrs.Server(hbm_budget=0, max_batch_cols=512)
    ida = sv.add_factor(A["F"])
    idb = sv.add_factor(B["F"])
    tickets = []
    for P, f, _ in reqs:
        tickets.append(sv.submit_solve(ida if P is A else idb, f))
    for (P, f, alone), (t, out) in zip(reqs, tickets):
        sv.wait(t)
        d = float((out - alone).abs().max() / alone.abs().max())
        if P is A:
            assert d == 0.0, d
        else:
            assert d <= 1e-6, d
    st = sv.stats()
    print(f"[server] {st['solves_done']} solves in {st['batches']} batches, {st['cols_done']} columns, "
          f"p50 {st['solve_p50_ms']:.2f} ms p99 {st['solve_p99_ms']:.2f} ms", flush=True)
    assert st["solves_done"] == len(reqs)
    assert st["batches"] < len(reqs)   # requests were batched
    sv.close()


def test_factor_requests_admitted_by_budget():
    need_gpu()
    budget = 400 << 20
    sv = rsrs.Server(hbm_budget=budget, max_batch_cols=64)
    jobs = []
    for i in range(4):
        n, k = 64, 32
        pts = inputs.jittered_grid2d(n, seed_offset=50 + i)
        tc = rsrs.rsrs_build_tree(pts, 64)
        s = tc.samples_required(k, k)
        op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
        t = sv.submit_factor(tc, op, s, 1000 + i, k, precision=rsrs.RSRS_PREC_F32_MIXED)
        jobs.append((pts, tc, s, op, t))
    f = dev(inputs.rhs(64 * 64, 4))
    for i, (pts, tc, s, op, t) in enumerate(jobs):
        fid, lat = sv.wait(t)
        tk, out = sv.submit_solve(fid, f)
        sv.wait(tk)
        # the same factor built directly
        op2 = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / 64)
        smp = rsrs.rsrs_sample(tc, op2, s, 1000 + i, dtype=rsrs.RSRS_F32)
        F = rsrs.rsrs_factor(tc, smp, 32, precision=rsrs.RSRS_PREC_F32_MIXED)
        ref = F.solve(f)
        d = float((out - ref).abs().max() / ref.abs().max())
        print(f"[server factor] request {i}: latency {lat:.1f} ms, |u - u_direct| {d:.1e}", flush=True)
        assert d <= 1e-6
        sv.release(fid)
    st = sv.stats()
    print(f"[server factor] peak charged {st['hbm_peak'] / 2**20:.0f} MiB of {budget / 2**20:.0f}", flush=True)
    assert st["factors_done"] == 4 and 0 < st["hbm_peak"] <= budget
    # a request that can never fit is refused at once
    sv2 = rsrs.Server(hbm_budget=1 << 20, max_batch_cols=64)
    pts, tc, s, op, _ = jobs[0]
    with pytest.raises(rsrs.RSRSError) as e:
        sv2.submit_factor(tc, op, s, 1, 32, precision=rsrs.RSRS_PREC_F32_MIXED)
    assert e.value.status == 6
    sv2.close()
    sv.close()


def test_solves_overlap_a_running_factorization():
    need_gpu()
    small = _factor(32, 16, mixed=False, seed_off=5, m=32)
    sv = rsrs.Server(hbm_budget=0, max_batch_cols=256)
    fid = sv.add_factor(small["F"])
    n, k = 128, 64
    pts = inputs.jittered_grid2d(n, seed_offset=77)
    tc = rsrs.rsrs_build_tree(pts, 64)
    s = tc.samples_required(k, k)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
    tf = sv.submit_factor(tc, op, s, 5, k)
    f = dev(inputs.rhs(small["N"], 8))
    solves = [sv.submit_solve(fid, f) for _ in range(20)]
    lats = [sv.wait(t)[1] for t, _ in solves]
    big_id, lat_f = sv.wait(tf)
    print(f"[server overlap] factorization {lat_f:.0f} ms; solves max {max(lats):.1f} ms", flush=True)
    assert max(lats) < lat_f
    tk, out = sv.submit_solve(big_id, dev(inputs.rhs(n * n, 2)))
    sv.wait(tk)
    assert torch.isfinite(out).all()
    sv.close()


def test_served_solves_refined_to_tolerance():
    """With refinement attached to a resident factor, every served result
    meets the tolerance through the operator's FP64 residual (mixed factor,
    one-shot residual ~1e-5), alone and batched with other requests; the
    stats report the refined batches and the largest residual."""
    need_gpu()
    P = _factor(48, 32, mixed=True, seed_off=4)
    sv = rsrs.Server(hbm_budget=0, max_batch_cols=256)
    fid = sv.add_factor(P["F"])
    sv.set_refine(fid, P["op"], tol=1e-10, maxit=20)
    rng = np.random.default_rng(12)
    reqs = []
    for w in (1, 4, 16, 64, 3):
        f = dev(rng.standard_normal((P["N"], w)))
        t, out = sv.submit_solve(fid, f)
        reqs.append((f, t, out))
    for f, t, out in reqs:
        sv.wait(t)
        r = f - P["op"].matvec(out)
        rel = float((r.norm(dim=0) / f.norm(dim=0)).max())
        assert rel <= 1e-10, rel
    st = sv.stats()
    print(f"[server refine] batches {st['refined_batches']}, corrections {st['refine_steps']}, "
          f"max residual {st['max_relres']:.1e}", flush=True)
    assert st["refined_batches"] >= 1 and st["max_relres"] <= 1e-10 and st["refine_steps"] >= 1
    sv.close()


def test_budget_counts_the_kept_scratch():
    """Device memory kept by the library from finished factorizations counts
    against the budget and is trimmed when a factor request would not fit
    otherwise: with a budget just above one request's estimate, requests
    submitted one after another are all admitted and served."""
    need_gpu()
    n, k = 48, 32
    pts = inputs.jittered_grid2d(n, seed_offset=21)
    tc = rsrs.rsrs_build_tree(pts, 64)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
    s = tc.samples_required(k, k)
    # a large factorization first leaves its scratch in the pool
    big = _factor(96, 64, mixed=False, seed_off=5)
    del big
    sv = rsrs.Server(hbm_budget=1 << 30, max_batch_cols=64)
    for j in range(3):
        t = sv.submit_factor(tc, op, s, inputs.BASE_SEED + j, k)
        fid, _ = sv.wait(t, timeout_ms=60000)
        st = sv.stats()
        assert st["hbm_peak"] <= 1 << 30
        sv.release(fid)
    sv.close()
