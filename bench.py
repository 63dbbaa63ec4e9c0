#!/usr/bin/env python
"""Benchmark of the RSRS hot path on one MI355X.

Workload: 2D log-kernel operator A_ij = delta_ij + h^2 (-log|x_i - x_j| / 2 pi),
A_ii = 1 + h^2/2, on the 256 x 256 cell-centred grid of [0,1]^2 (N = 65,536,
h = 1/256), quadtree leaf 64, rank k = 64, p = k, 16 right-hand sides
N(0,1).  The configured s = 640 is below the sample count the method requires
(s >= |B_a| + |N_a| + k + p for every box), so the step runs at
s = max(640, s_required) and reports both.

One step = the whole hot path on one batch: build the tree, draw Omega/Psi
and sample Y = A Omega, Z = A^T Psi through the operator, factor (Algorithm
1), solve the 16 right-hand sides and refine with the FP64 residual of the
operator until the relative residual is <= 1e-6.  The operator is symmetric,
so the step uses the symmetric variant (U = L^T, one sketch side); it runs in
two precisions: mixed (BF16 sample products with FP32 accumulation, FP32
sketches and MFMA products in the factorization, FP64 pivots, inverses and
residuals) and plain FP64, and both again with the general two-sided
algorithm.  value = right-hand-side columns solved per second of step time
of the mixed symmetric path; the others are reported beside it
("mixed_general", "fp64", "fp64_general").  The
operator itself (the black box) is built once outside the timed region.

Prints ONE JSON line (rank 0).  Extra fields: per-phase times, p50/p99 solve
latency of the resident factor, the roofline of the dominant kernel measured
with HIP events inside the timed region, and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "factor s + solved RHS cols/s at rel. residual 1e-6, mixed vs FP64; p99 solve ms"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

GRID_N = 256
LEAF = 64
K = 64
S_CFG = 640
NRHS = 16
TOL = 1e-6


def workload_config(s_req: int, s_eff: int, reproject: int) -> dict:
    return {"workload": f"2D log-kernel operator on a {GRID_N}x{GRID_N} grid (N={GRID_N**2}), "
                        f"quadtree leaf {LEAF}, k=p={K}, {NRHS} RHS, residual <= {TOL:g} "
                        "(FP64 residual), mixed precision vs FP64",
            "N": GRID_N ** 2, "leaf": LEAF, "k": K, "p": K, "s_configured": S_CFG,
            "s_required": s_req, "s": s_eff, "nrhs": NRHS, "tol": TOL,
            "projection_passes": 1 + reproject,
            "precision": "mixed: BF16 sample products (FP32 accumulation), FP32 sketches, MFMA "
                         "products and Gram Cholesky in the factorization, FP64 pivoted-QR "
                         "decisions, Gauss-Jordan and residuals; FP64 beside it",
            "variant": "symmetric (A = A^T: U = L^T, one sketch side); the general two-sided "
                       "algorithm is reported beside it"}


def gpu_bench(steps: int, warmup: int, do_profile: bool, latency_reps: int = 40,
              calib_copy_mib: int = 0, mode: str = "fp64", ctx: dict | None = None,
              symmetric: bool = True, reproject: int = 0):
    import torch
    from paper_2311_01451_amd import inputs, rsrs

    if calib_copy_mib > 0:
        # a plain copy of known size: reference for the HBM byte counters
        n = calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = {} if ctx is None else ctx
    pts = inputs.grid2d(GRID_N)
    h = 1.0 / GRID_N
    if "op" not in ctx:
        ctx["op"] = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, h)
        ctx["f"] = torch.tensor(inputs.rhs(GRID_N ** 2, NRHS), dtype=torch.float64, device="cuda")
    op, f = ctx["op"], ctx["f"]
    mixed = mode != "fp64"
    dtype = {"bf16": rsrs.RSRS_BF16, "fp32": rsrs.RSRS_F32, "fp64": rsrs.RSRS_F64}[mode]
    prec = rsrs.RSRS_PREC_F32_MIXED if mixed else rsrs.RSRS_PREC_F64
    if mixed:   # the rounded copies of the kernel matrix belong to the operator, built once
        op.matvec(torch.zeros((GRID_N ** 2, 8), dtype=torch.float32, device="cuda"), bf16=mode == "bf16")
    torch.cuda.synchronize()

    def step(record):
        t0 = time.perf_counter()
        tree = rsrs.rsrs_build_tree(pts, LEAF)
        s_req = tree.samples_required(K, K)
        s_eff = max(S_CFG, s_req)
        t1 = time.perf_counter()
        smp = rsrs.rsrs_sample(tree, op, s_eff, inputs.BASE_SEED, dtype=dtype, symmetric=symmetric)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        F = rsrs.rsrs_factor(tree, smp, K, precision=prec, symmetric=symmetric, reproject=reproject)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        u, rel, it = rsrs.rsrs_solve_refine(F, op, f, tol=TOL, maxit=30)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        record.append(dict(tree=t1 - t0, sample=t2 - t1, factor=t3 - t2, solve=t4 - t3,
                           relres=rel, iters=it, s_req=s_req, s_eff=s_eff,
                           flops=F.info()["flops"], u=u))
        return F

    warm = []
    for _ in range(warmup):
        F = step(warm)
        del F
    prof_all, dominant = {}, None
    if do_profile:
        # one untimed step with every launch bracketed: the per-kernel
        # breakdown, and the kernel with the largest share of GPU time
        rsrs.rsrs_profile_reset()
        rsrs.rsrs_profile_filter(None)
        rsrs.rsrs_profile_enable(True)
        F = step([])
        del F
        rsrs.rsrs_profile_enable(False)
        prof_all = rsrs.rsrs_profile_read()
        rsrs.rsrs_profile_reset()
        merged = by_kernel(prof_all)
        dominant = max(merged, key=lambda t: merged[t]["ms"])
        # the timed steps bracket only that kernel's launches
        rsrs.rsrs_profile_filter(dominant)
        rsrs.rsrs_profile_enable(True)
    rec = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        F = step(rec)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {}
    if do_profile:
        rsrs.rsrs_profile_enable(False)
        prof = rsrs.rsrs_profile_read()
        rsrs.rsrs_profile_reset()
        rsrs.rsrs_profile_filter(None)

    # solve latency of the resident factor (16 RHS per request): one-shot
    # solves, and solves refined to the tolerance through the operator
    lat, latr = [], []
    for _ in range(latency_reps + 5):
        torch.cuda.synchronize()
        a = time.perf_counter()
        F.solve(f)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    for _ in range(max(latency_reps // 4, 3) + 2):
        torch.cuda.synchronize()
        a = time.perf_counter()
        rsrs.rsrs_solve_refine(F, op, f, tol=TOL, maxit=30)
        torch.cuda.synchronize()
        latr.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat[5:] if len(lat) > 5 else lat)
    latr = np.array(latr[2:])
    # one-shot residual of the last factor (FP64 residual through the
    # operator), outside the timed steps
    r = f - op.matvec(F.solve(f))
    rec[-1]["relres_oneshot"] = float((r.norm(dim=0) / f.norm(dim=0)).max())
    wm = rsrs.rsrs_work_model(rsrs.rsrs_build_tree(pts, LEAF), K, rec[-1]["s_eff"], symmetric,
                              4 if mixed else 8)
    rec[-1]["model_flops"] = wm["flops"]
    return rec, elapsed, (prof, prof_all), (lat, latr)


def by_kernel(prof: dict) -> dict:
    """Merge call-site tags ("<kernel>:<site>") into one entry per kernel."""
    out = {}
    for tag, v in prof.items():
        k = tag.split(":")[0]
        e = out.setdefault(k, dict(launches=0, ms=0.0, flops=0.0, bytes=0.0))
        for f in e:
            e[f] += v[f]
    return out


# HBM traffic measured by rocprofv3 counters for the kernels that can be the
# dominant one: tag -> committed summary (kernel name, bytes per launch and
# the hash of the source the kernel was built from when measured)
TRAFFIC_FILES = {
    "chol32_panel": os.path.join(ROOT, "profiles", "chol32_panel_65k_log2d_mixed_traffic.json"),
    "gemm32_nt_syrk_128x128": os.path.join(ROOT, "profiles", "gemm32_syrk_128x128_65k_log2d_mixed_traffic.json"),
    "gemm32_nt_syrk_64x64": os.path.join(ROOT, "profiles", "gemm32_syrk_64x64_65k_log2d_mixed_traffic.json"),
    "gemm32_nn_full_64x64": os.path.join(ROOT, "profiles", "gemm32_nn_64x64_65k_log2d_mixed_traffic.json"),
    "gemm_bf16_hipblaslt": os.path.join(ROOT, "profiles", "gemm_bf16_hipblaslt_65k_log2d_mixed_traffic.json"),
    "gemm32_nt_full_64x64": os.path.join(ROOT, "profiles", "gemm32_nt_64x64_65k_log2d_mixed_traffic.json"),
    "gauss_jordan_blk": os.path.join(ROOT, "profiles", "gje_blk_65k_log2d_mixed_traffic.json"),
    "id_pchol": os.path.join(ROOT, "profiles", "id_pchol_65k_log2d_mixed_traffic.json"),
    "gemm_nn_full_128x128": os.path.join(ROOT, "profiles", "gemm_f64_nn_128x128_65k_log2d_fp64_traffic.json"),
}
# machine balance of MI355X in FP64 (flops per HBM byte): below it a kernel
# is priced against HBM bandwidth
MACHINE_BALANCE = 78.6e12 / 8.0e12


def measured_traffic(tag: str):
    """HBM bytes per launch from the committed counter summary, or None when
    there is none for this kernel or its source changed since."""
    import hashlib
    path = TRAFFIC_FILES.get(tag)
    if not path:
        return None
    try:
        t = json.load(open(path))
        src = open(os.path.join(ROOT, t["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != t.get("source_sha256"):
        return None
    return round(t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"], 1)


def roofline_entry(tag: str, e: dict, total_ms: float, all_ms: float, steps: int) -> dict:
    """Roofline of one kernel from its summed launches: GEMM forms run on
    MFMA (peak of their operand type); kernels whose algorithmic flops per
    byte fall below the machine balance are priced by their bytes against
    HBM; the rest are FP64 vector work."""
    streaming = e["bytes"] > 0 and e["flops"] < MACHINE_BALANCE * e["bytes"]
    if tag.startswith(("gemm", "rocblas")) or (e["flops"] > 0 and not streaming):
        ach = e["flops"] / (e["ms"] * 1e-3) / 1e12
        if tag.startswith("gemm_bf16"):
            bound, peak = "mfma", PEAK_BF16_TFLOPS
        elif tag.startswith(("gemm32", "chol32", "rocblas_sgemm")):
            bound, peak = "mfma", PEAK_FP32_TFLOPS
        elif tag.startswith(("gemm", "gauss_jordan", "chol", "rocblas_dgemm")):
            bound, peak = "mfma", PEAK_FP64_TFLOPS
        else:
            bound, peak = "alu", PEAK_FP64_TFLOPS
        unit = "TFLOP/s"
    else:
        ach = e["bytes"] / (e["ms"] * 1e-3) / 1e9
        bound, peak, unit = "hbm", PEAK_HBM_GBS, "GB/s"
    return {"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 4), "traffic": measured_traffic(tag), "kernel": tag,
            "launches_per_step": e["launches"] / steps,
            "avg_launch_ms": e["ms"] / e["launches"],
            "algorithmic_flops_per_launch": e["flops"] / e["launches"],
            "algorithmic_bytes_per_launch": e["bytes"] / e["launches"],
            "share_of_kernel_time": round(total_ms / all_ms, 4)}


def per_level_roofline(prof_all: dict) -> dict | None:
    """Roofline of the factorization's own dominant kernel (operator products
    and solves left out), from the profiled step (every launch bracketed)."""
    if not prof_all:
        return None
    keep = {t: v for t, v in prof_all.items()
            if not t.endswith(":operator") and not t.startswith("solve") and ":solve" not in t}
    merged = by_kernel(keep)
    if not merged:
        return None
    tag = max(merged, key=lambda t: merged[t]["ms"])
    all_ms = sum(v["ms"] for v in by_kernel(prof_all).values())
    out = roofline_entry(tag, merged[tag], merged[tag]["ms"], all_ms, 1)
    out["timed"] = "profiled step (every launch bracketed by HIP events)"
    return out


def roofline_from_profile(prof: dict, prof_all: dict, steps: int) -> dict | None:
    """Roofline of the kernel with the largest share of GPU time in the
    profiled step, from its launches in the timed steps (HIP events on the
    launch stream)."""
    if not prof or not prof_all:
        return None
    prof, prof_all = by_kernel(prof), by_kernel(prof_all)
    tag = max(prof_all, key=lambda t: prof_all[t]["ms"])
    if tag not in prof:
        return None
    e = prof[tag]
    total_ms = sum(v["ms"] for v in prof_all.values())
    return roofline_entry(tag, e, prof_all[tag]["ms"], total_ms, steps)


def host_info() -> dict:
    """CPU model, usable cores and the BLAS the oracle runs on."""
    from threadpoolctl import threadpool_info
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in threadpool_info()]
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "blas": blas}


def cpu_baseline(s_eff: int, nbox: int = 4) -> dict:
    """The oracle, as it stands, on a bounded sample of the same workload
    (symmetric variant, the headline's): `nbox` boxes of the first colour
    class of the first processed level, whose sketches are still the initial
    ones, each with its sketch rows Y_B = A_B Omega formed from the oracle's
    dense operator rows and its full step of Algorithm 1.  The measured
    oracle rate (work of those boxes by the work model of Sec. 4.5 over their
    time) prices the whole factorization, root and a 16-column solve; the
    sampling is scaled by rows (N / sampled rows)."""
    from threadpoolctl import threadpool_info
    from oracle import flops as ofl
    from oracle import rsrs as orr
    from oracle import tree as ot
    from paper_2311_01451_amd import inputs

    pts = inputs.grid2d(GRID_N)
    N = GRID_N ** 2
    h = 1.0 / GRID_N
    t = ot.build_tree(pts, LEAF)
    sch = ot.schedule(t, K)
    li = [i for i, c in enumerate(sch.order) if c][0]
    lev = sch.levels[li]
    cls0 = sch.order[li][0]
    step = max(1, len(cls0) // nbox)
    boxes = cls0[::step][:nbox]
    perm = t.perm
    Om_full = inputs.gaussian(N, s_eff, 0)
    Om = Om_full[perm]
    Y = np.zeros((N, s_eff))
    t_sample = t_factor = 0.0
    rows = 0
    done = []
    for box in boxes:
        nb = sch.nbrs[lev][box]
        Ba = np.arange(t.pt_begin[box], t.pt_end[box])
        Na = np.sort(np.concatenate([np.arange(t.pt_begin[x], t.pt_end[x]) for x in nb]))
        a = time.perf_counter()
        # sketch rows of the box: rows of the kernel matrix times Omega
        diff = pts[perm[Ba]][:, None, :] - pts[None, :, :]
        r = np.sqrt(np.sum(diff * diff, axis=2))
        with np.errstate(divide="ignore"):
            Arows = (h * h) * (-np.log(r) / (2 * np.pi))
        Arows[np.arange(len(Ba)), perm[Ba]] = 1.0 + 0.5 * h * h
        Y[Ba] = Arows @ Om_full
        t_sample += time.perf_counter() - a
        rows += len(Ba)
        del diff, r, Arows
        a = time.perf_counter()
        orr._process_box(int(box), lev, 0, Ba, Na, Y, Y, Om, Om, K, False, True)
        t_factor += time.perf_counter() - a
        done.append(ofl.box_work(len(Ba), len(Na), K, s_eff, symmetric=True))
    rate = sum(w.flops for w in done) / t_factor
    fw = ofl.factor_work(t, K, s_eff, symmetric=True)
    sf, _ = ofl.solve_work(fw, NRHS)
    est_factor = fw.flops / rate
    est_solve = sf / rate
    est_sample = t_sample * N / rows
    est = est_factor + est_solve + est_sample
    hi = host_info()
    threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    return {"value": round(NRHS / est, 6), "unit": "RHS cols/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"partial, priced: symmetric oracle on {len(done)} boxes of the first colour class of level {lev} "
                      f"(b={done[0].b}, l={done[0].b + done[0].n}, s={s_eff}; {t_factor:.1f} s, "
                      f"{rate / 1e9:.1f} GFLOP/s by the work model) and their {rows} sketch rows "
                      f"({t_sample:.1f} s); whole step priced at that rate by the work model "
                      f"(factor {fw.flops:.2e} flops -> {est_factor:.0f} s, 16-column solve "
                      f"{est_solve:.2f} s) and sampling scaled by rows ({est_sample:.0f} s)",
            "est_step_s": round(est, 1), "host": hi}


def cpu_oracle_config0(reps: int = 3) -> dict:
    """The whole oracle on the 64 x 64 workload (N = 4096, leaf 64,
    k = p = 32, s = max(320, s_required), general variant, FP64): dense
    sampling Y = A Omega, Z = A^T Psi, Algorithm 1, and a 16-column solve,
    timed end to end `reps` times with every BLAS thread (median reported)
    and once with one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import operators as oop
    from oracle import rsrs as orr
    from oracle import tree as ot
    from paper_2311_01451_amd import inputs

    n, k = 64, 32
    pts = inputs.grid2d(n)
    A = oop.log2d(pts, 1.0 / n)
    t = ot.build_tree(pts, LEAF)
    s = max(320, ot.samples_required(t, k, k))
    Om, Psi = inputs.test_matrices(n * n, s)
    f = inputs.rhs(n * n, NRHS)

    def once():
        a = time.perf_counter()
        F = orr.factor(t, A @ Om, A.T @ Psi, Om, Psi, k)
        b = time.perf_counter()
        orr.solve(F, f)
        c = time.perf_counter()
        return c - a, b - a, c - b

    all_threads = [once() for _ in range(reps)]
    with threadpool_limits(limits=1):
        one = once()
    med = sorted(all_threads)[len(all_threads) // 2]
    return {"workload": "64x64 log kernel (N=4096), leaf 64, k=p=32, s=%d, general variant, FP64: "
                        "sampling + Algorithm 1 + 16-column solve" % s,
            "all_threads_step_s": [round(x[0], 3) for x in all_threads], "median_step_s": round(med[0], 3),
            "median_factor_s": round(med[1], 3), "median_solve_s": round(med[2], 4),
            "one_thread_step_s": round(one[0], 3), "one_thread_factor_s": round(one[1], 3),
            "cols_per_s_median": round(NRHS / med[0], 4), "host": host_info()}


def serving_bench(duration_s: float, load: float = 0.7) -> dict:
    """Serving workload: a resident mixed-precision factor of the 3D kernel
    A_ij = delta_ij + (1/N) / (4 pi |x_i - x_j|) on N = 32768 uniform random
    points in [0,1]^3 (adaptive octree, leaf 64, k = p = 128), behind the
    continuous-batching server with a 24 GB HBM budget.  A Poisson stream of
    requests: 90% solves with widths uniform in {1, 4, 16, 64, 256} (N(0,1)
    entries), 10% new-factor requests for 64 x 64 jittered-grid log-kernel
    operators (k = p = 32, mixed precision), each used for one 16-column solve
    and then released.  The arrival rate is `load` times the saturated solve
    request rate measured first with a burst."""
    import threading

    import torch
    from paper_2311_01451_amd import inputs, rsrs

    rng = np.random.default_rng(inputs.BASE_SEED + 5)
    N, K4 = 32768, 128
    pts = inputs.uniform_points(N, 3)
    t0 = time.perf_counter()
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_INVR3D, pts)
    tree = rsrs.rsrs_build_tree(pts, LEAF)
    s_req = tree.samples_required(K4, K4)
    s = max(2048, s_req)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    smp = rsrs.rsrs_sample(tree, op, s, inputs.BASE_SEED, dtype=rsrs.RSRS_BF16)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    F = rsrs.rsrs_factor(tree, smp, K4, precision=rsrs.RSRS_PREC_F32_MIXED)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    del smp
    f16 = torch.tensor(inputs.rhs(N, 16), dtype=torch.float64, device="cuda")
    _, rel, it = rsrs.rsrs_solve_refine(F, op, f16, tol=TOL, maxit=30)
    fi = F.info()
    budget = 24 << 30
    sv = rsrs.Server(hbm_budget=budget, max_batch_cols=1024)
    fid = sv.add_factor(F)
    # served solves are refined through the FP64 operator to the metric's
    # tolerance (the server reports the largest residual a batch ended with)
    sv.set_refine(fid, op, tol=TOL, maxit=10)
    widths = [1, 4, 16, 64, 256]
    pool = {w: torch.randn((N, w), dtype=torch.float64, device="cuda") for w in widths}
    # operators for the new-factor requests (built up front: creating one
    # synchronises the device, which would stall the arrival process)
    n0 = 64
    small = []
    for j in range(8):
        p0 = inputs.jittered_grid2d(n0, seed_offset=500 + j)
        t0s = rsrs.rsrs_build_tree(p0, LEAF)
        small.append((t0s, rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, p0, 1.0 / n0),
                      t0s.samples_required(32, 32)))
    f0 = torch.tensor(inputs.rhs(n0 * n0, 16), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    # saturated solve throughput: a burst of solve requests only
    burst = [int(rng.choice(widths)) for _ in range(200)]
    sv.stats(reset=True)
    a = time.perf_counter()
    tk = [sv.submit_solve(fid, pool[w], torch.empty_like(pool[w]))[0] for w in burst]
    for t in tk:
        sv.wait(t)
    sat_s = time.perf_counter() - a
    sat = sv.stats(reset=True)

    jnext = [0]

    def submit_factor():
        t0s, op0, s0 = small[jnext[0] % len(small)]
        jnext[0] += 1
        return (sv.submit_factor(t0s, op0, s0, inputs.BASE_SEED + jnext[0], 32,
                                 precision=rsrs.RSRS_PREC_F32_MIXED, dtype=rsrs.RSRS_BF16), op0)

    def use_and_release(tk_op):
        t, op0 = tk_op
        fid2, lat = sv.wait(t)
        sv.set_refine(fid2, op0, tol=TOL, maxit=10)
        tk2, _ = sv.submit_solve(fid2, f0)
        sv.wait(tk2)
        sv.release(fid2)
        return lat

    # saturated rate of the request mix (90% solves, 10% new factors)
    kinds = [rng.random() < 0.1 for _ in range(300)]
    a = time.perf_counter()
    tk, fk = [], []
    for is_f in kinds:
        if is_f:
            fk.append(submit_factor())
        else:
            w = int(rng.choice(widths))
            tk.append(sv.submit_solve(fid, pool[w], torch.empty_like(pool[w]))[0])
    for t in tk:
        sv.wait(t)
    for t in fk:
        use_and_release(t)
    mix_s = time.perf_counter() - a
    sv.stats(reset=True)
    mix_rate = len(kinds) / mix_s
    lam = load * mix_rate

    # Poisson stream at `load` times the saturated rate of the mix
    lock = threading.Lock()
    fact_tickets = []
    done_submitting = threading.Event()

    def factor_client():
        while True:
            with lock:
                t = fact_tickets.pop(0) if fact_tickets else None
            if t is None:
                if done_submitting.is_set():
                    with lock:
                        if not fact_tickets:
                            return
                    continue
                time.sleep(0.001)
                continue
            use_and_release(t)

    th = threading.Thread(target=factor_client)
    th.start()
    tickets = []
    nfact = 0
    start = time.perf_counter()
    tnext = start
    while True:
        tnext += rng.exponential(1.0 / lam)
        if tnext - start > duration_s:
            break
        d = tnext - time.perf_counter()
        if d > 0:
            time.sleep(d)
        if rng.random() < 0.1:
            t = submit_factor()
            with lock:
                fact_tickets.append(t)
            nfact += 1
        else:
            w = int(rng.choice(widths))
            tickets.append(sv.submit_solve(fid, pool[w], torch.empty_like(pool[w]))[0])
    for t in tickets:
        sv.wait(t)
    solves_end = time.perf_counter()
    done_submitting.set()
    th.join()
    elapsed = time.perf_counter() - start
    st = sv.stats()
    sv.close()
    return {
        "workload": f"3D kernel delta_ij + (1/N)/(4 pi r), N={N} uniform random points, adaptive octree "
                    f"leaf {LEAF}, k=p={K4}, s={s} (configured 2048, required {s_req}), mixed precision "
                    "(BF16 sample products), "
                    "resident; Poisson stream of solves (widths {1,4,16,64,256}) with 10% new-factor "
                    "requests (64x64 jittered log kernel, k=32), HBM budget 24 GB",
        "factor_s": round(t3 - t2, 3), "sample_s": round(t2 - t1, 3),
        "factor_tflops_algorithmic": round(fi["flops"] / (t3 - t2) / 1e12, 3),
        "stored_gb": round(fi["stored_bytes"] / 1e9, 3),
        "refine": {"relres": rel, "iters": it},
        "saturated_solves": {"requests_per_s": round(len(burst) / sat_s, 1),
                      "cols_per_s": round(sat["cols_done"] / sat_s, 1),
                      "solve_p50_ms": round(sat["solve_p50_ms"], 3),
                      "solve_p99_ms": round(sat["solve_p99_ms"], 3),
                      "mean_batch_cols": round(sat["cols_done"] / max(sat["batches"], 1), 1)},
        "saturated_mix_requests_per_s": round(mix_rate, 1),
        "load": load, "arrival_rate_per_s": round(lam, 1), "duration_s": round(elapsed, 2),
        "solves": st["solves_done"], "factors": st["factors_done"], "factor_requests": nfact,
        "cols_per_s": round(st["cols_done"] / (solves_end - start), 1),
        "solve_p50_ms": round(st["solve_p50_ms"], 3), "solve_p99_ms": round(st["solve_p99_ms"], 3),
        "factor_p50_ms": round(st["factor_p50_ms"], 3), "factor_p99_ms": round(st["factor_p99_ms"], 3),
        "mean_batch_cols": round(st["cols_done"] / max(st["batches"], 1), 1),
        "hbm_peak_gb": round(st["hbm_peak"] / 1e9, 3),
        "served_solves": f"refined through the FP64 operator to {TOL:g}",
        "refined_batches": st.get("refined_batches"), "refine_steps": st.get("refine_steps"),
        "served_max_relres": st.get("max_relres"),
        "saturated_served_max_relres": sat.get("max_relres"),
    }


def config0_leg(steps: int = 3) -> dict:
    """Plain FP64 RSRS (general two-sided algorithm) on the 64 x 64 grid:
    N = 4096, leaf 64, k = p = 32, s = max(320, s_required), 16 right-hand
    sides refined to 1e-10 through the FP64 operator.  Factor time, RHS
    columns per second of the whole step (sampling, factor, refined solve)."""
    import torch
    from paper_2311_01451_amd import inputs, rsrs

    n, k = 64, 32
    pts = inputs.grid2d(n)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
    f = torch.tensor(inputs.rhs(n * n, NRHS), dtype=torch.float64, device="cuda")
    rec = []
    for it_ in range(steps + 1):
        torch.cuda.synchronize()
        a = time.perf_counter()
        tc = rsrs.rsrs_build_tree(pts, LEAF)
        s = max(320, tc.samples_required(k, k))
        smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=rsrs.RSRS_F64)
        torch.cuda.synchronize()
        b = time.perf_counter()
        F = rsrs.rsrs_factor(tc, smp, k)
        torch.cuda.synchronize()
        c = time.perf_counter()
        u, rel, its = rsrs.rsrs_solve_refine(F, op, f, tol=1e-10, maxit=10)
        torch.cuda.synchronize()
        d = time.perf_counter()
        if it_ > 0:   # the first step warms up
            rec.append((d - a, c - b, rel, its, s))
    step_s = float(np.mean([r[0] for r in rec]))
    return {"workload": "2D log kernel on the 64x64 grid (N=4096), leaf 64, k=p=32, FP64, general variant, "
                        "16 RHS refined to 1e-10",
            "s": rec[-1][4], "steps": steps, "cols_per_s": round(NRHS / step_s, 2),
            "ms_per_step": round(step_s * 1e3, 3), "factor_s": round(float(np.mean([r[1] for r in rec])), 4),
            "relres": rec[-1][2], "refine_iters": rec[-1][3]}


def config2_leg() -> dict:
    """3D variable-coefficient Poisson, mixed precision: 7-point
    -div(a grad u) on the 48^3 interior grid (N = 110592), a = exp(box3(g)),
    octree leaves of 4^3 nodes, k = p = 96, s = max(1200, s_required), FP32
    samples through the sparse product, 16 right-hand sides refined to 1e-8
    with the FP64 sparse residual.  One step (sampling, factor, refined
    solve), with the fixed rank and with a rank tolerance of 1e-7."""
    import torch
    from paper_2311_01451_amd import inputs, rsrs

    n, k = 48, 96
    h = 1.0 / (n + 1)
    pts = inputs.grid3d_interior(n)
    coef = inputs.smooth_log_coefficient(n + 2)
    op = rsrs.rsrs_op_create_poisson7(n, coef)
    f = torch.tensor(inputs.rhs(n ** 3, NRHS), dtype=torch.float64, device="cuda")
    out = {"workload": "3D Poisson -div(a grad u), 48^3 interior nodes (N=110592), leaves 4^3, k=p=96, "
                       "mixed precision (FP32 samples and products, FP64 pivots and residual), 16 RHS "
                       "refined to 1e-8"}
    for label, tol in (("fixed_rank", 0.0), ("rank_tol_1e-7", 1e-7)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        tc = rsrs.rsrs_build_tree(pts, LEAF, root_lo=[h / 2] * 3, root_side=64 * h)
        s = max(1200, tc.samples_required(k, k))
        smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=rsrs.RSRS_F32)
        torch.cuda.synchronize()
        b = time.perf_counter()
        F = rsrs.rsrs_factor(tc, smp, k, precision=rsrs.RSRS_PREC_F32_MIXED, rank_tol=tol)
        del smp
        torch.cuda.synchronize()
        c = time.perf_counter()
        u, rel, its = rsrs.rsrs_solve_refine(F, op, f, tol=1e-8, maxit=30)
        torch.cuda.synchronize()
        d = time.perf_counter()
        info = F.info()
        out[label] = {"s": s, "sample_s": round(b - a, 3), "factor_s": round(c - b, 3),
                      "solve_refine_s": round(d - c, 3), "cols_per_s": round(NRHS / (d - a), 3),
                      "relres": rel, "refine_iters": its,
                      "factor_tflops_algorithmic": round(info["flops"] / (c - b) / 1e12, 3),
                      "stored_gb": round(info["stored_bytes"] / 1e9, 3)}
        del F
    return out


def config3_leg() -> dict:
    """The many-problem workload: 48 jittered 2D log-kernel problems (N
    log-uniform from about 2,000 to 33,000, k in {32, 48, 64}, leaf 64,
    s = s_required, FP32 samples and products with FP64 pivots), factored
    by one batched call; 16 right-hand sides per problem refined to 1e-6
    through each problem's FP64 operator.  Beside it, the same problems
    factored one at a time."""
    import torch
    from paper_2311_01451_amd import inputs, rsrs

    specs = inputs.uneven_batch()
    trees, ks, ss, model = [], [], [], 0.0
    for P in specs:
        P["pts"] = inputs.jittered_grid2d(P["n"], seed_offset=P["geom_seed"])
        tc = rsrs.rsrs_build_tree(P["pts"], LEAF)
        s = tc.samples_required(P["k"], P["k"])
        trees.append(tc)
        ks.append(P["k"])
        ss.append(s)
        model += rsrs.rsrs_work_model(tc, P["k"], s, False, 4)["flops"]

    def samples():
        out = []
        for P, tc, s in zip(specs, trees, ss):
            op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, P["pts"], 1.0 / P["n"])
            out.append(rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED + P["seed"], dtype=rsrs.RSRS_F32))
            torch.cuda.synchronize()
            del op
        return out

    smps = samples()
    torch.cuda.synchronize()
    a = time.perf_counter()
    Fs = rsrs.rsrs_factor_batched(trees, smps, ks, precision=rsrs.RSRS_PREC_F32_MIXED)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - a
    del smps
    t_ref, worst, iters = 0.0, 0.0, []
    for P, F in zip(specs, Fs):
        op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, P["pts"], 1.0 / P["n"])
        f = torch.tensor(inputs.rhs(P["n"] ** 2, NRHS, P["seed"]), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        a = time.perf_counter()
        u, rel, it = rsrs.rsrs_solve_refine(F, op, f, tol=TOL, maxit=30)
        torch.cuda.synchronize()
        t_ref += time.perf_counter() - a
        worst = max(worst, rel)
        iters.append(it)
        del op
    del Fs
    smps = samples()
    t_single = 0.0
    for tc, smp, k in zip(trees, smps, ks):
        torch.cuda.synchronize()
        a = time.perf_counter()
        F = rsrs.rsrs_factor(tc, smp, k, precision=rsrs.RSRS_PREC_F32_MIXED)
        torch.cuda.synchronize()
        t_single += time.perf_counter() - a
        del F
    del smps
    Ns = [P["n"] ** 2 for P in specs]
    return {"workload": f"{len(specs)} jittered 2D log-kernel problems, N log-uniform in [{min(Ns)}, {max(Ns)}] "
                        f"(total {sum(Ns)}), k in {{32, 48, 64}}, leaf 64, s = s_required, mixed precision, "
                        "16 RHS each refined to 1e-6",
            "batch_factor_s": round(t_batch, 4), "one_at_a_time_factor_s": round(t_single, 4),
            "batch_speedup": round(t_single / t_batch, 3),
            "refine_s_all": round(t_ref, 4), "cols_per_s": round(NRHS * len(specs) / (t_batch + t_ref), 2),
            "worst_relres": worst, "refine_iters_max": int(max(iters)),
            "factor_tflops_work_model": round(model / t_batch / 1e12, 3)}


def factor_options_leg(ctx: dict) -> dict:
    """The factor options beside the default (all s columns, fixed rank k),
    one step each after one warm-up:
      * per-box column subsets (a box reads its first s_B = min(s, l + k + p)
        sample columns in its nullification, ID and extraction);
      * a rank tolerance (k_B = the numerical rank of the ID's sketch relative
        to ||[Y_B Z_B]||, capped at k);
    on the 64 x 64 grid in FP64 (general variant, k = p = 32: factor time and
    the factorization's relerr ||A - A_approx|| / ||A|| from the dense apply)
    and on the headline workload (256 x 256, mixed, symmetric: sampling +
    factor time, one-shot residual, refinement steps to 1e-6, columns per
    second)."""
    import torch
    from paper_2311_01451_amd import inputs, rsrs

    variants = (("default", {}), ("col_subset", {"col_subset": True}))
    out = {}
    n, k = 64, 32
    pts = inputs.grid2d(n)
    op0 = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
    eye = torch.eye(n * n, dtype=torch.float64, device="cuda")
    A = op0.matvec(eye)
    nA = float(torch.linalg.matrix_norm(A, 2))
    c0 = {}
    for label, kw in variants + (("rank_tol_1e-10", {"rank_tol": 1e-10}),):
        for rep in range(2):
            tc = rsrs.rsrs_build_tree(pts, LEAF)
            s = max(320, tc.samples_required(k, k))
            smp = rsrs.rsrs_sample(tc, op0, s, inputs.BASE_SEED, dtype=rsrs.RSRS_F64)
            torch.cuda.synchronize()
            a = time.perf_counter()
            F = rsrs.rsrs_factor(tc, smp, k, **kw)
            torch.cuda.synchronize()
            b = time.perf_counter()
        Aap = F.apply(eye)
        c0[label] = {"factor_ms": round((b - a) * 1e3, 3),
                     "relerr": float(torch.linalg.matrix_norm(A - Aap, 2)) / nA,
                     "stored_mb": round(F.info()["stored_bytes"] / 1e6, 2)}
        if "rank_tol" not in kw:
            c0[label]["work_model_gflop"] = round(
                rsrs.rsrs_work_model(tc, k, s, False, 8, col_subset=bool(kw.get("col_subset")))["flops"] / 1e9, 2)
        del F, Aap
    del A, eye
    out["config0_fp64_k32"] = c0
    op, f = ctx["op"], ctx["f"]
    pts1 = inputs.grid2d(GRID_N)
    c1 = {}
    for label, kw in variants + (("rank_tol_1e-6", {"rank_tol": 1e-6}),):
        for rep in range(2):
            tc = rsrs.rsrs_build_tree(pts1, LEAF)
            s = max(S_CFG, tc.samples_required(K, K))
            torch.cuda.synchronize()
            a = time.perf_counter()
            smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=rsrs.RSRS_BF16, symmetric=True)
            F = rsrs.rsrs_factor(tc, smp, K, precision=rsrs.RSRS_PREC_F32_MIXED, symmetric=True, **kw)
            torch.cuda.synchronize()
            b = time.perf_counter()
            u0 = F.solve(f)
            r0 = float(torch.linalg.norm(f - op.matvec(u0)) / torch.linalg.norm(f))
            torch.cuda.synchronize()
            c = time.perf_counter()
            u, rel, its = rsrs.rsrs_solve_refine(F, op, f, tol=TOL, maxit=30)
            torch.cuda.synchronize()
            d = time.perf_counter()
            del smp
        c1[label] = {"sample_factor_ms": round((b - a) * 1e3, 3), "relres_oneshot": r0, "relres": rel,
                     "refine_iters": its, "cols_per_s": round(NRHS / ((b - a) + (d - c)), 2),
                     "stored_mb": round(F.info()["stored_bytes"] / 1e6, 1)}
        if "rank_tol" not in kw:
            c1[label]["work_model_gflop"] = round(
                rsrs.rsrs_work_model(tc, K, s, True, 4, col_subset=bool(kw.get("col_subset")))["flops"] / 1e9, 2)
        del F
    out["headline_mixed_symmetric"] = c1
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-reps", type=int, default=40)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--reproject", type=int, default=0, choices=(0, 1),
                    help="second projection pass in the factorization (the refinement reaches "
                         "the tolerance in one step either way)")
    ap.add_argument("--modes", default="mixed,mixed_general,fp64,fp64_general",
                    help="comma list of the precision/variant runs (the first is the headline)")
    ap.add_argument("--serving", type=float, default=0.0,
                    help="run only the serving workload for this many seconds and print its line")
    ap.add_argument("--serving-seconds", type=float, default=8.0,
                    help="length of the Poisson stream of the serving leg in the default run")
    ap.add_argument("--cpu-config0", action="store_true",
                    help="only time the whole oracle on the 64x64 workload on the host (median of 3, "
                         "and one thread) and print its line")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in GEMM tile rule instead of tuning each run's launches first")
    ap.add_argument("--no-configs", action="store_true",
                    help="leave out the legs of the other workloads (configs 0, 2 and 4)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {a.gpus}); "
              "a sharded run across GPUs is not part of this benchmark", file=sys.stderr)
        sys.exit(2)
    if a.cpu_config0:
        print(json.dumps({"metric": "oracle on the host, 64x64 workload", **cpu_oracle_config0()}))
        return
    if a.serving > 0:
        out = {"metric": "serving: p50/p99 solve latency (ms) and RHS cols/s under Poisson arrivals",
               "n_gpus": 1, "data": "synthetic"}
        out.update(serving_bench(a.serving))
        print(json.dumps(out))
        return
    ctx = {}
    runs = {}
    plan = (("mixed", "bf16", True), ("mixed_general", "bf16", False),
            ("fp64", "fp64", True), ("fp64_general", "fp64", False))
    want = a.modes.split(",")
    tune = None
    if not a.no_autotune:
        # tile choice of every GEMM launch of each run's factorization, timed on
        # that workload (Gaussian samples, untimed)
        from paper_2311_01451_amd import inputs as _in, rsrs as _r
        t0 = time.perf_counter()
        tc = _r.rsrs_build_tree(_in.grid2d(GRID_N), LEAF)
        s_t = max(S_CFG, tc.samples_required(K, K))
        tune = {}
        for name, mode, sym in plan:
            if name in want:
                prec = _r.RSRS_PREC_F64 if mode == "fp64" else _r.RSRS_PREC_F32_MIXED
                tune[name] = _r.rsrs_gemm_autotune_workload(tc, K, s_t, precision=prec, symmetric=sym,
                                                             reproject=a.reproject)
        tune["seconds"] = round(time.perf_counter() - t0, 3)
    for name, mode, sym in plan:
        if name not in want:
            continue
        runs[name] = gpu_bench(a.steps, a.warmup, not a.no_profile, a.latency_reps,
                               a.calib_copy_mib if name == "mixed" else 0, mode, ctx, sym, a.reproject)
    def summary(rec, elapsed, profs, lats, steps):
        prof, prof_all = profs
        lat, latr = lats
        fs = float(np.mean([r["factor"] for r in rec]))
        return {
            "value": round(NRHS * steps / elapsed, 4),
            "ms_per_step": round(elapsed / steps * 1e3, 3),
            "factor_s": round(float(np.mean([r["factor"] for r in rec])), 4),
            "sample_s": round(float(np.mean([r["sample"] for r in rec])), 4),
            "solve_refine_ms": round(float(np.mean([r["solve"] for r in rec])) * 1e3, 3),
            "refine_iters": int(rec[-1]["iters"]),
            "relres": rec[-1]["relres"],
            "relres_oneshot": rec[-1]["relres_oneshot"],
            # the kernels' own flop count, and the method's (work model of Sec. 4.5)
            "factor_tflops_algorithmic": round(rec[-1]["flops"] / fs / 1e12, 3),
            "factor_tflops_work_model": round(rec[-1]["model_flops"] / fs / 1e12, 3),
            "oneshot_solve_ms_p50": round(float(np.percentile(lat, 50)), 3),
            "oneshot_solve_ms_p99": round(float(np.percentile(lat, 99)), 3),
            "refined_solve_ms_p50": round(float(np.percentile(latr, 50)), 3),
            "refined_solve_ms_p99": round(float(np.percentile(latr, 99)), 3),
            "refined_solve_cols_per_s": round(NRHS / (float(np.median(latr)) * 1e-3), 1),
            "roofline": roofline_from_profile(prof, prof_all, steps),
            "roofline_factor_kernel": per_level_roofline(prof_all),
            "kernels_one_step": {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                                     "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3)}
                                 for k, v in sorted(prof_all.items(), key=lambda kv: -kv[1]["ms"])[:14]},
            "gpu_ms_one_step": round(sum(v["ms"] for v in prof_all.values()), 3),
        }

    if "mixed" not in runs:
        print("bench.py: the headline run 'mixed' must be among --modes", file=sys.stderr)
        sys.exit(2)
    sums = {name: summary(*r, a.steps) for name, r in runs.items()}
    sm = sums["mixed"]
    rec = runs["mixed"][0]
    s_req, s_eff = rec[-1]["s_req"], rec[-1]["s_eff"]
    out = {
        "metric": METRIC,
        "value": sm["value"],
        "unit": "RHS cols/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": sm["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32",
        "data": "synthetic",
        "config": workload_config(s_req, s_eff, a.reproject),
    }
    out.update({k: v for k, v in sm.items() if k not in ("value", "ms_per_step")})
    out["gemm_autotune"] = tune
    for name in ("mixed_general", "fp64", "fp64_general"):
        if name in sums:
            keep = name == "fp64"
            out[name] = {k: v for k, v in sums[name].items() if keep or k != "kernels_one_step"}
    if "fp64" in runs:
        ua, ub = runs["mixed"][0][-1]["u"], runs["fp64"][0][-1]["u"]
        out["mixed_vs_fp64"] = {"speedup": round(sm["value"] / sums["fp64"]["value"], 3),
                                "factor_speedup": round(sums["fp64"]["factor_s"] / sm["factor_s"], 3),
                                "solution_rel_diff": float(((ua - ub).norm() / ub.norm()).item())}
    if not a.no_configs:
        import torch
        out["configs"] = {}
        for name, fn in (("config0_fp64", config0_leg), ("config2_poisson_mixed", config2_leg),
                         ("config3_batch_mixed", config3_leg)):
            out["configs"][name] = fn()
            torch.cuda.synchronize()
        out["configs"]["config4_serving"] = serving_bench(a.serving_seconds)
        out["factor_options"] = factor_options_leg(ctx)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s_eff)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
