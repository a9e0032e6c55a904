#!/usr/bin/env python3
"""Throughput of the fast direct high-order FEM solve on one MI355X.

Headline workload large_2d: -Lap u = f on [0,1]^2 with Dirichlet data,
Lagrange order n = 9, K = 1024 elements per axis, (9*1024-1)^2 = 84,916,225
unknowns, f^h i.i.d. uniform[-1,1) (seed 0), resident in HBM before timing
starts.  A step is one whole solve (every pass of algorithm (a)).  `value`
is the FP64 solve's unknowns/s.

Beside it, on the same input: the FP32-transform solve with FP64
refinement (fixed step count, no host synchronisation), the FP32-
preconditioned conjugate-gradient form (FP64 residuals, stops on a relative
update of 1e-13), the unrefined FP32 solve, and their relative l2 distances
to the FP64 solution.  Per-pass durations come from HIP events the library
records around each kernel on the stream it runs on; `roofline` reports the
pass that takes most time.

Further workloads (one entry each under other_workloads):
  batch_2d    256 independent 2D problems (K in {32..256}, n in {2..6}, 4 RHS
              each), one batched call replayed from a HIP graph;
  cube_3d     3D n = 4, K = 128 (511^3 unknowns), Gauss load of a manufactured f plus noise;
  varcoef_3d  -div(a grad u) = f, 3D n = 3, K = 64, PCG to 1e-10.

`cpu_baseline` times the CPU oracle (dense eigenvector products along both
axes) on the host for the whole large_2d right-hand side; since it is exact
it also yields the FP64 parity figure of the run.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only NAMES]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
# the line-pass sources: their hash keys the committed HBM counter summary
# (and the autotuner's cache)
KERNEL_SOURCES = ("linepass.h", "linepass.hip", "linepass_dispatch.hip", "kernels.h")


def kernel_sha():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1609_07758_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kind):
    """HBM bytes per launch of the dominant pass from the committed rocprofv3
    counter summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_sha():
        return None
    entry = d.get("passes", {}).get(kind)
    return None if entry is None else entry.get("hbm_bytes_per_launch")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_calls(torch, fn, steps, warmup, stream=None):
    """Mean milliseconds per call of fn, HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, f_host, u_gpu64, others):
    """Time the oracle's dense solve on the host; return the record and the
    parity of the GPU solutions against it."""
    import numpy as np
    from oracle import solve as osolve, spectral

    t0 = time.perf_counter()
    for n, K in zip(cfg["orders"], cfg["Ks"]):
        spectral.basis(n, K)             # eigen data (cached) and dense V
    t_setup = time.perf_counter() - t0
    # whole right-hand sides through the oracle until about 10 s of CPU work
    # (at most three); the first one also serves the parity figures
    t_apply, reps = 0.0, 0
    while reps < 3 and (reps == 0 or t_apply < 10.0):
        t0 = time.perf_counter()
        ref = osolve.solve(f_host, cfg["orders"], cfg["Ks"], cfg["X"], cfg["alpha"])
        t_apply += time.perf_counter() - t0
        reps += 1
    M = ref.size
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 0) for p in threadpool_info()), default=cores)
    except Exception:
        threads = cores
    nref = np.linalg.norm(ref)
    parity = {"fp64_rel_l2": float(np.linalg.norm(u_gpu64 - ref) / nref)}
    for name, u in others.items():
        parity[name + "_rel_l2"] = float(np.linalg.norm(u - ref) / nref)
    rec = {"value": M * reps / t_apply, "unit": "unknowns/s", "cores": int(threads), "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{reps} solves of the whole {cfg['name']} right-hand side ({M} unknowns) "
                     f"through the oracle's dense eigenvector products (FP64, {t_apply:.1f} s); "
                     f"eigen data and dense V construction timed apart: {t_setup:.1f} s"}
    return rec, parity


def bench_headline(args, torch, H, np, workloads, dev):
    cfg = dict(workloads.CONFIGS["large_2d"])
    cfg["name"] = "large_2d"
    shp = workloads.shape(cfg["orders"], cfg["Ks"])
    M = int(np.prod(shp))
    f_host = workloads.uniform_rhs(shp, seed=0)
    f64 = torch.from_numpy(f_host).to(dev)
    f32 = f64.float()
    S = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], cfg["alpha"])
    u64 = torch.empty_like(f64)
    uir = torch.empty_like(f64)
    upcg = torch.empty_like(f64)
    u32 = torch.empty_like(f32)
    ws_ir = S.workspace("fp32_ir")
    ws_pcg = S.workspace("fp32_pcg")
    torch.cuda.synchronize()
    log("large_2d: FP64")

    # FP64 solve (the headline figure), with per-pass event timing.
    S.set_timing(True)
    for _ in range(args.warmup):
        S.solve(f64, u64, mode="fp64")
    S.pass_times()
    ms64 = time_calls(torch, lambda: S.solve(f64, u64, mode="fp64"), args.steps, 0)
    passes64 = S.pass_times()
    S.set_timing(False)

    if args.profile_fp64:
        # counter runs: the FP64 solves alone
        S.close()
        return {"value": M / (ms64 * 1e-3), "ms_per_step": ms64,
                "config": {"workload": "large_2d", "profile_fp64_only": True}}

    # attainable HBM bandwidth on this GPU: a plain 1 GiB device copy (read
    # and write), beside the 8 TB/s specification peak
    ca = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    cb = torch.empty_like(ca)
    ms_copy = time_calls(torch, lambda: cb.copy_(ca), 10, 2)
    copy_gbs = 2.0 * ca.numel() * 8 / (ms_copy * 1e-3) / 1e9
    del ca, cb

    log("large_2d: algorithm (b)")
    ub = torch.empty_like(f64)
    S.set_timing(True)
    ms_b = time_calls(torch, lambda: S.solve(f64, ub, mode="fp64_b"), args.steps, args.warmup)
    passes_b = S.pass_times()
    S.set_timing(False)

    log("large_2d: implicit heat steps and the Dirichlet lift")
    # implicit time stepping (backward Euler, dt = 1e-3: alpha = 1000) and
    # the boundary lift of Dirichlet data, at the same size
    Sh = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], 1000.0)
    Th = H.Stepper(Sh, "heat")
    uh = f64.clone()
    sh_stream = torch.cuda.Stream()
    with torch.cuda.stream(sh_stream):
        Th.run(uh, 2, f=f64, use_graph=True, stream=sh_stream.cuda_stream)
        ms_heat = time_calls(torch, lambda: Th.run(uh, 10, f=f64, use_graph=True,
                                                    stream=sh_stream.cuda_stream), 2, 1,
                             sh_stream) / 10
    torch.cuda.synchronize()
    Th.close()
    Sh.close()
    bext = torch.rand(tuple(m + 2 for m in shp), dtype=torch.float64, device=dev)
    lift = torch.empty_like(f64)
    ms_lift = time_calls(torch, lambda: S.dirichlet_rhs(bext, f64, out=lift), args.steps,
                         args.warmup)
    del bext, lift, uh

    log("large_2d: periodic, Neumann and non-power-of-two axes")
    # the same orders and meshes with both axes periodic (alpha = 1): Bloch
    # waves, m = nK per axis
    Sp = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], 1.0, bcs=("periodic", "periodic"))
    fp = torch.rand(Sp.size, dtype=torch.float64, device=dev)
    up = torch.empty_like(fp)
    Sp.set_timing(True)
    ms_per = time_calls(torch, lambda: Sp.solve(fp, up, mode="fp64"), args.steps, args.warmup)
    passes_per = Sp.pass_times()
    Sp.set_timing(False)
    M_per = Sp.size
    Sp.close()
    del fp, up
    # Neumann axes with the same orders and meshes (alpha = 1): m = nK + 1
    # per axis, cosine passes with the band-edge blocks
    Sn = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], 1.0, bcs=("neumann", "neumann"))
    fn_ = torch.rand(Sn.size, dtype=torch.float64, device=dev)
    un_ = torch.empty_like(fn_)
    Sn.set_timing(True)
    ms_neu = time_calls(torch, lambda: Sn.solve(fn_, un_, mode="fp64"), args.steps, args.warmup)
    passes_neu = Sn.pass_times()
    Sn.set_timing(False)
    M_neu = Sn.size
    Sn.close()
    del fn_, un_
    # K not a power of two (n = 9, K = 384 per axis): dense eigenvector
    # transforms on the FP64 matrix cores, four m^3 products per solve
    Sd = H.Solver(cfg["orders"], (384, 384), cfg["X"], cfg["alpha"])
    fd_ = torch.rand(Sd.size, dtype=torch.float64, device=dev)
    ud_ = torch.empty_like(fd_)
    wsd = Sd.workspace("fp64")
    ms_dense = time_calls(torch, lambda: Sd.solve(fd_, ud_, mode="fp64", ws=wsd), args.steps, args.warmup)
    m_d = Sd.shape[0]
    M_dense = Sd.size
    Sd.close()
    del fd_, ud_, wsd

    log("large_2d: autotuned launch shapes (FP64)")
    tune = S.autotune("fp64", nrhs=1, reps=3, f=f64, u=u64)
    ms64_tuned = time_calls(torch, lambda: S.solve(f64, u64, mode="fp64"), args.steps, args.warmup)
    H.hofem_solver_tune_reset(S.handle)
    S.solve(f64, u64, mode="fp64")

    log("large_2d: FP32 + refinement")
    S.set_timing(True)
    ms_ir = time_calls(torch, lambda: S.solve(f64, uir, mode="fp32_ir", ws=ws_ir,
                                              max_iter=args.ir_iters, tol=0.0),
                       args.steps, args.warmup)
    passes_ir = S.pass_times()
    S.set_timing(False)
    ms32 = time_calls(torch, lambda: S.solve(f32, u32, mode="fp32"), args.steps, args.warmup)

    log("large_2d: FP32-preconditioned CG")
    pcg_info = {}

    def pcg():
        _, info, _ = S.solve(f64, upcg, mode="fp32_pcg", ws=ws_pcg, max_iter=30, tol=1e-13,
                             want_info=True, raise_noconv=False)
        pcg_info["it"] = info.iterations
        pcg_info["upd"] = info.rel_update
        pcg_info["res"] = info.rel_residual
    ms_pcg = time_calls(torch, pcg, max(1, args.steps // 4), 1)

    nrm = torch.linalg.vector_norm(u64)
    dist = lambda u: float(torch.linalg.vector_norm(u.double() - u64) / nrm)
    hist = []
    tmp = torch.empty_like(f64)
    for it in range(0, 6):
        S.solve(f64, tmp, mode="fp32_ir", ws=ws_ir, max_iter=it, tol=0.0)
        hist.append(dist(tmp))
    torch.cuda.synchronize()

    dom = max(passes64, key=lambda p: p["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    achieved = dom["bytes"] / (avg_ms * 1e-3) / 1e9
    kind = f"{dom['kind']}_axis{dom['axis']}_fp64"
    traffic = measured_traffic("large_2d", kind)
    tot_bytes = sum(p["bytes"] * p["launches"] for p in passes64)
    tot_ms = sum(p["ms"] for p in passes64)
    rec = {
        "value": M / (ms64 * 1e-3),
        "ms_per_step": ms64,
        "hbm_all_passes": {"algorithmic_bytes_per_solve": tot_bytes / max(1, args.steps),
                           "gbs": tot_bytes / (tot_ms * 1e-3) / 1e9,
                           "frac": tot_bytes / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "frac_of_copy": tot_bytes / (tot_ms * 1e-3) / 1e9 / copy_gbs},
        "hbm_copy": {"bytes_per_copy": 2 * (1 << 30), "ms": ms_copy, "gbs": copy_gbs,
                     "frac_of_peak": copy_gbs / HBM_PEAK_GBS,
                     "note": "plain 1 GiB device-to-device copy: the attainable HBM rate"},
        "algorithm_b": {"unknowns_per_s": M / (ms_b * 1e-3), "ms_per_step": ms_b,
                        "passes": [dict(p, avg_ms=p["ms"] / p["launches"]) for p in passes_b]},
        "autotune_fp64": {"ms_default": ms64, "ms_tuned": ms64_tuned, "passes": tune},
        "heat_steps": {"alpha": 1000.0, "ms_per_step": ms_heat,
                       "unknowns_per_s": M / (ms_heat * 1e-3),
                       "note": "backward Euler step: mass update + FP64 solve, HIP-graph replay"},
        "dirichlet_lift": {"ms": ms_lift, "unknowns_per_s": M / (ms_lift * 1e-3)},
        "dense_fp64": {"unknowns": M_dense, "orders": cfg["orders"], "K_per_axis": 384,
                       "ms_per_step": ms_dense, "unknowns_per_s": M_dense / (ms_dense * 1e-3),
                       "tflops": 8.0 * m_d ** 3 / (ms_dense * 1e-3) / 1e12,
                       "tflops_frac_of_fp64_mfma": 8.0 * m_d ** 3 / (ms_dense * 1e-3) / 1e12 / 78.6,
                       "note": "K not a power of two: four dense m x m products per solve (FP64 MFMA)"},
        "neumann_fp64": {"unknowns": M_neu, "orders": cfg["orders"], "K_per_axis": cfg["Ks"][0], "alpha": 1.0,
                         "ms_per_step": ms_neu, "unknowns_per_s": M_neu / (ms_neu * 1e-3),
                         "passes": [dict(p, avg_ms=p["ms"] / p["launches"],
                                         gbs=p["bytes"] / (p["ms"] / p["launches"] * 1e-3) / 1e9)
                                    for p in passes_neu],
                         "note": "cosine (DCT-I) passes with the band-edge blocks"},
        "periodic_fp64": {"unknowns": M_per, "alpha": 1.0, "ms_per_step": ms_per,
                          "unknowns_per_s": M_per / (ms_per * 1e-3),
                          "passes": [dict(p, avg_ms=p["ms"] / p["launches"],
                                          gbs=p["bytes"] / (p["ms"] / p["launches"] * 1e-3) / 1e9)
                                     for p in passes_per]},
        "config": {"workload": "large_2d", "N": 2, "order_n": cfg["orders"][0],
                   "K_per_axis": cfg["Ks"][0], "unknowns": M, "rhs": "uniform[-1,1) seed 0",
                   "alpha": cfg["alpha"]},
        "fp32_refined": {"unknowns_per_s": M / (ms_ir * 1e-3), "ms_per_step": ms_ir,
                         "refinement_steps": args.ir_iters, "speedup_vs_fp64": ms64 / ms_ir,
                         "rel_l2_vs_fp64_gpu": dist(uir),
                         "algorithm_b_rel_l2_vs_fp64_gpu": dist(ub),
                         "rel_l2_vs_fp64_gpu_by_steps": hist},
        "fp32_pcg": {"unknowns_per_s": M / (ms_pcg * 1e-3), "ms_per_solve": ms_pcg,
                     "iterations": pcg_info.get("it"), "rel_update": pcg_info.get("upd"),
                     "rel_residual": pcg_info.get("res"), "speedup_vs_fp64": ms64 / ms_pcg,
                     "rel_l2_vs_fp64_gpu": dist(upcg)},
        "fp32_unrefined": {"unknowns_per_s": M / (ms32 * 1e-3), "ms_per_step": ms32,
                           "rel_l2_vs_fp64_gpu": dist(u32)},
        "passes_fp64": [dict(p, avg_ms=p["ms"] / p["launches"],
                             gbs=p["bytes"] / (p["ms"] / p["launches"] * 1e-3) / 1e9)
                        for p in passes64],
        "passes_fp32_refined": [dict(p, avg_ms=p["ms"] / p["launches"]) for p in passes_ir],
        "roofline": {"bound": "hbm", "kernel": kind, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": dom["bytes"], "avg_launch_ms": avg_ms},
    }
    if not args.no_cpu_baseline:
        log("large_2d: CPU oracle")
        base, parity = cpu_baseline(cfg, f_host, u64.cpu().numpy(),
                                    {"fp32_refined": uir.cpu().numpy(),
                                     "fp32_pcg": upcg.cpu().numpy(),
                                     "algorithm_b": ub.cpu().numpy()})
        rec["cpu_baseline"] = base
        rec["parity_vs_oracle"] = parity
    else:
        rec["cpu_baseline"] = None
    S.close()
    return rec


def bench_batch(args, torch, H, np, workloads, dev):
    cfg = workloads.BATCH
    pairs = workloads.batch_problems(cfg["count"], seed=0)
    solvers = {}
    probs = []
    for n, K in pairs:
        if (n, K) not in solvers:
            solvers[(n, K)] = H.Solver((n, n), (K, K), cfg["X"], cfg["alpha"])
        probs.append((solvers[(n, K)], cfg["nrhs"]))
    B = H.Batch(probs)
    f = torch.empty(B.total, dtype=torch.float64, device=dev)
    for p, arr in enumerate(workloads.batch_rhs(pairs, cfg["nrhs"], seed=0)):
        B.view(f, p).copy_(torch.from_numpy(arr))
    u = torch.empty_like(f)
    uir = torch.empty_like(f)
    ws = B.workspace("fp32_ir")
    s = torch.cuda.Stream()
    steps = max(2, args.steps // 4)
    log(f"batch_2d: {len(pairs)} problems, {B.groups} groups, {B.total} unknowns")
    with torch.cuda.stream(s):
        ms64 = time_calls(torch, lambda: B.solve(f, u, mode="fp64", use_graph=True,
                                                 stream=s.cuda_stream), steps, 2, s)
        ms64_eager = time_calls(torch, lambda: B.solve(f, u, mode="fp64", use_graph=False,
                                                       stream=s.cuda_stream), steps, 1, s)
        ms_ir = time_calls(torch, lambda: B.solve(f, uir, mode="fp32_ir", ws=ws,
                                                  max_iter=args.ir_iters, use_graph=True,
                                                  stream=s.cuda_stream), steps, 2, s)
    torch.cuda.synchronize()
    err = float(torch.linalg.vector_norm(uir - u) / torch.linalg.vector_norm(u))
    B.close()

    # per-(n, K) groups: one FP64 solve of a group's right-hand sides, the
    # default launch shapes against the autotuned ones
    log("batch_2d: per-(n, K) groups, default vs autotuned shapes")
    counts = {}
    for n, K in pairs:
        counts[(n, K)] = counts.get((n, K), 0) + 1
    breakdown = []
    for (n, K), cnt in sorted(counts.items()):
        S = solvers[(n, K)]
        r = cnt * cfg["nrhs"]
        fg = torch.rand(r * S.size, dtype=torch.float64, device=dev) * 2 - 1
        ug = torch.empty_like(fg)
        t_def = time_calls(torch, lambda: S.solve(fg, ug, mode="fp64", nrhs=r), steps, 1)
        S.autotune("fp64", nrhs=r, reps=2, f=fg, u=ug)
        t_tun = time_calls(torch, lambda: S.solve(fg, ug, mode="fp64", nrhs=r), steps, 1)
        breakdown.append({"n": n, "K": K, "problems": cnt, "unknowns": r * S.size,
                          "ms_default": t_def, "ms_tuned": t_tun,
                          "unknowns_per_s_tuned": r * S.size / (t_tun * 1e-3)})
        del fg, ug
    B = H.Batch(probs)          # fresh graph with the tuned shapes
    f2 = torch.empty(B.total, dtype=torch.float64, device=dev)
    for p, arr in enumerate(workloads.batch_rhs(pairs, cfg["nrhs"], seed=0)):
        B.view(f2, p).copy_(torch.from_numpy(arr))
    u2 = torch.empty_like(f2)
    with torch.cuda.stream(s):
        ms64_tuned = time_calls(torch, lambda: B.solve(f2, u2, mode="fp64", use_graph=True,
                                                       stream=s.cuda_stream), steps, 2, s)
    torch.cuda.synchronize()
    rec = {"workload": "batch_2d", "problems": len(pairs), "groups": B.groups,
           "rhs_per_problem": cfg["nrhs"], "unknowns": B.total,
           "fp64": {"unknowns_per_s": B.total / (ms64 * 1e-3), "ms_per_batch": ms64,
                    "ms_per_batch_without_graph": ms64_eager,
                    "ms_per_batch_tuned": ms64_tuned,
                    "unknowns_per_s_tuned": B.total / (ms64_tuned * 1e-3)},
           "per_n_K": breakdown,
           "fp32_refined": {"unknowns_per_s": B.total / (ms_ir * 1e-3), "ms_per_batch": ms_ir,
                            "refinement_steps": args.ir_iters, "rel_l2_vs_fp64_gpu": err}}
    B.close()
    for S in solvers.values():
        S.close()
    return rec


def gauss_load_1d(H, np, n, K, X, g):
    """1D scaled load vector of g by the (n+1)-point Gauss rule per element
    (Section 2, paragraph 5), from the plan's Gauss nodes, weights and basis
    values: sum over elements of sum_q w_q g(x_q) e_r(xi_q), interior points."""
    P = H.Plan1D(n, K)
    try:
        gx, gw = P.table("gx"), P.table("gw")
        B = P.table("B").reshape(n + 1, n + 1)   # B[q, r] = e_r(xi_q)
    finally:
        P.close()
    h = X / K
    x = np.arange(K)[:, None] * h + (gx[None, :] + 1.0) * (h / 2.0)
    contrib = (gw[None, :] * g(x)) @ B            # [element, r]
    b = np.zeros(n * K + 1)
    for r in range(n + 1):
        np.add.at(b, n * np.arange(K) + r, contrib[:, r])
    return b[1:-1]


def bench_cube(args, torch, H, np, workloads, dev):
    cfg = workloads.CONFIGS["cube_3d"]
    shp = workloads.shape(cfg["orders"], cfg["Ks"])
    M = int(np.prod(shp))
    # f^h: Gauss load of f = 11 pi^2 sin(pi x) sin(pi y) sin(3 pi z) (= -Lap of
    # sin(pi x) sin(pi y) sin(3 pi z)) plus N(0, 1e-3^2) noise on every entry
    ls = [gauss_load_1d(H, np, n, K, X, (lambda x, c=c: np.sin(c * np.pi * x)))
          for n, K, X, c in zip(cfg["orders"], cfg["Ks"], cfg["X"], (1, 1, 3))]
    fh = (11 * np.pi ** 2) * np.multiply.outer(np.multiply.outer(ls[0], ls[1]), ls[2])
    fh += workloads.normal_noise(fh.shape, 1e-3, seed=0)
    f64 = torch.from_numpy(fh).to(dev)
    S = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], cfg["alpha"])
    u64 = torch.empty_like(f64)
    uir = torch.empty_like(f64)
    ws = S.workspace("fp32_ir")
    steps = max(2, args.steps // 2)
    log(f"cube_3d: {M} unknowns")
    S.set_timing(True)
    ms64 = time_calls(torch, lambda: S.solve(f64, u64, mode="fp64"), steps, 1)
    passes64 = S.pass_times()
    S.set_timing(False)
    ms_ir = time_calls(torch, lambda: S.solve(f64, uir, mode="fp32_ir", ws=ws,
                                              max_iter=args.ir_iters, tol=0.0), steps, 1)
    err = float(torch.linalg.vector_norm(uir - u64) / torch.linalg.vector_norm(u64))
    rec = {"workload": "cube_3d", "unknowns": M,
           "fp64": {"unknowns_per_s": M / (ms64 * 1e-3), "ms_per_step": ms64,
                    "passes": [dict(p, avg_ms=p["ms"] / p["launches"],
                                    gbs=p["bytes"] / (p["ms"] / p["launches"] * 1e-3) / 1e9)
                               for p in passes64]},
           "fp32_refined": {"unknowns_per_s": M / (ms_ir * 1e-3), "ms_per_step": ms_ir,
                            "refinement_steps": args.ir_iters, "rel_l2_vs_fp64_gpu": err}}
    S.close()
    return rec


def bench_varcoef(args, torch, H, np, workloads, dev):
    cfg = workloads.CONFIGS["varcoef_3d"]
    shp = workloads.shape(cfg["orders"], cfg["Ks"])
    M = int(np.prod(shp))
    S = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], cfg["alpha"])
    c0, c1, ts = workloads.sine_coefficient(workloads.wavenumbers(3, seed=0))
    tabs = []
    for i, (n, K, X) in enumerate(zip(cfg["orders"], cfg["Ks"], cfg["X"])):
        gx = H.Plan1D(n, K).table("gx")      # Gauss nodes of the library's rule
        pts = (np.arange(K)[:, None] + (gx[None, :] + 1.0) / 2.0) * (X / K)
        tabs.append(torch.from_numpy(ts[i](pts)).to(dev))
    coef = H.make_coef(1, c0, c1, t=tuple(tabs))
    f = torch.from_numpy(workloads.uniform_rhs(shp, seed=0)).to(dev)
    u = torch.empty_like(f)
    ws = S.pcg_workspace(coef)
    log(f"varcoef_3d: {M} unknowns")
    info = {}

    def run():
        _, inf, _ = S.pcg(f, u, coef=coef, rtol=1e-10, max_iter=300, ws=ws)
        info["it"] = inf.iterations
        info["res"] = inf.rel_residual
    ms = time_calls(torch, run, 2, 1)
    out = torch.empty_like(f)
    ms_op = time_calls(torch, lambda: S.apply_coef_operator(u, coef, out=out, ws=ws), 5, 1)
    rec = {"workload": "varcoef_3d", "unknowns": M, "rtol": 1e-10,
           "iterations": info["it"], "rel_residual": info["res"], "ms_per_solve": ms,
           "unknowns_per_s": M / (ms * 1e-3),
           "operator": {"ms_per_apply": ms_op, "unknowns_per_s": M / (ms_op * 1e-3)}}
    S.close()
    return rec


def profile_bc(args, torch, H, workloads):
    """FP64 algorithm-(a) solves of the large 2D mesh (n = 9, K = 1024 per
    axis, alpha = 1) with both axes periodic, then both Neumann, for profiler
    counter runs."""
    cfg = workloads.CONFIGS["large_2d"]
    out = {}
    for bc in ("periodic", "neumann"):
        S = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], 1.0, bcs=(bc, bc))
        f = torch.rand(S.size, dtype=torch.float64, device="cuda")
        u = torch.empty_like(f)
        ms = time_calls(torch, lambda: S.solve(f, u, mode="fp64"), args.steps, args.warmup)
        out[bc] = {"ms_per_solve": ms, "unknowns": S.size}
        S.close()
        del f, u
        torch.cuda.empty_cache()
    return {"profile_bc_only": out, "kernel_sha": kernel_sha()}


def profile_operator(args, torch, H, workloads):
    """FP64 operator L u (the kernels of the FP32 forms' residual) on the
    large 2D and the cube workloads, for profiler counter runs."""
    out = {}
    for name in ("large_2d", "cube_3d"):
        cfg = workloads.CONFIGS[name]
        shp = workloads.shape(cfg["orders"], cfg["Ks"])
        u = torch.from_numpy(workloads.uniform_rhs(shp, seed=0)).cuda()
        S = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], cfg["alpha"])
        ws = S.operator_workspace(u.device)
        r = torch.empty_like(u)
        ms = time_calls(torch, lambda: S.apply_operator(u, out=r, ws=ws), args.steps, args.warmup)
        out[name] = {"ms_per_apply": ms, "unknowns": u.numel()}
        S.close()
        del u, r, ws
        torch.cuda.empty_cache()
    import numpy as np
    cfg = workloads.CONFIGS["varcoef_3d"]
    shp = workloads.shape(cfg["orders"], cfg["Ks"])
    S = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], cfg["alpha"])
    c0, c1, ts = workloads.sine_coefficient(workloads.wavenumbers(3, seed=0))
    tabs = []
    for i, (n, K, X) in enumerate(zip(cfg["orders"], cfg["Ks"], cfg["X"])):
        gx = H.Plan1D(n, K).table("gx")
        pts = (np.arange(K)[:, None] + (gx[None, :] + 1.0) / 2.0) * (X / K)
        tabs.append(torch.from_numpy(ts[i](pts)).cuda())
    coef = H.make_coef(1, c0, c1, t=tuple(tabs))
    u = torch.from_numpy(workloads.uniform_rhs(shp, seed=0)).cuda()
    r = torch.empty_like(u)
    ws = S.pcg_workspace(coef)
    ms = time_calls(torch, lambda: S.apply_coef_operator(u, coef, out=r, ws=ws), args.steps, args.warmup)
    out["varcoef_3d"] = {"ms_per_apply": ms, "unknowns": u.numel()}
    S.close()
    return {"profile_operator_only": out, "kernel_sha": kernel_sha()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ir-iters", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-fp64", action="store_true",
                    help="large_2d FP64 solves only (for profiler counter runs)")
    ap.add_argument("--profile-bc", action="store_true",
                    help="FP64 solves of large_2d with periodic and with Neumann axes only (for profiler runs)")
    ap.add_argument("--profile-operator", action="store_true",
                    help="FP64 operator applies of large_2d and cube_3d only (for profiler runs)")
    ap.add_argument("--only", default="large_2d,batch_2d,cube_3d,varcoef_3d",
                    help="comma-separated workloads; large_2d is the headline")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1609_07758_amd as H
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibration_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.profile_operator:
        print(json.dumps(profile_operator(args, torch, H, workloads)), flush=True)
        return
    if args.profile_bc:
        print(json.dumps(profile_bc(args, torch, H, workloads)), flush=True)
        return

    only = set(args.only.split(","))
    record = {"metric": "unknowns/s, 2D n=9 K=2^10: FP64 vs FP32+refine @1e-12 rel L2; % HBM peak",
              "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
              "data": "synthetic"}
    if "large_2d" in only:
        record.update(bench_headline(args, torch, H, np, workloads, dev))
    others = {}
    for name, fn in (("batch_2d", bench_batch), ("cube_3d", bench_cube),
                     ("varcoef_3d", bench_varcoef)):
        if name in only:
            others[name] = fn(args, torch, H, np, workloads, dev)
            torch.cuda.empty_cache()
    if others:
        record["other_workloads"] = others
    record["kernel_sha"] = kernel_sha()
    print(json.dumps(record), flush=True)


if __name__ == "__main__":
    main()
