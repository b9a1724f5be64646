#!/usr/bin/env python3
"""Benchmark of pairwise-perturbation CP-ALS against dimension-tree ALS on one MI355X.

Workload (default): order-3 800 x 800 x 800 tensor, planted rank-50 CP whose
factor columns have collinearity 0.9 (shared + independent N(0,1) parts,
normalised), 1e-3 relative Gaussian noise, seed 0; decomposition rank 50 from
a seeded uniform [0,1) initial guess; PP threshold eps = 0.1 on ||dA||/||A||;
200 sweeps.  One benchmark step is one whole PP-CP-ALS decomposition of that
tensor (Algorithm 3: ALS sweeps, operator builds, PP sweeps, fit), with the
tensor already resident in HBM.  value = PP-ALS sweeps per second.

Beside it the script reports the dimension-tree ALS run on the same tensor
(Algorithm 1), the time each needs to reach the same fit, the roofline of the
dominant kernel (HIP events recorded by the library on its launch stream during
one extra, untimed step) and the CPU oracle timed on the host.

Prints one JSON line on stdout; progress goes to stderr.
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

METRIC = "ALS sweeps/sec, PP vs dimension-tree ALS at equal fit; MFMA % and HBM GB/s"
PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "f64_TFs": 78.6,
    "f32_TFs": 157.3,
    "bf16_TFs": 2500.0,
}


# The paper's own speedups for this path (context, not targets): Intel Xeon Phi KNL nodes
# (68 cores, 64 threads for the BLAS and tensor-transpose libraries), precision not stated.
PAPER_NUMBERS = {
    "hardware": "Intel Xeon Phi KNL (Stampede2), one node, 64 threads; NumPy/MKL/HPTT",
    "pp_approx_vs_dt_sweep": {"order3_R_eq_s": 6.3, "orders3to6_R50": 33.0},
    "pp_init_over_dt_sweep": [1.5, 2.0],
    "time_to_solution_collinear_synthetic": 2.0,
    "tucker_pp_approx_vs_hooi_sweep_order6_R5": 10.6,
    "tucker_time_to_solution_images": [1.05, 1.13],
    "source": "Section 5.1 (per-sweep comparison, synthetic collinearity and image-data "
              "experiments)",
}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def time_to_fit(recs, ms, target):
    t = 0.0
    for r, m in zip(recs, ms):
        t += m
        if r["fit_est"] >= target:
            return t
    return None


def cpu_baseline(X, init, rank, eps, gpu_kinds, budget_s):
    """Time the float64 oracle's sweep kinds on the host and weight them by the GPU
    run's kind counts (a bounded sample; the oracle is used as it stands)."""
    import threadpoolctl
    from oracle import cp as ocp
    from oracle import pp as opp

    threads = max((p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()), default=1)
    A = [a.copy() for a in init]
    S = [a.T @ a for a in A]
    normX2 = float(np.sum(X * X))
    t_als, t_init, t_appr = [], [], []
    start = time.perf_counter()
    for _ in range(8):
        t0 = time.perf_counter()
        ocp.als_sweep(X, A, S, normX2)
        t_als.append(time.perf_counter() - t0)
        if time.perf_counter() - start > budget_s * 0.4:
            break
    t0 = time.perf_counter()
    st = opp.build_operators(X, A)
    opp.pp_sweep(st, A, S, normX2, True, "pp_init")
    t_init.append(time.perf_counter() - t0)
    for _ in range(40):
        t0 = time.perf_counter()
        opp.pp_sweep(st, A, S, normX2, True, "pp_approx")
        t_appr.append(time.perf_counter() - t0)
        if time.perf_counter() - start > budget_s:
            break
    per = {"als": float(np.mean(t_als)), "pp_init": float(np.mean(t_init)),
           "pp_approx": float(np.mean(t_appr))}
    counts = {k: gpu_kinds.count(k) for k in per}
    total = sum(counts[k] * per[k] for k in per)
    return {
        "value": len(gpu_kinds) / total if total > 0 else None,
        "unit": "sweeps/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"float64 oracle on the same tensor: {len(t_als)} ALS, {len(t_init)} PP-init "
                   f"(build + first PP sweep), {len(t_appr)} PP-approx sweeps timed "
                   f"({time.perf_counter() - start:.1f} s); per-kind mean times weighted by the GPU "
                   f"run's sweep mix {counts}"),
        "per_sweep_s": per,
        "host_cpus": len(os.sched_getaffinity(0)),
    }


def oracle_replay(X, init, kinds, cap_s):
    """The float64 oracle replaying the GPU run's sweep-kind sequence on the same tensor
    (host cores): per-kind sweep times and, when the whole sequence ran within cap_s,
    the final factors and the oracle's fit of them."""
    import threadpoolctl
    from oracle import cp as ocp
    from oracle import pp as opp

    threads = max((p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()), default=1)
    A = [a.copy() for a in init]
    S = [a.T @ a for a in A]
    normX2 = float(np.sum(X * X))
    times = {"als": [], "pp_init": [], "pp_approx": []}
    state = None
    start = time.perf_counter()
    done = 0
    for i, kind in enumerate(kinds):
        t0 = time.perf_counter()
        if kind == "als":
            ocp.als_sweep(X, A, S, normX2)
        elif kind == "pp_init":
            state = opp.build_operators(X, A)
            opp.pp_sweep(state, A, S, normX2, True, "pp_init")
        else:
            opp.pp_sweep(state, A, S, normX2, True, "pp_approx")
        times[kind].append(time.perf_counter() - t0)
        done = i + 1
        if done % 25 == 0:
            log(f"oracle replay: {done}/{len(kinds)} sweeps, {time.perf_counter() - start:.1f} s")
        if time.perf_counter() - start > cap_s:
            break
    out = {"threads": int(threads), "sweeps": done, "seconds": time.perf_counter() - start,
           "per_sweep_s": {k: (float(np.mean(v)) if v else None) for k, v in times.items()},
           "complete": done == len(kinds), "A": None, "fit": None}
    if out["complete"]:
        out["A"] = A
        out["fit"] = oracle_fit(X, A)
    return out


def oracle_fit(X, A):
    """1 - ||X - [[A]]||_F / ||X||_F by the oracle's identity with the exact right-hand
    side of the last mode."""
    from oracle import cp as ocp
    N = X.ndim
    S = [a.T @ a for a in A]
    M = ocp.mttkrp(X, A, N - 1)
    return ocp.fit_identity(float(np.sum(X * X)), M, A[N - 1], ocp.hadamard_except(S, N - 1),
                            S[N - 1])


COPY_BYTES = 1 << 30


def copy_calibration(torch, dev):
    """A plain device-to-device copy of COPY_BYTES, five times: under a counter profiler
    its FETCH_SIZE / WRITE_SIZE per dispatch give the scale from counter units to bytes."""
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": COPY_BYTES, "dispatches": 5}), flush=True)


def batch_specs(count, seed=0):
    """Sizes and ranks of the batched workload: s_n ~ U{32..192} per mode, R ~ U{4..48},
    from SeedSequence(seed).spawn(count); the tensor of problem p uses seed p."""
    out = []
    for p, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(ss)
        dims = tuple(int(d) for d in rng.integers(32, 193, 3))
        out.append((dims, int(rng.integers(4, 49)), p))
    return out


def batch_cpu_baseline(specs, eps, sweeps, tol, budget_s):
    """The float64 oracle on a bounded sample of the batched workload: whole
    decompositions of the first problems (same recipe, host generator) until the
    budget is spent; sweeps per second over the sample."""
    import threadpoolctl
    import tensorgen
    from oracle import pp as opp
    threads = max((p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()), default=1)
    done = 0
    t_all = 0.0
    used = 0
    start = time.perf_counter()
    for dims, R, seed in specs:
        prob = tensorgen.make_problem(dims, R, seed=seed, eta=1e-3)
        Xh = prob.X.astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        _, recs = opp.pp_als(Xh, prob.init, eps=eps, sweeps=sweeps)
        fits = [r.fit_est for r in recs]
        n = len(recs)
        for k in range(1, len(fits)):
            if abs(fits[k] - fits[k - 1]) < tol:
                n = k + 1
                break
        t_all += (time.perf_counter() - t0) * n / len(recs)
        done += n
        used += 1
        if time.perf_counter() - start > budget_s:
            break
    return {"value": done / t_all if t_all > 0 else None, "unit": "sweeps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"float64 oracle, the first {used} problems of the batch run to convergence "
                      f"(|dfit| < {tol}) or {sweeps} sweeps: {done} sweeps in {t_all:.1f} s",
            "host_cpus": len(os.sched_getaffinity(0))}


def batch_bench(args, torch, dev):
    print(json.dumps(batch_leg(args, torch, dev, cpu=not args.no_cpu_baseline)), flush=True)


def batch_leg(args, torch, dev, cpu=True, warmup=None):
    """The batched workload (512 order-3 problems in one HIP graph per batched sweep):
    returns its result line."""
    import paper_1811_10573_amd as pp
    import tensorgen
    count, sweeps, eps, tol = args.batch_count, 100, 0.1, 1e-5
    specs = batch_specs(count)
    log(f"generating {count} problems (s ~ U{{32..192}}, R ~ U{{4..48}})")
    X, A = [], []
    for dims, R, seed in specs:
        prob = tensorgen.make_problem_device(dims, R, seed, eta=1e-3, dtype="f32", device=dev)
        X.append(prob.X.reshape(-1))
        A.append([torch.from_numpy(a.copy()).to(dev) for a in prob.init])
    init = [[a.clone() for a in fs] for fs in A]
    b = pp.Batch([(d, R) for d, R, _ in specs], sweeps)
    ws = b.workspace(dev)
    log(f"workspace {b.workspace_bytes / 2**30:.2f} GiB, tensors "
        f"{sum(x.numel() for x in X) * 4 / 2**30:.2f} GiB")

    def reset():
        for fs, f0 in zip(A, init):
            for a, a0 in zip(fs, f0):
                a.copy_(a0)
        b.bind(X, A, ws, eps, tol)

    reset()
    b.autotune(ws, reps=3)
    tune = b.describe()
    for w in range(args.warmup if warmup is None else warmup):
        reset()
        b.run(ws, sweeps, use_graph=True)
        torch.cuda.synchronize()
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(ws, sweeps, use_graph=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    res = b.results(ws)
    total = sum(r["sweeps"] for r in res)
    conv = [r["time_to_converge_ms"] for r in res if r["converged_sweep"] > 0]
    value = total / elapsed
    log(f"{total} problem-sweeps in {elapsed * 1e3:.1f} ms -> {value:.0f} sweeps/s; "
        f"{len(conv)}/{count} converged")
    # roofline of the grouped first-level contraction from the autotuner's timings
    # (contiguous-mode and leading-mode contractions of every problem, chosen variant);
    # most problems have R < 40, where the contraction is bound by HBM (AI = R/2 flop/B)
    nbytes = sum(2 * (4.0 * d[0] * d[1] * d[2] + 4.0 * R * (d[0] * d[1] + d[1] * d[2]) / 2)
                 for d, R, _ in specs)
    flops = sum(2.0 * R * (d[0] * d[1] * d[2]) * 2 for d, R, _ in specs)
    ms = sum(bk[f"ms_{bk['tile_rows']}"] for bk in tune["buckets"])
    achieved = nbytes / (ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
            "frac": achieved / PEAK["hbm_GBs"],
            "traffic": measured_traffic("k_b_gemm", None, None, None, workload=f"f32_batch{count}"),
            "kernel": "k_b_gemm",
            "avg_ms": ms / 2, "work_per_launch": nbytes / 2,
            "TFLOP_s": flops / (ms * 1e-3) / 1e12}
    cpu_line = None
    if cpu:
        log("timing the float64 oracle on the host (bounded sample)")
        cpu_line = batch_cpu_baseline(specs, eps, sweeps, tol, args.cpu_seconds)
    kinds = {"als": sum(r["n_als"] for r in res), "pp_init": sum(r["n_pp_init"] for r in res),
             "pp_approx": sum(r["n_pp_approx"] for r in res)}
    line = {
        "metric": "aggregate ALS sweeps/sec over a batch of independent PP-CP-ALS decompositions",
        "value": value, "unit": "sweeps/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded planted CP + noise)",
        "config": {"workload": f"{count} order-3 FP32 problems, s_n ~ U{{32..192}}, R ~ U{{4..48}}, "
                               f"N(0,1) planted factors, 1e-3 noise, eps={eps}, {sweeps} sweeps max, "
                               f"stop at |dfit| < {tol}, one HIP graph per batched sweep",
                   "count": count},
        "roofline": roof, "cpu_baseline": cpu_line,
        "batch": {"converged": len(conv),
                  "time_to_converge_ms_p50": float(np.percentile(conv, 50)) if conv else None,
                  "time_to_converge_ms_p99": float(np.percentile(conv, 99)) if conv else None,
                  "sweep_kinds": kinds, "autotune": tune},
    }
    del ws, b, X, A, init
    torch.cuda.empty_cache()
    return line


def roof_of(stat, bound, peak, traffic=None):
    """Roofline entry of one kernel class from its HIP-event statistics (algorithmic work
    per launch over the average launch time)."""
    if not stat or stat["launches"] == 0:
        return None
    if bound == "mfma":
        ach = stat["flops"] / (stat["total_ms"] * 1e-3) / 1e12
        unit, work = "TFLOP/s", stat["flops"]
    else:
        ach = stat["bytes"] / (stat["total_ms"] * 1e-3) / 1e9
        unit, work = "GB/s", stat["bytes"]
    return {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
            "traffic": traffic, "launches": stat["launches"], "avg_ms": stat["avg_ms"],
            "work_per_launch": work / stat["launches"]}


def f64_leg(pp, torch, dev, prob, shape, R, eps, sweeps, kinds_replay, warmup, steps):
    """The same decomposition with the FP64 tier on the FP64 tensor: free-running sweeps/s
    (graph replays, X resident), the per-kernel roofline from one profiled step, and a
    replay of the FP32 run's sweep kinds whose final factors go to the oracle comparison."""
    X = torch.from_numpy(prob.X).to(dev).reshape(-1)
    plan = pp.Plan(shape, R, "f64", "f64", True)
    ws = plan.workspace(dev)
    A0 = [torch.from_numpy(a).to(dev) for a in prob.init]
    A = [a.clone() for a in A0]
    S = torch.zeros(len(shape) * R * R, dtype=torch.float64, device=dev)
    rec = pp.new_record(dev)
    nrm = torch.zeros(1, dtype=torch.float64, device=dev)
    pp.tensor_norm2(X, nrm)
    normX2 = float(nrm.item())

    def run(replay=None, timing=False):
        for a, a0 in zip(A, A0):
            a.copy_(a0)
        return pp.run(plan, X, None, A, S, normX2, ws, rec, eps=eps, max_sweeps=sweeps,
                      replay=replay, timing=timing)

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for _ in range(steps):
        recs, _ = run()
        done += len(recs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    recs, ms = run(timing=True)
    kinds = [r["kind"] for r in recs]
    pp.get_profile(plan, reset=True)
    pp.set_profiling(plan, True)
    run()
    torch.cuda.synchronize()
    pp.set_profiling(plan, False)
    prof = pp.get_profile(plan, reset=True)
    res2 = torch.zeros(1, dtype=torch.float64, device=dev)
    pp.exact_residual2(plan, X, A, res2, ws)
    fit_free = 1.0 - float(np.sqrt(res2.item() / normX2))
    run(replay=kinds_replay)
    torch.cuda.synchronize()
    A_replay = [a.cpu().numpy().reshape(s, R) for a, s in zip(A, shape)]
    out = {
        "sweeps_per_s": done / elapsed, "steps": steps, "ms_per_step": elapsed / steps * 1e3,
        "sweep_mix": {k: kinds.count(k) for k in ("als", "pp_init", "pp_approx")},
        "per_kind_ms": {k: (float(np.mean([m for r, m in zip(recs, ms) if r["kind"] == k]))
                            if k in kinds else None) for k in ("als", "pp_init", "pp_approx")},
        "final_fit_exact": fit_free,
        "roofline_level1": roof_of(prof.get("level1_gemm"), "mfma", PEAK["f64_TFs"],
                                   measured_traffic("level1_gemm", "f64", shape, R)),
        "roofline_pp_ttv": roof_of(prof.get("pp_correct_ttv"), "hbm", PEAK["hbm_GBs"],
                                   measured_traffic("pp_correct_ttv", "f64", shape, R)),
    }
    log(f"FP64 tier: {out['sweeps_per_s']:.1f} sweeps/s, mix {out['sweep_mix']}, "
        f"fit {fit_free:.10f}")
    del ws, X
    torch.cuda.empty_cache()
    return out, A_replay


def c1_leg(pp, torch, dev, tensorgen, runs=20):
    """64^3 FP64 tensor, planted rank 10 (N(0,1) factors), 1e-3 noise, rank 10, 20 ALS
    sweeps from the seeded uniform start: sweeps/s over `runs` whole runs and the
    per-sweep fit estimates (compared with the oracle in the oracle leg)."""
    prob = tensorgen.make_problem((64, 64, 64), 10, seed=0, eta=1e-3)
    plan = pp.Plan(prob.shape, 10, "f64")
    X = torch.from_numpy(prob.X).to(dev)
    A0 = [torch.from_numpy(a).to(dev) for a in prob.init]
    A = [a.clone() for a in A0]
    S = torch.zeros(3 * 100, dtype=torch.float64, device=dev)
    ws = plan.workspace(dev)
    rec = pp.new_record(dev)
    nrm = torch.zeros(1, dtype=torch.float64, device=dev)
    pp.tensor_norm2(X, nrm)

    def run():
        for a, a0 in zip(A, A0):
            a.copy_(a0)
        return pp.run(plan, X, None, A, S, float(nrm.item()), ws, rec, eps=0.0, max_sweeps=20,
                      timing=False)

    recs, _ = run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        recs, _ = run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = {"workload": "64x64x64 FP64, planted rank 10, 1e-3 noise, rank 10, 20 ALS sweeps",
           "sweeps_per_s": 20 * runs / elapsed, "ms_per_run": elapsed / runs * 1e3,
           "fits": [r["fit_est"] for r in recs]}
    log(f"C1: {out['sweeps_per_s']:.0f} sweeps/s ({out['ms_per_run']:.2f} ms per 20-sweep run)")
    return out, prob


def c3_level1_leg(pp, torch, dev, tensorgen, reps=5):
    """First-level contractions of the order-4 workload (160^4 FP32 tensor, planted rank 64,
    1e-2 noise, assembled on the device; R = 64): the two two-mode contractions of the ALS
    dimension tree (K = 160^2), FP32 and BF16-input tiers, timed with HIP events."""
    shape, R = (160, 160, 160, 160), 64
    prob = tensorgen.make_problem_device(shape, R, 0, eta=1e-2, dtype="f32", device=dev)
    X = prob.X.reshape(-1)
    Xb = torch.empty(X.numel(), dtype=torch.int16, device=dev)
    pp.cast_bf16(X, Xb)
    A = [torch.from_numpy(a).to(dev) for a in prob.init]
    out = {"workload": "160^4 FP32 (BF16 copy for the BF16 tier), R = 64; X contracted with "
                       "the Khatri-Rao product of modes (3,4) and of modes (1,2)"}
    for tier in ("f32", "bf16"):
        plan = pp.Plan(shape, R, "f32", tier, True)
        ws = plan.workspace(dev)
        res = {}
        for name, modes in (("contract_modes_34", (2, 3)), ("contract_modes_12", (0, 1))):
            o = torch.empty(160 * 160 * R, dtype=torch.float32, device=dev)
            pp.level1(plan, X, Xb, A, modes, o, ws)
            torch.cuda.synchronize()
            pp.get_profile(plan, reset=True)
            pp.set_profiling(plan, True)
            for _ in range(reps):
                pp.level1(plan, X, Xb, A, modes, o, ws)
            torch.cuda.synchronize()
            pp.set_profiling(plan, False)
            prof = pp.get_profile(plan, reset=True)
            g = prof["level1_gemm"]
            e = {"avg_ms": g["avg_ms"], "TFLOP_s": g["flops"] / (g["total_ms"] * 1e-3) / 1e12,
                 "HBM_GB_s": g["bytes"] / (g["total_ms"] * 1e-3) / 1e9}
            e["mfma_frac"] = e["TFLOP_s"] / PEAK["f32_TFs" if tier == "f32" else "bf16_TFs"]
            e["hbm_frac"] = e["HBM_GB_s"] / PEAK["hbm_GBs"]
            sr = prof.get("split_reduce")
            if sr and sr["launches"]:
                e["split_reduce_avg_ms"] = sr["avg_ms"]
            res[name] = e
            del o
        out[tier] = res
        log(f"C3 level 1 {tier}: " + ", ".join(f"{k} {v['avg_ms']:.3f} ms {v['TFLOP_s']:.1f} TF/s"
                                                 for k, v in res.items()))
        del ws, plan
    del X, Xb, prob
    torch.cuda.empty_cache()
    return out


def tucker_leg(pp, torch, dev, tensorgen, s=800, R=40, eta=0.1, eps=0.3, sweeps=12, reps=3,
               cpu_seconds=0.0):
    """Order-3 Tucker (Algorithms 2 and 4) on an s^3 FP64 planted Tucker tensor (orthonormal
    factors, N(0,1) core of rank R = 0.05 s, noise eta): HOSVD from seeded random bases,
    the mean time of HOOI, PP-initialisation and PP-approximated sweeps, the TTMc
    contraction rate, and whole runs of `sweeps` sweeps of HOOI (eps = 0) and
    PP-Tucker-ALS (eps) from the same HOSVD."""
    from oracle import tucker as ot
    shape = (s, s, s)
    t0 = time.perf_counter()
    prob = tensorgen.make_tucker_problem(shape, (R, R, R), seed=0, eta=eta)
    log(f"Tucker: generated {shape} rank-{R} in {time.perf_counter() - t0:.1f} s")
    plan = pp.TuckerPlan(shape, R)
    X = torch.from_numpy(prob.X.reshape(-1)).to(dev)
    ws = plan.workspace(dev)
    normX2 = float(np.sum(prob.X ** 2))
    V0 = [torch.from_numpy(v).to(dev) for v in tensorgen.subspace_start(shape, R, seed=1)]
    A = [torch.empty(n * R, dtype=torch.float64, device=dev) for n in shape]
    G = torch.empty(R ** 3, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pp.tucker_hosvd_interlaced(plan, ws, X, V0, A, G)
    hosvd_il_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    hinfo = pp.tucker_hosvd(plan, ws, X, V0, A, G)
    hosvd_ms = (time.perf_counter() - t0) * 1e3
    A0 = [a.clone() for a in A]
    G0 = G.clone()
    out = {"workload": f"Tucker, {s}^3 FP64 planted rank ({R},{R},{R}) orthonormal factors, "
                       f"N(0,1) core, {eta:g} noise; R = 0.05 s as in the paper's order-3 "
                       f"per-sweep comparison; eps = {eps}",
           "hosvd_ms": hosvd_ms, "hosvd_interlaced_ms": hosvd_il_ms,
           "hosvd_iterations": [h[0] for h in hinfo]}

    def reset():
        for a, a0 in zip(A, A0):
            a.copy_(a0)
        G.copy_(G0)

    # per-sweep times (each call synchronises; ms is the host wall time of the sweep)
    reset()
    als = [pp.tucker_als_sweep(plan, ws, X, A, G, normX2) for _ in range(reps + 1)][1:]
    pp.tucker_pp_build(plan, ws, X, A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pp.tucker_pp_build(plan, ws, X, A)
    init = pp.tucker_pp_sweep(plan, ws, A, G, normX2, "pp_init")
    init_ms = (time.perf_counter() - t0) * 1e3
    appr = [pp.tucker_pp_sweep(plan, ws, A, G, normX2, "pp_approx") for _ in range(reps)]
    mean = lambda xs: float(sum(xs) / len(xs))
    als_ms = mean([r["ms"] for r in als])
    appr_ms = mean([r["ms"] for r in appr])
    out["per_sweep_ms"] = {"hooi": als_ms, "pp_init": init_ms, "pp_approx": appr_ms}
    out["pp_approx_speedup_vs_hooi_sweep"] = als_ms / appr_ms
    out["pp_init_over_hooi_sweep"] = init_ms / als_ms
    out["subspace_iterations"] = {"hooi": [r["iters"] for r in als],
                                  "pp_approx": [r["iters"] for r in appr]}
    # TTMc rate: Y^(1) = (X x_3 A3^T) x_2 A2^T, 2 s^3 R + 2 s^2 R^2 flops, X read once
    Y = torch.empty(s * R * R, dtype=torch.float64, device=dev)
    pp.tucker_ttmc(plan, ws, X, A, 0, Y)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        pp.tucker_ttmc(plan, ws, X, A, 0, Y)
    ev[1].record()
    torch.cuda.synchronize()
    ttmc_ms = ev[0].elapsed_time(ev[1]) / reps
    flops = 2.0 * s ** 3 * R + 2.0 * s ** 2 * R * R
    out["ttmc_mode1"] = {"avg_ms": ttmc_ms, "TFLOP_s": flops / (ttmc_ms * 1e-3) / 1e12,
                         "mfma_frac": flops / (ttmc_ms * 1e-3) / 1e12 / PEAK["f64_TFs"],
                         "HBM_GB_s": 8.0 * s ** 3 / (ttmc_ms * 1e-3) / 1e9}
    # whole runs from the HOSVD
    runs = {}
    for name, e in (("hooi", 0.0), ("pp", eps)):
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = pp.tucker_run(plan, ws, X, A, G, eps=e, sweeps=sweeps)
        runs[name] = {"seconds": time.perf_counter() - t0,
                      "kinds": [r["kind"] for r in recs],
                      "fit": [r["fit"] for r in recs],
                      "ms": [r["ms"] for r in recs]}
    out["runs"] = {k: {"seconds": v["seconds"], "final_fit": v["fit"][-1],
                       "kinds": {kk: v["kinds"].count(kk) for kk in set(v["kinds"])}}
                   for k, v in runs.items()}
    out["pp_vs_hooi_run_speedup"] = runs["hooi"]["seconds"] / runs["pp"]["seconds"]
    out["final_fit_diff_pp_vs_hooi"] = runs["pp"]["fit"][-1] - runs["hooi"]["fit"][-1]
    log(f"Tucker {s}^3 R {R}: HOSVD {hosvd_ms:.0f} ms; sweep HOOI {als_ms:.2f} ms, PP init "
        f"{init_ms:.2f} ms, PP approx {appr_ms:.2f} ms ({als_ms / appr_ms:.2f}x); TTMc "
        f"{out['ttmc_mode1']['TFLOP_s']:.1f} TF/s; runs HOOI {runs['hooi']['seconds']:.3f} s, "
        f"PP {runs['pp']['seconds']:.3f} s")
    if cpu_seconds > 0:
        # float64 oracle: HOOI sweeps on the same tensor from the oracle's own HOSVD
        t0 = time.perf_counter()
        Ao, Go = ot.hosvd(prob.X, (R, R, R))
        t_hosvd = time.perf_counter() - t0
        t0 = time.perf_counter()
        n = 0
        while n < 1 or (time.perf_counter() - t0 < cpu_seconds and n < 5):
            Go, _, _ = ot.tucker_sweep(prob.X, Ao, Go, normX2)
            n += 1
        per = (time.perf_counter() - t0) / n
        out["cpu_oracle"] = {"hooi_sweep_s": per, "hosvd_s": t_hosvd, "sweeps": n,
                             "threads": torch.get_num_threads(),
                             "gpu_hooi_sweep_speedup": per / (als_ms * 1e-3)}
        log(f"Tucker oracle: HOSVD {t_hosvd:.1f} s, HOOI sweep {per:.2f} s")
    del X, ws, Y
    torch.cuda.empty_cache()
    return out


def tucker_sweeps_leg(pp, torch, dev, tensorgen, shape, R, eta=0.1, n_approx=6):
    """Per-sweep times of HOOI, PP-initialisation and PP-approximated Tucker sweeps on an
    order-N FP64 planted Tucker tensor (device-generated), kinds forced from the HOSVD
    start: three HOOI sweeps, a PP initialisation, n_approx PP sweeps (the paper's
    per-sweep comparison, Section 5.1)."""
    t0 = time.perf_counter()
    X, _, _ = tensorgen.make_tucker_problem_device(shape, (R,) * len(shape), 0, eta=eta, device=dev)
    X = X.reshape(-1)
    gen_s = time.perf_counter() - t0
    plan = pp.TuckerPlan(shape, R)
    ws = plan.workspace(dev)
    V0 = [torch.from_numpy(v).to(dev) for v in tensorgen.subspace_start(shape, R, seed=1)]
    A = [torch.empty(n * R, dtype=torch.float64, device=dev) for n in shape]
    G = torch.empty(R ** len(shape), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pp.tucker_hosvd_interlaced(plan, ws, X, V0, A, G)
    hosvd_il_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    pp.tucker_hosvd(plan, ws, X, V0, A, G)
    hosvd_ms = (time.perf_counter() - t0) * 1e3
    kinds = ["als"] * 3 + ["pp_init"] + ["pp_approx"] * n_approx
    recs = pp.tucker_run(plan, ws, X, A, G, eps=0.3, sweeps=len(kinds), replay=kinds)
    per = {}
    for k in ("als", "pp_init", "pp_approx"):
        t = [r["ms"] for i, r in enumerate(recs) if r["kind"] == k and i > 0]
        per[k] = float(np.mean(t))
    out = {"shape": list(shape), "rank": R, "ms": per, "hosvd_ms": hosvd_ms,
           "hosvd_interlaced_ms": hosvd_il_ms,
           "pp_approx_speedup_vs_hooi_sweep": per["als"] / per["pp_approx"],
           "pp_init_over_hooi_sweep": per["pp_init"] / per["als"],
           "iterations": {k: [r["iters"] for r in recs if r["kind"] == k][-1]
                          for k in ("als", "pp_approx")},
           "workspace_GB": plan.workspace_bytes / 1e9, "generation_s": gen_s}
    log(f"Tucker sweep kinds {shape} R {R}: HOOI {per['als']:.2f} ms, PP-init {per['pp_init']:.2f} ms, "
        f"PP-approx {per['pp_approx']:.3f} ms ({out['pp_approx_speedup_vs_hooi_sweep']:.1f}x); "
        f"HOSVD {hosvd_ms:.0f} ms, interlaced {hosvd_il_ms:.0f} ms")
    del X, ws, plan
    torch.cuda.empty_cache()
    return out


# the paper's order-varying Tucker comparison: s = 1200^(3/N), R = 5
PAPER_TUCKER_CONFIGS = (((1200,) * 3, 5), ((205,) * 4, 5), ((70,) * 5, 5), ((35,) * 6, 5))


def build_leg(pp, torch, dev, tensorgen, shape=(160, 160, 160, 160), R=64, tier="f32", reps=3):
    """PP operator build of Section 3.2.3 on one configuration, with the dimension tree and
    with the direct build (every operator from X and the Khatri-Rao product of the other
    N - 2 factors): workspace, bytes of the tree's intermediates, build time (HIP events
    around pp_build_operators) and first-level rate."""
    prob = tensorgen.make_problem_device(shape, R, 0, eta=1e-2, dtype=tier, device=dev)
    X = prob.X.reshape(-1)
    A = [torch.from_numpy(a).to(dev) for a in prob.init]
    out = {"workload": f"PP operator build, order {len(shape)} {'x'.join(map(str, shape))} "
                       f"{tier.upper()}, R = {R}"}
    for build in ("tree", "direct"):
        plan = pp.Plan(shape, R, tier, tier, True, pp_build=build)
        d = plan.describe()
        ws = plan.workspace(dev)
        pp.pp_build_operators(plan, X, None, A, ws)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            pp.pp_build_operators(plan, X, None, A, ws)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        fl = d["pp_build_level1_flops"] + d["pp_build_tree_ttv_flops"] + d["pp_build_mp_flops"]
        out[build] = {"ms": ms, "workspace_GB": plan.workspace_bytes / 1e9,
                      "intermediate_GB": d["pp_build_intermediate_bytes"] / 1e9,
                      "level1_launches": sum(1 for o in d["pp_build_ops"] if o["op"] == "level1"),
                      "strided_launches": sum(1 for o in d["pp_build_ops"] if o.get("strided")),
                      "GFLOP": fl / 1e9, "TFLOP_s": fl / (ms * 1e-3) / 1e12}
        del ws, plan
        torch.cuda.empty_cache()
    out["direct_over_tree_time"] = out["direct"]["ms"] / out["tree"]["ms"]
    out["workspace_saved_GB"] = out["tree"]["workspace_GB"] - out["direct"]["workspace_GB"]
    log(f"build {shape} R {R} {tier}: tree {out['tree']['ms']:.2f} ms ws {out['tree']['workspace_GB']:.2f} GB; "
        f"direct {out['direct']['ms']:.2f} ms ws {out['direct']['workspace_GB']:.2f} GB")
    del X, prob
    torch.cuda.empty_cache()
    return out


def sweep_kinds_leg(pp, torch, dev, tensorgen, shape, R, tier, n_approx=6, pp_build="auto"):
    """Per-sweep device time of each sweep kind on one configuration, with the kinds forced
    (three ALS sweeps, a PP initialisation, n_approx PP-approximated sweeps; the first ALS
    sweep is a warm-up), as in the paper's per-sweep comparison of Section 5.1."""
    prob = tensorgen.make_problem_device(shape, R, 0, eta=1e-2, dtype=tier, device=dev)
    X = prob.X.reshape(-1)
    plan = pp.Plan(shape, R, tier, tier, True, pp_build=pp_build)
    ws = plan.workspace(dev)
    A = [torch.from_numpy(a).to(dev) for a in prob.init]
    S = torch.zeros(len(shape) * R * R, dtype=torch.float64, device=dev)
    rec = pp.new_record(dev)
    nrm = torch.zeros(1, dtype=torch.float64, device=dev)
    pp.tensor_norm2(X, nrm)
    kinds = ["als"] * 3 + ["pp_init"] + ["pp_approx"] * n_approx
    recs, ms = pp.run(plan, X, None, A, S, float(nrm.item()), ws, rec, eps=0.1,
                      max_sweeps=len(kinds), replay=kinds, timing=True)
    got = [r["kind"] for r in recs]
    assert got == kinds, got
    per = {}
    for k in ("als", "pp_init", "pp_approx"):
        t = [m for i, (r, m) in enumerate(zip(recs, ms)) if r["kind"] == k and i > 0]
        per[k] = float(np.mean(t))
    d = plan.describe()
    out = {"shape": list(shape), "rank": R, "tier": tier, "ms": per,
           "pp_build_levels": d["pp_build_levels"], "workspace_GB": plan.workspace_bytes / 1e9,
           "pp_approx_speedup_vs_dt_sweep": per["als"] / per["pp_approx"],
           "pp_init_over_dt_sweep": per["pp_init"] / per["als"]}
    log(f"sweep kinds {shape} R {R} {tier}: DT {per['als']:.3f} ms, PP-init {per['pp_init']:.3f} ms, "
        f"PP-approx {per['pp_approx']:.3f} ms ({out['pp_approx_speedup_vs_dt_sweep']:.1f}x)")
    del X, ws, plan, prob
    torch.cuda.empty_cache()
    return out


PAPER_SWEEP_CONFIGS = (
    # order 3 with R = s (the rank cap is 128)
    ((64, 64, 64), 64), ((128, 128, 128), 128),
    # s = 960^(3/N), R = 50 for N = 3..6
    ((960,) * 3, 50), ((172,) * 4, 50), ((62,) * 5, 50), ((31,) * 6, 50),
)


def ablation_bench(args, torch, dev):
    """The second-order correction ablation of the synthetic collinearity experiments
    (Section 5.1): fit against time for dimension-tree ALS, PP with the second-order
    term V at eps = 0.1, and PP without it at eps = 0.1 and at the paper's conservative
    eps = 0.02.  Order-3 tensors with exact rank-R decompositions whose factor columns
    have collinearity C; each run stops at the first sweep whose fit changes by less than
    1e-5 (the paper's stopping tolerance) or after --abl-sweeps sweeps."""
    import paper_1811_10573_amd as pp
    import tensorgen
    s, R, C, sweeps = args.abl_size, args.abl_rank, args.abl_coll, args.abl_sweeps
    tdt = "f64" if args.tier == "f64" else "f32"
    variants = [("dt_als", 0.0, True), ("pp_v_eps0.1", 0.1, True), ("pp_noV_eps0.1", 0.1, False),
                ("pp_noV_eps0.02", 0.02, False)]
    per_seed = []
    curves = {}
    for seed in range(args.abl_seeds):
        prob = tensorgen.make_problem((s, s, s), R, seed=seed, eta=0.0, collinearity=C)
        X = torch.from_numpy(prob.X if tdt == "f64" else prob.X.astype(np.float32)).to(dev)
        nrm = torch.zeros(1, dtype=torch.float64, device=dev)
        pp.tensor_norm2(X, nrm)
        res = {}
        for name, eps, so in variants:
            plan = pp.Plan((s, s, s), R, tdt, args.tier, so)
            ws = plan.workspace(dev)
            A = [torch.from_numpy(a.copy()).to(dev) for a in prob.init]
            S = torch.zeros(3 * R * R, dtype=torch.float64, device=dev)
            rec = pp.new_record(dev)
            recs, ms = pp.run(plan, X, None, A, S, float(nrm.item()), ws, rec, eps=eps,
                              max_sweeps=sweeps)
            fits = [r["fit_est"] for r in recs]
            kinds = [r["kind"] for r in recs]
            stop = len(fits) - 1
            diverged = None
            for k in range(len(fits)):
                if not np.isfinite(fits[k]) or any(not np.isfinite(x) for x in recs[k]["rel_change"][:3]):
                    diverged = k
                    stop = max(0, k - 1)
                    break
                if k > 0 and abs(fits[k] - fits[k - 1]) < 1e-5:
                    stop = k
                    break
            t = np.cumsum(ms)
            # exact fit at the stopping sweep: the run is deterministic, so the same decisions
            # replayed up to that sweep give the factors it had there
            for a, a0 in zip(A, prob.init):
                a.copy_(torch.from_numpy(a0).to(dev).reshape(a.shape))
            pp.run(plan, X, None, A, S, float(nrm.item()), ws, rec, eps=eps, max_sweeps=stop + 1,
                   replay=kinds[:stop + 1], timing=False)
            r2 = torch.zeros(1, dtype=torch.float64, device=dev)
            pp.exact_residual2(plan, X, A, r2, ws)
            fit_exact = 1.0 - float(np.sqrt(max(0.0, r2.item()) / nrm.item()))
            res[name] = {"sweeps": stop + 1, "fit": fits[stop], "fit_exact": fit_exact,
                         "estimate_clamped": bool(any(f >= 1.0 for f in fits[:stop + 1])),
                         "time_ms": float(t[stop]),
                         "pp_approx": kinds[:stop + 1].count("pp_approx"),
                         "pp_init": kinds[:stop + 1].count("pp_init"),
                         "min_fit_after_5": float(min(fits[5:stop + 1])) if stop > 5 else None,
                         # time until the fit estimate first reaches 0.99 (None if never,
                         # or if the estimate was clamped at 1 before: then it is no guide)
                         "time_to_fit_0.99_ms": next(
                             (float(t[k]) for k in range(stop + 1) if fits[k] >= 0.99
                              and not any(f >= 1.0 for f in fits[:k + 1])), None),
                         "diverged_at_sweep": diverged}
            if seed == 0:
                idx = list(range(0, stop + 1, 10)) + ([stop] if stop % 10 else [])
                curves[name] = [[round(float(t[i]), 3), round(float(fits[i]), 7)] for i in idx]
            del ws, plan
        dt = res["dt_als"]
        for name, _, _ in variants[1:]:
            r = res[name]
            # both runs stopped by the same rule; a diverged run has no speed-up
            r["speedup_vs_dt_at_stop"] = (dt["time_ms"] / r["time_ms"]
                                          if r["diverged_at_sweep"] is None else None)
            r["exact_fit_minus_dt"] = r["fit_exact"] - dt["fit_exact"]
        per_seed.append(res)
        log(f"ablation seed {seed}: " + ", ".join(
            f"{k} {v['sweeps']} sw fit {v['fit_exact']:.6f} (est {v['fit']:.6f}) {v['time_ms']:.1f} ms"
            + (f" DIVERGED@{v['diverged_at_sweep']}" if v["diverged_at_sweep"] is not None else "")
            for k, v in res.items()))
        del X
    summary = {}
    for name, _, _ in variants:
        rows = [r[name] for r in per_seed]
        sp = [r.get("speedup_vs_dt_at_stop") for r in rows if r.get("speedup_vs_dt_at_stop")]
        summary[name] = {
            "median_sweeps": float(np.median([r["sweeps"] for r in rows])),
            "median_time_ms": float(np.median([r["time_ms"] for r in rows])),
            "median_fit_exact": float(np.median([r["fit_exact"] for r in rows])),
            "estimate_clamped_runs": sum(r["estimate_clamped"] for r in rows),
            "diverged": sum(r["diverged_at_sweep"] is not None for r in rows),
            "median_speedup_vs_dt": float(np.median(sp)) if sp else None,
            "runs_reaching_0.99": sum(r["time_to_fit_0.99_ms"] is not None for r in rows),
            "median_speedup_to_0.99": (float(np.median(
                [d["dt_als"]["time_to_fit_0.99_ms"] / r["time_to_fit_0.99_ms"]
                 for d, r in zip(per_seed, rows)
                 if r["time_to_fit_0.99_ms"] and d["dt_als"]["time_to_fit_0.99_ms"]]))
                if any(r["time_to_fit_0.99_ms"] for r in rows) else None),
        }
    line = {
        "metric": "time to |dfit| < 1e-5, second-order correction ablation (PP vs dimension-tree ALS)",
        "value": summary["pp_v_eps0.1"]["median_speedup_vs_dt"], "unit": "x (DT time / PP time)",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": tdt,
        "data": "synthetic (seeded exact-rank CP with collinear factor columns, tensorgen)",
        "config": {"workload": f"order-3 {s}^3 exact rank-{R} CP, factor collinearity {C}, "
                               f"R = {R}, {args.abl_seeds} seeds, at most {sweeps} sweeps",
                   "size": s, "rank": R, "collinearity": C, "seeds": args.abl_seeds},
        "summary": summary, "per_seed": per_seed, "curve_seed0_time_ms_fit": curves,
    }
    print(json.dumps(line), flush=True)


# source file of each kernel class whose HBM traffic has a committed counter summary
# sources whose SHA-256 (of their concatenation, in this order) the counter summary names
TRAFFIC_SOURCE = {"level1_gemm": ["k_level1.hip"], "pp_correct_ttv": ["k_ttv.hip", "tail_bodies.h"],
                  "k_b_gemm": ["k_batch.hip"]}


def measured_traffic(kernel, tier, shape, rank, workload=None):
    """HBM bytes per launch from the committed counter summary of this kernel and
    workload (named by tier, shape and rank, or by ``workload``), or None when there is
    none or the kernel source changed since."""
    import re
    stem = workload if workload is not None else f"{tier}_{'x'.join(map(str, shape))}_r{rank}"
    fn = os.path.join(ROOT, "profiles", f"{kernel}_{stem}_counters.md")
    if kernel not in TRAFFIC_SOURCE or not os.path.exists(fn):
        return None
    txt = open(fn).read()
    m = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    if not m or not h:
        return None
    if h.group(1) != kernel_source_hash(TRAFFIC_SOURCE[kernel]):
        return None
    return float(m.group(1))


def kernel_source_hash(srcs=("k_level1.hip",)):
    import hashlib
    d = os.path.join(ROOT, "paper_1811_10573_amd", "csrc")
    hsh = hashlib.sha256()
    for src in ([srcs] if isinstance(srcs, str) else srcs):
        hsh.update(open(os.path.join(d, src), "rb").read())
    return hsh.hexdigest()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tier", default="f32", choices=["f64", "f32", "bf16"])
    ap.add_argument("--size", type=int, default=800)
    ap.add_argument("--rank", type=int, default=50)
    ap.add_argument("--sweeps", type=int, default=200)
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--collinearity", type=float, default=0.9,
                    help="column collinearity of the planted factors (< 0: i.i.d. N(0,1) factors)")
    ap.add_argument("--order", type=int, default=3)
    ap.add_argument("--shape", default=None,
                    help="comma-separated mode sizes (overrides --size and --order)")
    ap.add_argument("--pp-build", default="auto", choices=["tree", "direct", "auto"],
                    help="operator build of the PP-ALS run (orders >= 4): the PP tree, every "
                         "operator straight from X, or the level count the plan's cost model picks")
    ap.add_argument("--dist", default="normal", choices=["normal", "uniform"],
                    help="distribution of the planted factors when --collinearity < 0")
    ap.add_argument("--eta", type=float, default=1e-3, help="relative noise level")
    ap.add_argument("--device-gen", action="store_true",
                    help="assemble the tensor on the GPU (tensorgen.make_problem_device)")
    ap.add_argument("--compare-f64", action="store_true",
                    help="replay the run's sweep kinds with the FP64 tier and report the difference")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dt", action="store_true")
    ap.add_argument("--workload", default="pp",
                    choices=["pp", "batch", "ablation", "tucker", "build", "sweeps", "tucker_sweeps"],
                    help="pp: the 800^3 decomposition (default); batch: 512 independent problems; "
                         "ablation: PP with and without the second-order term against DT-ALS")
    ap.add_argument("--abl-size", type=int, default=64)
    ap.add_argument("--abl-rank", type=int, default=64)
    ap.add_argument("--abl-coll", type=float, default=0.7)
    ap.add_argument("--abl-seeds", type=int, default=5)
    ap.add_argument("--abl-sweeps", type=int, default=3000)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64 tier, the 64^3 ALS and the 160^4 first-level legs")
    ap.add_argument("--oracle-cap", type=float, default=300.0,
                    help="seconds the oracle replay of the run's sweep kinds may take")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding of this path is a design note, not an implementation)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1811_10573_amd as pp
    import tensorgen

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(torch, dev)
        return
    if args.workload == "batch":
        batch_bench(args, torch, dev)
        return
    if args.workload == "ablation":
        ablation_bench(args, torch, dev)
        return
    if args.workload == "sweeps":
        res = [sweep_kinds_leg(pp, torch, dev, tensorgen, shape, R, tier)
               for tier in ("f64", "f32") for shape, R in PAPER_SWEEP_CONFIGS]
        res += [sweep_kinds_leg(pp, torch, dev, tensorgen, shape, R, "f64", pp_build="tree")
                for shape, R in PAPER_SWEEP_CONFIGS[3:]]
        print(json.dumps(res), flush=True)
        return
    if args.workload == "tucker_sweeps":
        res = [tucker_sweeps_leg(pp, torch, dev, tensorgen, shape, R) for shape, R in PAPER_TUCKER_CONFIGS]
        print(json.dumps(res), flush=True)
        return
    if args.workload == "build":
        res = [build_leg(pp, torch, dev, tensorgen, (160,) * 4, 64, "f32"),
               build_leg(pp, torch, dev, tensorgen, (160,) * 4, 64, "f64"),
               build_leg(pp, torch, dev, tensorgen, (48,) * 5, 32, "f32"),
               build_leg(pp, torch, dev, tensorgen, (24,) * 6, 16, "f32")]
        print(json.dumps(res), flush=True)
        return
    if args.workload == "tucker":
        s = args.size
        R = args.rank if args.rank != 50 else max(1, round(0.05 * s))
        out = tucker_leg(pp, torch, dev, tensorgen, s=s, R=R,
                         cpu_seconds=0.0 if args.no_cpu_baseline else args.cpu_seconds)
        print(json.dumps(out), flush=True)
        return
    s, R = args.size, args.rank
    shape = (s,) * args.order
    if args.shape:
        shape = tuple(int(v) for v in args.shape.split(","))
        s = max(shape)
    coll = args.collinearity if args.collinearity >= 0 else None
    log(f"generating {shape} rank-{R} planted tensor ({args.dist} factors, collinearity {coll}, "
        f"noise {args.eta}, seed {args.seed})")
    t0 = time.perf_counter()
    if args.device_gen:
        prob = tensorgen.make_problem_device(shape, R, args.seed, eta=args.eta, collinearity=coll,
                                             dist=args.dist, dtype="f64", device=dev)
        X64 = prob.X.reshape(-1)
    else:
        prob = tensorgen.make_problem(shape, R, seed=args.seed, eta=args.eta, collinearity=coll,
                                      dist=args.dist)
        X64 = None
    log(f"generated in {time.perf_counter() - t0:.1f} s")

    tdt = "f64" if args.tier == "f64" else "f32"
    plan = pp.Plan(shape, R, tdt, args.tier, True, pp_build=args.pp_build)
    build_levels = plan.describe()["pp_build_levels"]
    log(f"operator build: {args.pp_build} -> {build_levels} combined level(s)")
    if args.device_gen:
        X = X64 if tdt == "f64" else X64.to(torch.float32)
    elif tdt == "f64":
        X = torch.from_numpy(prob.X).to(dev)
    else:
        X = torch.from_numpy(prob.X.astype(np.float32)).to(dev)
    if tdt == "f32" and X64 is not None and not args.compare_f64:
        X64 = None
    Xb = None
    if args.tier == "bf16":
        Xb = torch.empty(X.numel(), dtype=torch.int16, device=dev)
        pp.cast_bf16(X, Xb)
    A0 = [torch.from_numpy(a).to(dev) for a in prob.init]
    A = [a.clone() for a in A0]
    S = torch.zeros(len(shape) * R * R, dtype=torch.float64, device=dev)
    ws = plan.workspace(dev)
    rec = pp.new_record(dev)
    nrm = torch.zeros(1, dtype=torch.float64, device=dev)
    pp.tensor_norm2(X, nrm)
    normX2 = float(nrm.item())
    log(f"workspace {plan.workspace_bytes / 2**30:.2f} GiB, ||X||^2 = {normX2:.6e}")

    def reset():
        for a, a0 in zip(A, A0):
            a.copy_(a0)

    def pp_run(timing=True):
        reset()
        return pp.run(plan, X, Xb, A, S, normX2, ws, rec, eps=args.eps, max_sweeps=args.sweeps,
                      timing=timing)

    for w in range(args.warmup):
        recs, ms = pp_run()
        torch.cuda.synchronize()
        log(f"warmup {w}: {len(recs)} sweeps, {sum(ms):.1f} ms device time")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for k in range(args.steps):
        recs, _ = pp_run(timing=False)
        done += len(recs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    # per-sweep device times (HIP events around every sweep) from one more, untimed step
    recs, ms = pp_run(timing=True)
    torch.cuda.synchronize()
    # one more step with per-kernel-class HIP events (they disable the graph replay of
    # PP-approximated sweeps, so they stay out of the timed steps)
    pp.get_profile(plan, reset=True)
    pp.set_profiling(plan, True)
    pp_run()
    torch.cuda.synchronize()
    pp.set_profiling(plan, False)
    prof = pp.get_profile(plan, reset=True)
    value = done / elapsed
    kinds = [r["kind"] for r in recs]
    log(f"timed {args.steps} steps: {done} sweeps in {elapsed:.3f} s -> {value:.1f} sweeps/s; "
        f"mix {{als: {kinds.count('als')}, pp_init: {kinds.count('pp_init')}, "
        f"pp_approx: {kinds.count('pp_approx')}}}")

    per_kind = {}
    for kind in ("als", "pp_init", "pp_approx"):
        t = [m for r, m in zip(recs, ms) if r["kind"] == kind]
        per_kind[kind] = {"count": len(t), "mean_ms": float(np.mean(t)) if t else None}
    res2 = torch.zeros(1, dtype=torch.float64, device=dev)
    pp.exact_residual2(plan, X, A, res2, ws)
    fit_pp = 1.0 - float(np.sqrt(res2.item() / normX2))
    A_pp = [a.clone() for a in A] if args.compare_f64 else None
    A_final = [a.cpu().numpy().reshape(sz, R) for a, sz in zip(A, shape)]

    out_dt = None
    speedup = None
    if not args.no_dt:
        reset()
        recs_dt, ms_dt = pp.run(plan, X, Xb, A, S, normX2, ws, rec, eps=0.0, max_sweeps=args.sweeps)
        torch.cuda.synchronize()
        pp.exact_residual2(plan, X, A, res2, ws)
        fit_dt = 1.0 - float(np.sqrt(res2.item() / normX2))
        target = min(recs[-1]["fit_est"], recs_dt[-1]["fit_est"])
        t_pp = time_to_fit(recs, ms, target)
        t_dt = time_to_fit(recs_dt, ms_dt, target)
        speedup = (t_dt / t_pp) if (t_pp and t_dt) else None
        out_dt = {
            "sweeps_per_s": len(recs_dt) / (sum(ms_dt) / 1e3),
            "mean_sweep_ms": float(np.mean(ms_dt)),
            "final_fit_exact": fit_dt,
            "time_to_equal_fit_ms": t_dt,
        }
        log(f"DT-ALS: {out_dt['sweeps_per_s']:.1f} sweeps/s, fit {fit_dt:.8f}; "
            f"PP fit {fit_pp:.8f}; equal-fit target {target:.8f}: PP {t_pp} ms vs DT {t_dt} ms")

    # roofline of the dominant kernel class of the timed region (among the classes
    # with algorithmic work)
    dom = max(((k, v) for k, v in prof.items() if v["flops"] > 0 or v["bytes"] > 0),
              key=lambda kv: kv[1]["total_ms"])
    name, st = dom
    mpeak = PEAK[{"f64": "f64_TFs", "f32": "f32_TFs", "bf16": "bf16_TFs"}[args.tier]]
    # the bound follows the arithmetic intensity against the ridge point of the tier
    mfma_bound = (name == "level1_gemm" and st["bytes"] > 0
                  and st["flops"] / st["bytes"] >= mpeak * 1e12 / (PEAK["hbm_GBs"] * 1e9))
    if mfma_bound:
        peak = mpeak
        achieved = st["flops"] / (st["total_ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak,
                "traffic": measured_traffic(name, args.tier, shape, R), "kernel": name,
                "launches": st["launches"], "avg_ms": st["avg_ms"],
                "work_per_launch": st["flops"] / max(1, st["launches"])}
    else:
        achieved = st["bytes"] / (st["total_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                "frac": achieved / PEAK["hbm_GBs"], "traffic": None, "kernel": name,
                "launches": st["launches"], "avg_ms": st["avg_ms"],
                "work_per_launch": st["bytes"] / max(1, st["launches"])}
    # the PP-correction contractions (HBM-bound) against the HBM peak
    roof_ttv = None
    st_t = prof.get("pp_correct_ttv")
    if st_t and st_t["launches"] > 0 and st_t["bytes"] > 0:
        ach = st_t["bytes"] / (st_t["total_ms"] * 1e-3) / 1e9
        roof_ttv = {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                    "frac": ach / PEAK["hbm_GBs"],
                    "traffic": measured_traffic("pp_correct_ttv", args.tier, shape, R),
                    "kernel": "pp_correct_ttv", "launches": st_t["launches"],
                    "avg_ms": st_t["avg_ms"],
                    "work_per_launch": st_t["bytes"] / max(1, st_t["launches"])}
    kernels = {}
    for k, v in prof.items():
        if v["launches"] == 0:
            continue
        e = {"launches": v["launches"], "total_ms": round(v["total_ms"], 3), "avg_ms": v["avg_ms"]}
        if v["flops"] > 0:
            e["TFLOP_s"] = v["flops"] / (v["total_ms"] * 1e-3) / 1e12
        if v["bytes"] > 0:
            e["GB_s"] = v["bytes"] / (v["total_ms"] * 1e-3) / 1e9
        kernels[k] = e

    vs64 = None
    if args.compare_f64 and args.tier != "f64":
        # the same decisions with the FP64 tier on the FP64 tensor
        if X64 is None:
            X64 = torch.from_numpy(prob.X).to(dev).reshape(-1)
        plan64 = pp.Plan(shape, R, "f64", "f64", True)
        ws64 = plan64.workspace(dev)
        A64 = [a.clone() for a in A0]
        S64 = torch.zeros_like(S)
        n64 = torch.zeros(1, dtype=torch.float64, device=dev)
        pp.tensor_norm2(X64, n64)
        recs64, _ = pp.run(plan64, X64, None, A64, S64, float(n64.item()), ws64, rec, eps=args.eps,
                           max_sweeps=len(recs), replay=kinds)
        pp.exact_residual2(plan64, X64, A64, res2, ws64)
        fit64 = 1.0 - float(np.sqrt(res2.item() / float(n64.item())))
        # this tier's final factors (the last timed step) on the FP64 tensor
        pp.exact_residual2(plan64, X64, A_pp, res2, ws64)
        fit_tier_on64 = 1.0 - float(np.sqrt(res2.item() / float(n64.item())))
        fdiff = max(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
                    for a, b in zip(A_pp, A64))
        vs64 = {"fit_f64_replay": fit64, "fit_this_tier_on_f64_tensor": fit_tier_on64,
                "fit_abs_diff": abs(fit_tier_on64 - fit64), "factor_rel_diff_max": fdiff}
        log(f"vs FP64 replay: fit {fit_tier_on64:.10f} vs {fit64:.10f}, factor rel diff {fdiff:.2e}")
        del ws64, X64
    # further legs of the default workload: the FP64 tier on the same decomposition, the
    # 64^3 ALS configuration and the first-level contractions of the 160^4 configuration
    extras = (not args.no_extras and args.tier == "f32" and shape == (800, 800, 800)
              and R == 50 and not args.device_gen)
    f64 = c1 = c3 = batch = tucker = build = sweep_cfgs = tucker_orders = None
    A_f64_replay = c1prob = None
    if extras:
        del ws
        torch.cuda.empty_cache()
        f64, A_f64_replay = f64_leg(pp, torch, dev, prob, shape, R, args.eps, args.sweeps, kinds,
                                    warmup=1, steps=2)
        c1, c1prob = c1_leg(pp, torch, dev, tensorgen)
        c3 = c3_level1_leg(pp, torch, dev, tensorgen)
        bl = batch_leg(args, torch, dev, cpu=False, warmup=1)
        batch = {k: bl[k] for k in ("value", "unit", "ms_per_step", "roofline", "batch")}
        batch["workload"] = bl["config"]["workload"]
        batch["batch"] = {k: v for k, v in batch["batch"].items() if k != "autotune"}
        tucker = tucker_leg(pp, torch, dev, tensorgen, s=800, R=40,
                            cpu_seconds=0.0 if args.no_cpu_baseline else 4.0)
        build = build_leg(pp, torch, dev, tensorgen, (160,) * 4, 64, "f32")
        sweep_cfgs = [sweep_kinds_leg(pp, torch, dev, tensorgen, shape, R, "f64")
                      for shape, R in PAPER_SWEEP_CONFIGS]
        tucker_orders = [tucker_sweeps_leg(pp, torch, dev, tensorgen, shp, r)
                         for shp, r in PAPER_TUCKER_CONFIGS]

    cpu = None
    vs_oracle = None
    if not args.no_cpu_baseline:
        Xh = prob.X if not args.device_gen else prob.X.cpu().numpy()
        if extras:
            log("float64 oracle replaying the run's sweep kinds on the host")
            rep = oracle_replay(Xh, prob.init, kinds, args.oracle_cap)
            per = rep["per_sweep_s"]
            counts = {k: kinds.count(k) for k in per}
            total = sum(counts[k] * per[k] for k in per if per[k] is not None)
            cpu = {"value": len(kinds) / total if total > 0 else None, "unit": "sweeps/s",
                   "cores": rep["threads"], "kind": "oracle",
                   "sample": (f"float64 oracle replaying this run's {len(kinds)} sweep kinds on "
                              f"the same tensor: {rep['sweeps']} sweeps in {rep['seconds']:.1f} s; "
                              f"per-kind mean times weighted by the mix {counts}"),
                   "per_sweep_s": per, "host_cpus": len(os.sched_getaffinity(0))}
            if rep["complete"]:
                f_or = rep["fit"]
                f32_fit = oracle_fit(Xh, A_final)
                f64_fit = oracle_fit(Xh, A_f64_replay)

                def fdiff(G):
                    return max(float(np.linalg.norm(g - o) / np.linalg.norm(o))
                               for g, o in zip(G, rep["A"]))
                vs_oracle = {
                    "what": "final fit of the GPU factors and of the float64 oracle's, both "
                            "evaluated by the oracle on the FP64 tensor, with this run's sweep "
                            "kinds replayed by the oracle and by the FP64 tier",
                    "oracle_fit": f_or,
                    "f32_fit": f32_fit, "f32_fit_rel_err": abs(f32_fit - f_or) / abs(f_or),
                    "f32_factor_rel_diff_max": fdiff(A_final),
                    "f64_fit": f64_fit, "f64_fit_rel_err": abs(f64_fit - f_or) / abs(f_or),
                    "f64_factor_rel_diff_max": fdiff(A_f64_replay),
                }
                log(f"vs oracle: fit {f_or:.12f}; FP32 rel err {vs_oracle['f32_fit_rel_err']:.2e}, "
                    f"FP64 rel err {vs_oracle['f64_fit_rel_err']:.2e}")
            if c1 is not None:
                from oracle import cp as ocp
                _, ref = ocp.cp_als(c1prob.X, c1prob.init, 20)
                c1["fit_rel_err_max_vs_oracle"] = max(abs(g - o.fit_est) / abs(o.fit_est)
                                                      for g, o in zip(c1["fits"], ref))
                c1["final_fit"] = c1["fits"][-1]
            if c1 is not None:
                del c1["fits"]
        else:
            log("timing the float64 oracle on the host (bounded sample)")
            cpu = cpu_baseline(Xh, prob.init, R, args.eps, kinds, args.cpu_seconds)
        log(f"oracle: {cpu['value']:.4f} sweeps/s projected for the same sweep mix")
    elif c1 is not None:
        del c1["fits"]

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16": "bf16-in/f32-acc"}[args.tier],
        "data": "synthetic (seeded planted CP + Gaussian noise, tensorgen)",
        "config": {
            "workload": (f"PP-CP-ALS, order-{len(shape)} {'x'.join(map(str, shape))} {tdt.upper()} "
                         f"tensor, planted rank-{R} CP with "
                         f"{'collinearity ' + str(coll) if coll is not None else ('U[0,1) factors' if args.dist == 'uniform' else 'N(0,1) factors')}, "
                         f"{args.eta:g} noise, decomposition rank {R}, eps={args.eps}, "
                         f"{args.sweeps} sweeps per step"),
            "shape": list(shape), "rank": R, "eps": args.eps, "sweeps_per_step": args.sweeps,
            "tier": args.tier, "seed": args.seed,
            "pp_build": args.pp_build, "pp_build_levels": build_levels,
            "generator": "device" if args.device_gen else "host",
        },
        "roofline": roof,
        "roofline_pp_ttv": roof_ttv,
        "cpu_baseline": cpu,
        "pp": {"final_fit_exact": fit_pp, "final_fit_est": recs[-1]["fit_est"], "per_kind": per_kind},
        "dt_als": out_dt,
        "pp_vs_dt_time_to_equal_fit": speedup,
        "vs_f64": vs64 if vs64 is not None else vs_oracle,
        "f64_tier": f64,
        "c1_als": c1,
        "c3_level1": c3,
        "c5_batch": batch,
        "f1_tucker": tucker,
        "f2_direct_build": build,
        "paper_sweep_configs_f64": sweep_cfgs,
        "paper_tucker_configs_f64": tucker_orders,
        "paper_reference": PAPER_NUMBERS,
        "kernels": kernels,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
