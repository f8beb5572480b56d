#!/usr/bin/env python3
"""Benchmark: LocalPower local-iteration throughput on one MI355X.

Default workload (the FP32 fused-path configuration): A is 262144 x 1024 FP32,
low-rank-plus-noise with a spectral gap sigma_16/sigma_17 = 1.2, k = 16,
m = 32 equal partitions, p = 4, T = 50 rounds, sign-fixing.  One step is one
full lp_run (50 rounds = 200 local iterations on every partition, with the
local orthonormalisations, alignments, aggregations and global orths).

Other workloads (--workload): bf16-1048576x2048 (Gaussian rows with a power-law
covariance stored BF16, k = 32, m = 64, p = 8, 4, 2, 1 for 10 rounds each, OPT)
and fp32-uneven-500000x4096 (k = 64, m = 100 lognormal partition sizes, p = 4,
T = 30, OPT).

value  = algorithmic bytes of A streamed per step (local iterations * n * d * b)
         / step time.
roofline.achieved = n * d * b bytes (HBM-bound kernels) or 4 n d k flops
(the matrix-core-bound two-pass kernel) / average duration of one local
multiply (HIP events around the first local multiply of every round, on the
library's stream, inside the timed steps: bracketing every launch would add a
few microseconds of stream time per launch to the timed steps; when the rounds
run split in two halves on two streams, one pair brackets both halves' launches,
which run back to back); peak = the published 8 TB/s or 157.3 TFLOP/s (FP32 matrix).
The library's autotuner picks the local-multiply variant before the timed
region; the measured read and copy bandwidth of simple streaming kernels is
reported beside the roofline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "local-iter GB/s (% HBM peak); rounds to sinθ≤1e-6; jobs/s + p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP32_MATRIX_PEAK_TFS = 157.3
CSRC = os.path.join(ROOT, "paper_2002_08014_amd", "csrc")

# workload name -> generator, local-multiply sources (for the counter-file hash),
# counter summary file, bound of the local multiply
WORKLOADS = {
    "fp32-262144x1024": dict(gen="make_fp32_262144x1024", sources=("k_local.hip", "k_mfma.hip"),
                             traffic="local_multiply_traffic.json", bound="hbm",
                             gram_traffic="local_multiply_gram_traffic.json"),
    "bf16-1048576x2048": dict(gen="make_bf16_1048576x2048", sources=("k_mfma_bf16.hip",),
                              traffic="local_multiply_bf16_traffic.json", bound="hbm"),
    "fp32-uneven-500000x4096": dict(gen="make_fp32_uneven_500000x4096", sources=("k_gemm.hip",),
                                    traffic="local_multiply_gemm_traffic.json", bound="mfma"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash(sources):
    h = hashlib.sha256()
    for f in sources:
        path = os.path.join(CSRC, f)
        if os.path.exists(path):
            h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def traffic_per_launch(spec):
    """HBM bytes per local-multiply launch from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", spec["traffic"])))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash(spec["sources"]):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(w, budget_s=12.0):
    """The FP64 oracle on a bounded sample: the first 4 partitions, one round of
    p = 4 local iterations repeated until the time budget is used."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    parts = 4
    rows = int(w.offsets[parts])
    A = w.A[:rows].to("cpu").to(torch.float64).numpy()
    sub = np.asarray(w.offsets[:parts + 1])
    d = A.shape[1]
    b = w.A.element_size()
    iters = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        oracle.localpower(A, sub, w.k, [4], "sign", w.Y0)
        iters += 4
    el = time.perf_counter() - t0
    gbs = iters * rows * d * b / el / 1e9
    return {"value": gbs, "unit": "GB/s", "cores": int(cores), "kind": "oracle",
            "sample": f"first {parts} of {w.m} partitions ({rows}x{d} upcast to FP64), "
                      f"{iters // 4} rounds of p=4 sign-fixing in {el:.1f} s; bytes counted at the "
                      f"stored width ({b} B) like the GPU figure"}


def precision_report(lp, synth, w, P, tuning, sched):
    """The precision form's operand modes and storage forms, each a full run of
    the workload's schedule with the Ritz finalisation, against the library's
    FP64 path (parity-tested against the FP64 oracle) on (a) the BF16-stored
    values and (b) the original FP64 matrix, same schedule and start: sin theta
    between the final subspaces and the largest relative Ritz-value error."""
    dev = w.A.device

    def run(Pr):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lp.lp_run(Pr, w.k, sched, w.mode, w.Y0, ritz=True)
        torch.cuda.synchronize()
        return r["Z"], r["ritz"].to("cpu").numpy(), time.perf_counter() - t0

    runs = {}
    log("precision: BF16 storage, BF16 operands (fused kernel)")
    runs["bf16_storage_bf16_operands"] = run(P)
    log("precision: BF16 storage, FP32 operands (two-pass kernel)")
    lp.lp_set_tuning(P, 1, tuning["chunk_rows"])
    runs["bf16_storage_fp32_operands"] = run(P)
    lp.lp_set_tuning(P, tuning["local_kernel"], tuning["chunk_rows"], tuning["cached_loads"])
    log("precision: FP64 on the BF16-stored values")
    A64 = w.A.to(torch.float64)
    P64 = lp.lp_create(A64, w.offsets, w.k)
    runs["fp64_on_bf16_values"] = run(P64)
    del P64, A64
    torch.cuda.empty_cache()
    log("precision: FP32 storage")
    w32 = synth.make_bf16_1048576x2048(device=dev, dtype=torch.float32)
    P32 = lp.lp_create(w32.A, w32.offsets, w32.k)
    lp.lp_autotune(P32, w32.k)
    runs["fp32_storage"] = run(P32)
    del P32, w32
    torch.cuda.empty_cache()
    log("precision: FP64 original matrix")
    w64 = synth.make_bf16_1048576x2048(device=dev, dtype=torch.float64)
    P64 = lp.lp_create(w64.A, w64.offsets, w64.k)
    ref = run(P64)
    del P64, w64
    torch.cuda.empty_cache()
    ref_b = runs["fp64_on_bf16_values"]
    out = {"reference": "library FP64 path, same schedule, start and Ritz finalisation",
           "fp64_original_s_per_run": round(ref[2], 3)}
    for name, (Z, ritz, sec) in runs.items():
        rec = {"s_per_run": round(sec, 3),
               "sin_vs_fp64_original": lp.lp_sin_theta(Z, ref[0]),
               "ritz_rel_err_vs_fp64_original": float(np.max(np.abs(ritz - ref[1]) / np.abs(ref[1])))}
        if name.startswith("bf16"):
            rec["sin_vs_fp64_same_values"] = lp.lp_sin_theta(Z, ref_b[0])
        out[name] = rec
    return out


def rounds_to(hist, thresholds=(1e-1, 1e-2, 1e-3, 1e-6)):
    out = {}
    for th in thresholds:
        hit = [i + 1 for i, v in enumerate(hist) if v <= th]
        out[f"{th:.0e}"] = hit[0] if hit else None
    return out


def convergence(lp, P, w, k):
    """Rounds to sin theta thresholds for p = 1, p = 4 (sign, OPT) and a decaying p, against
    the subspace of a long p = 1 run refined by Rayleigh-Ritz (the FP32 fixed point)."""
    ref = lp.lp_run(P, k, [1] * 150, "sign", w.Y0, ritz=True)["Z"]
    runs = {"p1": ([1] * 60, "sign"), "p4_sign": ([4] * 50, "sign"), "p4_opt": ([4] * 50, "opt"),
            "decay_4_2_1_x10": ([4] * 10 + [2] * 10 + [1] * 40, "sign")}
    out = {}
    for name, (sched, mode) in runs.items():
        h = lp.lp_run(P, k, sched, mode, w.Y0, U_ref=ref)["sin_hist"]
        out[name] = {"rounds_to": rounds_to(h), "final": float(h[-1]), "rounds": len(sched)}
    # no schedule: the truth-free stop rule with p halving from 4 (lp_solve)
    for mode in ("sign", "opt"):
        g = lp.lp_solve(P, k, mode, w.Y0, 4, 1e-6, 200)
        out[f"solve_{mode}_1e-6"] = {"status": g["status"], "rounds": g["stats"]["rounds"],
                                     "local_iters": g["stats"]["local_iters"],
                                     "p_used": [int(x) for x in g["p_used"]],
                                     "final": lp.lp_sin_theta(g["Z"], ref)}
    return out


def trends(lp, synth, w, k, rounds=40, ms=(8, 32, 128), ps=(1, 2, 4, 8, 16)):
    """sin theta after `rounds` rounds of fixed p (the error floor once p > 1) for
    several uniform partitionings of the same matrix, with eta of each partitioning
    (the paper's experiments on p and m; Corollary 1: the floor grows with p and
    with m, and OPT keeps it lower).  The reference is a long p = 1 run refined by
    Rayleigh-Ritz.  Runs through the local-Gram form (same method, fewer bytes)."""
    out = {}
    ref = None
    for m in ms:
        offs = synth.equal_offsets(w.n, m)
        P = lp.lp_create(w.A, offs, k)
        lp.lp_gram_enable(P)
        if ref is None:
            ref = lp.lp_run(P, k, [1] * 150, "sign", w.Y0, ritz=True)["Z"]
        eta, _ = lp.lp_eta(P, 300)
        row = {"eta": round(eta, 5)}
        for mode in ("sign", "opt"):
            row[mode] = {str(p): float(lp.lp_run(P, k, [p] * rounds, mode, w.Y0, U_ref=ref)["sin_hist"][-1])
                         for p in ps}
        out[f"m={m}"] = row
        lp.lp_destroy(P)
    return out


def make_job_mix(n_jobs, seed, device):
    """Seeded serving job list: d in {256, 512, 1024, 2048}, n = B d with B in
    [16, 64], m in {4, 16}, FP32 (k in {4, 8, 16, 32}) or BF16 (k in {4, 8, 12}),
    p0 = 4, target 1e-4; A low-rank-plus-noise with a gap of 1.5 at k, and the
    exact top-k subspace of the stored A for the accuracy check."""
    import synth
    rng = np.random.default_rng(seed)
    jobs = []
    for t in range(n_jobs):
        d = int(rng.choice([256, 512, 1024, 2048]))
        B = int(rng.integers(16, 65))
        m = int(rng.choice([4, 16]))
        bf16 = bool(rng.random() < 0.5)
        k = int(rng.choice([4, 8, 12] if bf16 else [4, 8, 16, 32]))
        mode = str(rng.choice(["sign", "opt"]))
        w = synth.make_small(B * d, d, k, m, seed=seed * 100003 + t,
                             dtype=torch.bfloat16 if bf16 else torch.float32, device=device, gap=1.5)
        A64 = w.A.to(torch.float64)
        _, V = torch.linalg.eigh(A64.T @ A64)
        del A64
        jobs.append((w, mode, V[:, -k:].contiguous()))
    torch.cuda.synchronize()
    return jobs


def serve_run(lp, jobs, rate, max_active, budget, seed):
    """Submit the jobs with Poisson arrivals at `rate` per second (all at once
    when rate is 0), collect every result; returns throughput and latencies."""
    S = lp.Server(hbm_budget_bytes=budget, max_active=max_active)
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, len(jobs)) if rate > 0 else np.zeros(len(jobs))
    arrivals = np.cumsum(gaps)
    ids = {}
    results = []
    t0 = time.perf_counter()
    for (w, mode, U), at in zip(jobs, arrivals):
        while time.perf_counter() - t0 < at:
            results += S.poll()
            time.sleep(0.0002)
        ids[S.submit(w.A, w.offsets, w.k, w.Y0, p0=4, mode=mode, target=1e-4, max_rounds=300)] = (U, w)
    while len(results) < len(jobs):
        S.wait(len(jobs) - len(results), timeout_s=1.0)
        results += S.poll()
    el = time.perf_counter() - t0
    S.close()
    lat = np.array([r["ms_total"] for r in results])
    worst = 0.0
    ok = 0
    errs = []
    for r in results:
        U, w = ids[r["id"]]
        ok += r["status"] == 0
        e = lp.lp_sin_theta(r["Z"], U)
        worst = max(worst, e)
        errs.append((e, {"d": w.d, "k": w.k, "m": w.m, "n": w.n, "dtype": str(w.A.dtype).split(".")[-1],
                         "rounds": r["rounds"], "local_iters": r["local_iters"], "change": r["change"],
                         "estimate": r["estimate"], "sin_theta_vs_truth": e}))
    errs.sort(key=lambda x: -x[0])
    return {"rate_per_s": rate if rate > 0 else "all at t=0", "max_active": max_active,
            "jobs": len(jobs), "jobs_per_s": round(len(jobs) / el, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "converged": ok, "max_sin_theta_vs_truth": worst, "worst_jobs": [x[1] for x in errs[:3]],
            "rounds_mean": round(float(np.mean([r["rounds"] for r in results])), 2)}


def serve_main(args):
    import paper_2002_08014_amd as lp
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n_jobs = args.jobs
    log(f"generating {n_jobs} serving jobs")
    jobs = make_job_mix(n_jobs, 4, dev)
    total_bytes = sum(w.A.numel() * w.A.element_size() for w, _, _ in jobs)
    budget = 64 << 30
    runs = []
    log("one job at a time, all submitted at t=0")
    runs.append(serve_run(lp, jobs, 0, 1, budget, 1))
    log("batched (16 active), all submitted at t=0")
    runs.append(serve_run(lp, jobs, 0, 16, budget, 1))
    for rate in args.rates:
        log(f"batched (16 active), Poisson arrivals at {rate}/s")
        runs.append(serve_run(lp, jobs, rate, 16, budget, 2))
    best = runs[1]
    out = {
        "metric": METRIC,
        "value": best["jobs_per_s"],
        "unit": "jobs/s",
        "n_gpus": 1,
        "steps": len(runs),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": f"serving: {n_jobs} LocalPower jobs (d 256..2048, n = 16d..64d, "
                               f"k 4..32, m 4/16, FP32 or BF16 A, p0 = 4 halved on stall, target 1e-4)",
                   "A_bytes_total": int(total_bytes)},
        "serving": runs,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fp32-262144x1024", choices=sorted(WORKLOADS) + ["serve"])
    ap.add_argument("--jobs", type=int, default=120, help="serving: number of jobs")
    ap.add_argument("--rates", type=float, nargs="*", default=[50.0, 200.0],
                    help="serving: Poisson arrival rates (jobs/s)")
    ap.add_argument("--rounds", type=int, default=0, help="override the workload's round count")
    ap.add_argument("--mode", default=None, choices=["sign", "opt", "vanilla"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-convergence", action="store_true")
    ap.add_argument("--gram", action="store_true",
                    help="local-Gram form: M_i = A_i^T A_i formed once (FP32/BF16 workloads)")
    ap.add_argument("--trends", action="store_true",
                    help="default workload: error floors over p and m and eta (Definition 2), "
                         "through the local-Gram form")
    ap.add_argument("--precision", action="store_true",
                    help="bf16 workload: both operand modes and both storage forms against FP64 runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the m LocalPower nodes are partitions on a single "
              f"device, so --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        serve_main(args)
        return
    import synth
    import paper_2002_08014_amd as lp

    spec = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"generating {args.workload} on the GPU")
    w = getattr(synth, spec["gen"])(device=dev)
    if args.mode:
        w.mode = args.mode
    if args.rounds:
        w.p_sched = (list(w.p_sched) * args.rounds)[:args.rounds]
    n, d, k = w.n, w.d, w.k
    torch.cuda.synchronize()
    P = lp.lp_create(w.A, w.offsets, k)
    log("autotuning the local multiply")
    tuning = lp.lp_autotune(P, k)
    log(f"chosen {tuning}")
    gram = None
    if args.gram:
        torch.cuda.synchronize()
        tg = time.perf_counter()
        lp.lp_gram_enable(P)
        torch.cuda.synchronize()
        gram = {"setup_ms": round((time.perf_counter() - tg) * 1e3, 3),
                "bytes_per_launch": w.m * d * d * 4}
        log(f"Gram form on: {gram}")
    buf = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
    read_gbs = lp.lp_bandwidth_probe(buf, 5)
    copy_gbs = lp.lp_copy_probe(buf[1 << 30:], buf[:1 << 30], 5)
    del buf
    torch.cuda.synchronize()
    sched = list(w.p_sched)
    iters_per_step = int(sum(sched))
    log(f"warmup x{args.warmup}")
    for _ in range(args.warmup):
        lp.lp_run(P, k, sched, w.mode, w.Y0, time_local=2)
    torch.cuda.synchronize()
    log(f"timed x{args.steps}")
    ms_local, launches, graph_rounds, split = 0.0, 0, 0, False
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = lp.lp_run(P, k, sched, w.mode, w.Y0, time_local=2)
        ms_local += r["stats"]["ms_local"]
        launches += r["stats"]["local_launches"]
        graph_rounds += r["stats"]["graph_rounds"]
        split = bool(r["stats"]["split_rounds"])
        log(f"step {i} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    bytes_iter = n * d * w.A.element_size()
    flops_iter = 4.0 * n * d * k
    value = args.steps * iters_per_step * bytes_iter / el / 1e9
    k1_ms = ms_local / max(launches, 1)
    if gram is not None:
        # the Gram form streams the m stacked d x d FP32 matrices per local multiply
        # (2 m d^2 k flops over 4 m d^2 bytes: k / 2 flop per byte)
        gbs = gram["bytes_per_launch"] / (k1_ms / 1e3) / 1e9
        if k / 2 > FP32_MATRIX_PEAK_TFS * 1e3 / HBM_PEAK_GBS:
            tfs = 2.0 * w.m * d * d * k / (k1_ms / 1e3) / 1e12
            roof = {"bound": "mfma", "achieved": round(tfs, 2), "peak": FP32_MATRIX_PEAK_TFS,
                    "unit": "TFLOP/s", "frac": round(tfs / FP32_MATRIX_PEAK_TFS, 4),
                    "hbm_gbs": round(gbs, 2)}
        else:
            roof = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4)}
    elif spec["bound"] == "hbm":
        achieved = bytes_iter / (k1_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4)}
    else:
        achieved = flops_iter / (k1_ms / 1e3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP32_MATRIX_PEAK_TFS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_MATRIX_PEAK_TFS, 4),
                "hbm_gbs": round(bytes_iter / (k1_ms / 1e3) / 1e9, 2)}
    if gram is None:
        traffic = traffic_per_launch(spec)
    elif "gram_traffic" in spec:
        traffic = traffic_per_launch({"traffic": spec["gram_traffic"], "sources": ("k_gemm.hip",)})
    else:
        traffic = None
    roof.update({"traffic": traffic, "kernel_ms": round(k1_ms, 5), "launches": launches,
                 "measured_read_gbs": round(read_gbs, 1), "measured_copy_gbs": round(copy_gbs, 1)})
    dtype = {torch.float32: "f32", torch.bfloat16: "bf16", torch.float64: "f64"}[w.A.dtype]
    ps = sorted(set(sched), reverse=True)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"localpower {dtype} A {n}x{d}, k={k}, m={w.m} "
                               f"{'lognormal' if args.workload.startswith('fp32-uneven') else 'equal'} "
                               f"partitions, p in {ps}, T={len(sched)} rounds, {w.mode} alignment"
                               + (", local-Gram form (value: A bytes per local iteration / time)"
                                  if gram else ""),
                   "n": n, "d": d, "k": k, "m": w.m, "p_sched": sched if len(ps) > 1 else ps[0],
                   "rounds": len(sched), "local_iters_per_step": iters_per_step,
                   "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
                   "tuning": tuning, "graph_rounds": graph_rounds, "split_rounds": split,
                   "rounds_total": args.steps * len(sched)},
        "roofline": roof,
    }
    if gram is not None:
        out["config"]["gram"] = gram
    if not args.no_convergence and args.workload == "fp32-262144x1024":
        log("convergence (rounds to sin theta thresholds)")
        out["convergence"] = convergence(lp, P, w, k)
    if args.trends and args.workload == "fp32-262144x1024":
        log("floors over p and m")
        out["trends"] = trends(lp, synth, w, k)
    if args.precision and args.workload == "bf16-1048576x2048":
        out["precision"] = precision_report(lp, synth, w, P, tuning, sched)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a sample)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
