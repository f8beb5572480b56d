#!/usr/bin/env python3
"""Benchmark: LocalPower local-iteration throughput on one MI355X.

Default run (no --workload): the headline workload and three sub-records.
* Headline, the FP32 fused-path configuration: A is 262144 x 1024 FP32,
  low-rank-plus-noise with a spectral gap sigma_16/sigma_17 = 1.2, k = 16,
  m = 32 equal partitions, p = 4, T = 50 rounds.  One step is two full lp_runs,
  one with sign-fixing and one with OPT alignment (2 x 50 rounds = 400 local
  iterations on every partition, with the local orthonormalisations, alignments,
  aggregations and global orths), plus rounds to sin theta thresholds against the
  exact subspace of the stored matrix.
* workloads: plain FP64 2000 x 100 (k = 5, m = 4, p = 4, T = 30, sign; latency and
  rounds), bf16-1048576x2048 (Gaussian rows with a power-law covariance stored
  BF16, k = 32, m = 64, p = 8, 4, 2, 1 for 10 rounds each, OPT) and
  fp32-uneven-500000x4096 (k = 64, m = 100 lognormal partition sizes, p = 4,
  T = 30, OPT), each with its own roofline, traffic and CPU baseline.
--workload NAME measures one workload alone (and `serve` the serving layer).

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
BF16_MATRIX_PEAK_TFS = 2500.0     # dense
SPLIT_TERMS = 6                   # BF16 products per FP32 product in the split-operand kernel
CSRC = os.path.join(ROOT, "paper_2002_08014_amd", "csrc")

# workload name -> generator, local-multiply sources (for the counter-file hash),
# counter summary file, bound of the local multiply, alignment modes timed per step
WORKLOADS = {
    "fp32-262144x1024": dict(gen="make_fp32_262144x1024", sources=("k_local.hip", "k_mfma.hip"),
                             traffic="local_multiply_traffic.json", bound="hbm",
                             gram_traffic="local_multiply_gram_traffic.json", modes=("sign", "opt"),
                             cpu_full=True),
    "plain-fp64-2000x100": dict(gen="make_fp64_2000x100", sources=("k_local.hip",), traffic=None,
                                bound="hbm", modes=("sign",), cpu_full=True, latency=True),
    "bf16-1048576x2048": dict(gen="make_bf16_1048576x2048", sources=("k_mfma_bf16.hip",),
                              traffic="local_multiply_bf16_traffic.json", bound="hbm", modes=("opt",)),
    "fp32-uneven-500000x4096": dict(gen="make_fp32_uneven_500000x4096", sources=("k_gemm.hip",),
                                    traffic="local_multiply_gemm_traffic.json", bound="mfma",
                                    modes=("opt",)),
}
SUB_WORKLOADS = ("plain-fp64-2000x100", "bf16-1048576x2048", "fp32-uneven-500000x4096")


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
    if not spec.get("traffic"):
        return None
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", spec["traffic"])))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash(spec["sources"]):
        return None
    return rec.get("bytes_per_launch")


def host_info():
    """CPU model, BLAS library and thread count of the host the oracle runs on."""
    info = {"cpu_model": None, "logical_cpus": os.cpu_count(), "blas": None, "blas_threads": None}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if blas:
            info["blas"] = f"{blas[0].get('internal_api')} {blas[0].get('version')} ({blas[0].get('architecture')})"
            info["blas_threads"] = int(blas[0].get("num_threads", 1))
    except Exception:
        pass
    return info


def cpu_baseline(w, sched, mode, budget_s=12.0, full=False):
    """The FP64 oracle on the host.  full: one complete run of the workload's
    schedule (affordable for the small workloads), else a bounded sample: the first
    4 partitions, rounds of the schedule's largest p repeated until the budget is
    used, with the full run's wall time extrapolated from the per-iteration time."""
    import oracle
    hi = host_info()
    b = w.A.element_size()
    d = w.d
    if full:
        A = w.A.to("cpu").to(torch.float64).numpy()
        t0 = time.perf_counter()
        runs = 0
        while True:
            oracle.localpower(A, w.offsets, w.k, sched, mode, w.Y0)
            runs += 1
            el = time.perf_counter() - t0
            if el >= budget_s or (runs >= 1 and el * (runs + 1) / runs > 3 * budget_s):
                break
        iters = runs * sum(sched)
        gbs = iters * w.n * d * b / el / 1e9
        sample = (f"{runs} full run(s) of the workload ({w.n}x{d} upcast to FP64, {len(sched)} rounds, "
                  f"{mode}) in {el:.1f} s; bytes counted at the stored width ({b} B) like the GPU figure")
        per_run = el / runs
        extrapolated = False
    else:
        parts = min(4, w.m)
        rows = int(w.offsets[parts])
        A = w.A[:rows].to("cpu").to(torch.float64).numpy()
        sub = np.asarray(w.offsets[:parts + 1])
        p = max(sched)
        iters = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            oracle.localpower(A, sub, w.k, [p], mode, w.Y0)
            iters += p
        el = time.perf_counter() - t0
        gbs = iters * rows * d * b / el / 1e9
        sample = (f"first {parts} of {w.m} partitions ({rows}x{d} upcast to FP64), {iters // p} rounds "
                  f"of p={p} {mode} in {el:.1f} s; bytes counted at the stored width ({b} B) like the GPU "
                  f"figure")
        per_run = el / iters * sum(sched) * (w.n / rows)
        extrapolated = True
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": int(hi["blas_threads"] or os.cpu_count()),
            "kind": "oracle", "sample": sample, "cpu_model": hi["cpu_model"], "blas": hi["blas"],
            "s_per_full_run": round(per_run, 3), "full_run_extrapolated": extrapolated}


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


def exact_subspace(A, k):
    """Top-k right singular vectors of the stored A: the FP64 Gram A^T A summed over
    row blocks on the GPU, its symmetric eigendecomposition on the host (LAPACK)."""
    n, d = A.shape
    G = torch.zeros(d, d, dtype=torch.float64, device=A.device)
    step = max(1, (1 << 27) // d)
    for r0 in range(0, n, step):
        B = A[r0:r0 + step].to(torch.float64)
        G += B.T @ B
    lam, V = np.linalg.eigh(G.cpu().numpy())
    order = np.argsort(lam)[::-1]
    return torch.as_tensor(np.ascontiguousarray(V[:, order[:k]]), device=A.device), lam[order]


def convergence(lp, P, w, k, U):
    """Rounds to sin theta thresholds against the exact subspace U of the stored
    matrix for p = 1, p = 4 (sign, OPT) and a decaying p, and the truth-free solve."""
    runs = {"p1": ([1] * 60, "sign"), "p4_sign": ([4] * 50, "sign"), "p4_opt": ([4] * 50, "opt"),
            "decay_4_2_1_x10": ([4] * 10 + [2] * 10 + [1] * 40, "sign")}
    out = {"reference": "exact top-k subspace of the stored matrix (FP64 Gram, LAPACK eigh)"}
    for name, (sched, mode) in runs.items():
        h = lp.lp_run(P, k, sched, mode, w.Y0, U_ref=U)["sin_hist"]
        out[name] = {"rounds_to": rounds_to(h), "final": float(h[-1]), "rounds": len(sched)}
    # no schedule: the truth-free stop rule with p halving from 4 (lp_solve)
    for mode in ("sign", "opt"):
        g = lp.lp_solve(P, k, mode, w.Y0, 4, 1e-6, 200)
        out[f"solve_{mode}_1e-6"] = {"status": g["status"], "rounds": g["stats"]["rounds"],
                                     "local_iters": g["stats"]["local_iters"],
                                     "p_used": [int(x) for x in g["p_used"]],
                                     "final": lp.lp_sin_theta(g["Z"], U)}
    return out


def trends(lp, synth, w, k, rounds=40, ms=(8, 32, 128), ps=(1, 2, 4, 8, 16)):
    """sin theta after `rounds` rounds of fixed p (the error floor once p > 1) for
    several uniform partitionings of the same matrix, with eta of each partitioning
    (the paper's experiments on p and m; Corollary 1: the floor grows with p and
    with m, and OPT keeps it lower).  The reference is a long p = 1 run refined by
    Rayleigh-Ritz.  Runs through the local-Gram form (same method, fewer bytes)."""
    out = {}
    ref = exact_subspace(w.A, k)[0]
    for m in ms:
        offs = synth.equal_offsets(w.n, m)
        P = lp.lp_create(w.A, offs, k)
        lp.lp_gram_enable(P)
        eta, _ = lp.lp_eta(P, 300)
        row = {"eta": round(eta, 5)}
        for mode in ("sign", "opt"):
            row[mode] = {str(p): float(lp.lp_run(P, k, [p] * rounds, mode, w.Y0, U_ref=ref)["sin_hist"][-1])
                         for p in ps}
        out[f"m={m}"] = row
        lp.lp_destroy(P)
    return out


def make_job_mix(n_jobs, seed):
    """Seeded serving job list (the serving configuration): d in {256, 512, 1024, 2048, 4096},
    n = B d with B uniform in [16, 256], k in {4, 8, 16, 32, 64} (k <= d), m in
    {4, 16, 64} equal partitions, sign or OPT alignment, p0 = 4, target 1e-4.  Each
    job's A is the exact-truth matrix (lp_generate: gap 1.2 after sigma_k, decay 0.97)
    generated by the server at admission from the job's seed, which also draws its
    start; its exact top-k subspace is known without an eigendecomposition."""
    rng = np.random.default_rng(seed)
    jobs = []
    for t in range(n_jobs):
        d = int(rng.choice([256, 512, 1024, 2048, 4096]))
        B = int(rng.integers(16, 257))
        k = int(rng.choice([4, 8, 16, 32, 64]))
        m = int(rng.choice([4, 16, 64]))
        mode = str(rng.choice(["sign", "opt"]))
        jobs.append({"n": B * d, "d": d, "k": min(k, d), "m": m, "mode": mode,
                     "seed": int(seed) * 1_000_003 + t})
    return jobs


def serve_run(lp, synth, jobs, dtype, rate, max_active, budget, seed, truth):
    """Submit the jobs (A generated at admission) with Poisson arrivals at `rate` per
    second, collect every result; returns throughput, latencies and accuracy."""
    S = lp.Server(hbm_budget_bytes=budget, max_active=max_active)
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, len(jobs)))
    ids = {}
    results = []
    t0 = time.perf_counter()
    for j, at in zip(jobs, arrivals):
        while time.perf_counter() - t0 < at:
            results += S.poll()
            time.sleep(0.0002)
        offs = synth.equal_offsets(j["n"], j["m"])
        jid = S.submit(None, offs, j["k"], None, p0=4, mode=j["mode"], target=1e-4, max_rounds=400,
                       gen=(j["n"], j["d"], dtype, j["seed"], 1.2, 0.97))
        ids[jid] = j
    last_report = time.perf_counter()
    while len(results) < len(jobs):
        S.wait(len(jobs) - len(results), timeout_s=1.0)
        results += S.poll()
        if time.perf_counter() - last_report > 30:
            last_report = time.perf_counter()
            log(f"  {len(results)} of {len(jobs)} jobs done")
    el = time.perf_counter() - t0
    S.close()
    lat = np.array([r["ms_total"] for r in results])
    worst, ok, errs = 0.0, 0, []
    for r in results:
        j = ids[r["id"]]
        ok += r["status"] == 0
        e = lp.lp_sin_theta(r["Z"], truth[(j["d"], j["k"], j["seed"])])
        worst = max(worst, e)
        errs.append((e, dict(j, rounds=r["rounds"], local_iters=r["local_iters"],
                             sin_theta_vs_truth=e, status=r["status"])))
    errs.sort(key=lambda x: -x[0])
    return {"rate_per_s": rate, "max_active": max_active, "jobs": len(jobs),
            "jobs_per_s": round(len(jobs) / el, 2), "wall_s": round(el, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "converged": ok, "within_1e-4": int(sum(1 for e, _ in errs if e <= 1e-4)),
            "max_sin_theta_vs_truth": worst, "worst_jobs": [x[1] for x in errs[:2]],
            "local_iters_mean": round(float(np.mean([r["local_iters"] for r in results])), 2)}


def serve_main(args):
    """Serving: the same seeded job list in two legs at every arrival rate: all FP32
    one job at a time (the plain per-job path) and all BF16 batched (--max-active, 16 by default,
    continuous batching).  Every job must end within 1e-4 of its exact subspace."""
    import synth
    import paper_2002_08014_amd as lp
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    jobs = make_job_mix(args.jobs, 4)
    log(f"{len(jobs)} jobs per rate; exact subspaces from the generator")
    truth = {}
    for j in jobs:
        key = (j["d"], j["k"], j["seed"])
        if key not in truth:
            truth[key] = lp.lp_generate(j["n"], j["d"], j["k"], 1.2, 0.97, j["seed"], dtype=None)[1]
    torch.cuda.synchronize()
    elems = sum(j["n"] * j["d"] for j in jobs)
    budget = 160 << 30
    legs = {"fp32_one_at_a_time": (torch.float32, 1), "bf16_batched": (torch.bfloat16, args.max_active)}
    runs = {leg: [] for leg in legs}
    for rate in args.rates:
        for leg, (dtype, active) in legs.items():
            log(f"{leg}: Poisson arrivals at {rate}/s")
            runs[leg].append(serve_run(lp, synth, jobs, dtype, rate, active, budget, 7, truth))
            log(f"  {runs[leg][-1]['jobs_per_s']} jobs/s, p50 {runs[leg][-1]['p50_ms']} ms, "
                f"p99 {runs[leg][-1]['p99_ms']} ms, worst sin theta {runs[leg][-1]['max_sin_theta_vs_truth']:.2e}")
    top = max(range(len(args.rates)), key=lambda i: args.rates[i])
    bf, fp = runs["bf16_batched"][top], runs["fp32_one_at_a_time"][top]
    out = {
        "metric": METRIC,
        "value": bf["jobs_per_s"],
        "unit": "jobs/s",
        "n_gpus": 1,
        "steps": len(args.rates) * len(legs),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"serving: {len(jobs)} LocalPower jobs per rate (d 256..4096, n = 16d..256d, "
                               f"k 4..64, m 4/16/64, p0 = 4 halved on stall, target 1e-4), A generated at "
                               f"admission; value = BF16 batched jobs/s at {args.rates[top]}/s",
                   "A_elements_per_rate": int(elems),
                   "fp32_one_at_a_time_jobs_per_s": fp["jobs_per_s"],
                   "bf16_batched_over_fp32": round(bf["jobs_per_s"] / fp["jobs_per_s"], 3)},
        "serving": runs,
    }
    print(json.dumps(out), flush=True)


def load_balance(lp, w, k, local_kernel=1):
    """How evenly one two-pass local multiply over the uneven partitions uses the
    GPU, from per-workgroup start/end stamps (lp_profile_local_multiply, the
    benchmark's kernel form at the default work-item size): workgroup busy times,
    the busy time per row of every partition, and per pass the busy fraction of the
    launch (sum of busy times over span x the largest number of workgroups seen
    running at once)."""
    P = lp.lp_create(w.A, w.offsets, k)
    lp.lp_set_tuning(P, local_kernel, 0)
    cr = lp.lp_get_tuning(P)["chunk_rows"]
    Z = np.linalg.qr(np.random.default_rng(0).standard_normal((w.d, k)))[0]
    st = lp.lp_profile_local_multiply(P, k, Z)
    lp.lp_destroy(P)
    item_part, item_rows = [], []
    for i in range(w.m):
        for r in range(int(w.offsets[i]), int(w.offsets[i + 1]), cr):
            item_part.append(i)
            item_rows.append(min(cr, int(w.offsets[i + 1]) - r))
    item_part, item_rows = np.array(item_part), np.array(item_rows)
    out = {"local_kernel": int(local_kernel), "work_item_rows": int(cr), "items": int(len(item_rows)),
           "workgroups": int(len(st))}
    busy_part = np.zeros(w.m)
    for ps in (1, 2):
        sel = st[st[:, 0] == ps]
        busy = sel[:, 3] - sel[:, 2]
        live = busy > 0
        full = live & (item_rows[sel[:, 1].astype(int)] == cr)
        ev = sorted([(t, 1) for t in sel[live, 2]] + [(t, -1) for t in sel[live, 3]])
        cur = peak = 0
        for _, dlt in ev:
            cur += dlt
            peak = max(peak, cur)
        span = float(sel[live, 3].max() - sel[live, 2].min())
        np.add.at(busy_part, item_part[sel[:, 1].astype(int)], busy)
        out[f"pass{ps}"] = {"span_us": round(span, 1), "peak_concurrent_workgroups": int(peak),
                            "busy_fraction": round(float(busy[live].sum()) / (span * peak), 4),
                            "workgroup_busy_us_max": round(float(busy[live].max()), 2),
                            "workgroup_busy_us_min": round(float(busy[live].min()), 2),
                            "full_item_busy_max_over_min": round(float(busy[full].max() / busy[full].min()), 3)}
    rate = busy_part / np.diff(np.asarray(w.offsets))
    out["partition_busy_us_per_row_max_over_min"] = round(float(rate.max() / rate.min()), 3)
    out["partition_rows_max_over_min"] = round(float(np.diff(w.offsets).max() / np.diff(w.offsets).min()), 2)
    return out


def measure(lp, synth, name, args, steps, warmup, headline=False):
    """Generate one workload, autotune, time `steps` steps (each step runs the
    workload's schedule once per alignment mode) after `warmup` untimed ones, and
    return its record (value, roofline, traffic, CPU baseline, ...)."""
    spec = WORKLOADS[name]
    dev = torch.device("cuda:0")
    log(f"generating {name} on the GPU")
    if headline and args.k:
        # the same matrix at another rank (the counter record applies to k = 16 only;
        # after autotuning, a k <= 8 run on the vector-ALU kernel takes its own)
        w = getattr(synth, spec["gen"])(device=dev, k=args.k)
        if args.k != 16:
            spec = dict(spec, traffic=None)
    else:
        w = getattr(synth, spec["gen"])(device=dev)
    modes = (args.mode,) if args.mode else spec["modes"]
    if args.rounds:
        w.p_sched = (list(w.p_sched) * args.rounds)[:args.rounds]
    n, d, k = w.n, w.d, w.k
    torch.cuda.synchronize()
    P = lp.lp_create(w.A, w.offsets, k)
    log("autotuning the local multiply")
    tuning = lp.lp_autotune(P, k)
    log(f"chosen {tuning}")
    split_products = spec["bound"] == "mfma" and tuning["local_kernel"] == 11
    if headline and args.k and args.k <= 8 and tuning["local_kernel"] == 0:
        # the fused vector-ALU kernel (its committed counters are for k = 8)
        spec = dict(spec, sources=("k_valu.hip",), bound="hbm",
                    traffic="local_multiply_valu_traffic.json" if args.k == 8 else None)
    if split_products:
        # the two-pass kernel on BF16 matrix cores with exactly split FP32 operands
        spec = dict(spec, sources=("k_gemm3.hip",), traffic="local_multiply_gemm3_traffic.json")
    gram = None
    if headline and args.gram:
        torch.cuda.synchronize()
        tg = time.perf_counter()
        lp.lp_gram_enable(P)
        torch.cuda.synchronize()
        gram = {"setup_ms": round((time.perf_counter() - tg) * 1e3, 3),
                "bytes_per_launch": w.m * d * d * 4}
        log(f"Gram form on: {gram}")
    read_gbs = copy_gbs = None
    if headline:
        buf = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
        read_gbs = lp.lp_bandwidth_probe(buf, 5)
        copy_gbs = lp.lp_copy_probe(buf[1 << 30:], buf[:1 << 30], 5)
        del buf
    torch.cuda.synchronize()
    sched = list(w.p_sched)
    iters_per_step = int(sum(sched)) * len(modes)

    def step():
        st = []
        for mode in modes:
            r = lp.lp_run(P, k, sched, mode, w.Y0, time_local=2)
            st.append(r["stats"])
        return st

    log(f"warmup x{warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log(f"timed x{steps}")
    ms_local, launches, graph_rounds, split = 0.0, 0, 0, False
    t0 = time.perf_counter()
    for i in range(steps):
        for stt in step():
            ms_local += stt["ms_local"]
            launches += stt["local_launches"]
            graph_rounds += stt["graph_rounds"]
            split = bool(stt["split_rounds"])
        if headline or i % 10 == 0:
            log(f"step {i} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    bytes_iter = n * d * w.A.element_size()
    flops_iter = 4.0 * n * d * k
    value = steps * iters_per_step * bytes_iter / el / 1e9
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
    elif split_products:
        # the contraction runs as SPLIT_TERMS BF16 products per FP32 product: its
        # roof is the BF16 matrix peak over the BF16 flops issued
        fp32_tfs = flops_iter / (k1_ms / 1e3) / 1e12
        achieved = SPLIT_TERMS * fp32_tfs
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": BF16_MATRIX_PEAK_TFS,
                "unit": "TFLOP/s", "frac": round(achieved / BF16_MATRIX_PEAK_TFS, 4),
                "fp32_equivalent_tflops": round(fp32_tfs, 2),
                "fp32_equivalent_frac_of_fp32_matrix_peak": round(fp32_tfs / FP32_MATRIX_PEAK_TFS, 4),
                "hbm_gbs": round(bytes_iter / (k1_ms / 1e3) / 1e9, 2)}
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
    roof.update({"traffic": traffic, "kernel_ms": round(k1_ms, 5), "launches": launches})
    if headline:
        roof.update({"measured_read_gbs": round(read_gbs, 1), "measured_copy_gbs": round(copy_gbs, 1)})
    if spec.get("latency"):
        roof["note"] = (f"latency-bound: {bytes_iter} B of A per local multiply, far below what "
                        "fills the GPU; the step time is launch and small-kernel latency")
    dtype = {torch.float32: "f32", torch.bfloat16: "bf16", torch.float64: "f64"}[w.A.dtype]
    ps = sorted(set(sched), reverse=True)
    part = "lognormal" if name.startswith("fp32-uneven") else "equal"
    rec = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(el / steps * 1e3, 3),
        "dtype": dtype,
        "config": {"workload": f"localpower {dtype} A {n}x{d}, k={k}, m={w.m} {part} partitions, "
                               f"p in {ps}, T={len(sched)} rounds, {' + '.join(modes)} alignment"
                               + (" (one run of each per step)" if len(modes) > 1 else "")
                               + (", local-Gram form (value: A bytes per local iteration / time)"
                                  if gram else ""),
                   "n": n, "d": d, "k": k, "m": w.m, "p_sched": sched if len(ps) > 1 else ps[0],
                   "rounds": len(sched), "modes": list(modes), "local_iters_per_step": iters_per_step,
                   "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
                   "tuning": tuning, "graph_rounds": graph_rounds, "split_rounds": split,
                   "rounds_total": steps * len(sched) * len(modes)},
        "roofline": roof,
    }
    if gram is not None:
        rec["config"]["gram"] = gram
    if headline and not args.no_convergence and name == "fp32-262144x1024":
        log("convergence (rounds to sin theta thresholds against the exact subspace)")
        U, _ = exact_subspace(w.A, k)
        rec["convergence"] = convergence(lp, P, w, k, U)
    if name == "plain-fp64-2000x100" and not args.no_convergence:
        U, _ = exact_subspace(w.A, k)
        rec["convergence"] = {}
        for label, (sch, md) in {"p1": ([1] * 30, "sign"), "p4_sign": (sched, "sign"),
                                 "p4_opt": (sched, "opt"), "p4_vanilla": (sched, "vanilla"),
                                 "decay_8_4_2_1_x10": ([8] * 10 + [4] * 10 + [2] * 10 + [1] * 10, "sign")
                                 }.items():
            h = lp.lp_run(P, k, sch, md, w.Y0, U_ref=U)["sin_hist"]
            rec["convergence"][label] = {"rounds_to": rounds_to(h, (1e-1, 1e-2, 1e-3, 1e-6, 1e-10)),
                                         "final": float(h[-1]), "rounds": len(sch)}
        rec["ms_per_run"] = round(el / steps / len(modes) * 1e3, 4)
    if headline and args.trends and name == "fp32-262144x1024":
        log("floors over p and m")
        rec["trends"] = trends(lp, synth, w, k)
    if name == "fp32-uneven-500000x4096":
        log("load balance of the uneven partitions (workgroup stamps)")
        rec["load_balance"] = load_balance(lp, w, k, tuning["local_kernel"])
    if args.precision and name == "bf16-1048576x2048":
        rec["precision"] = precision_report(lp, synth, w, P, tuning, sched)
    if not args.no_cpu_baseline:
        log("cpu baseline (the oracle)")
        rec["cpu_baseline"] = cpu_baseline(w, sched, modes[0], full=spec.get("cpu_full", False))
    lp.lp_destroy(P)
    del w, P
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None, choices=sorted(WORKLOADS) + ["serve"],
                    help="one workload alone (default: the headline plus the sub-records)")
    ap.add_argument("--jobs", type=int, default=200, help="serving: jobs per arrival rate")
    ap.add_argument("--max-active", type=int, default=16,
                    help="serving: jobs admitted at once in the batched BF16 leg")
    ap.add_argument("--rates", type=float, nargs="*", default=[10.0, 25.0, 50.0, 100.0, 200.0, 500.0],
                    help="serving: Poisson arrival rates (jobs/s)")
    ap.add_argument("--rounds", type=int, default=0, help="override the workload's round count")
    ap.add_argument("--mode", default=None, choices=["sign", "opt", "vanilla"])
    ap.add_argument("--k", type=int, default=0,
                    help="run the workload's matrix at this rank (k <= 8: the vector-ALU kernel)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-convergence", action="store_true")
    ap.add_argument("--no-sub", action="store_true", help="default run: the headline workload only")
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

    torch.cuda.set_device(torch.device("cuda:0"))
    name = args.workload or "fp32-262144x1024"
    out = measure(lp, synth, name, args, args.steps, args.warmup, headline=True)
    out.update({"n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "data": "synthetic"})
    if args.workload is None and not args.no_sub:
        out["workloads"] = {}
        for sub in SUB_WORKLOADS:
            steps = 20 if sub == "plain-fp64-2000x100" else 3
            out["workloads"][sub] = measure(lp, synth, sub, args, steps, 1)
    keys = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
            "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"]
    line = {k2: out[k2] for k2 in keys if k2 in out}
    line.update({k2: v for k2, v in out.items() if k2 not in line})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
