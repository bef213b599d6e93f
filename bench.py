"""Benchmark: logL + all-branch-gradient evaluations per second on one MI355X.

Workload (default): Yule tree with N=1000 tips, branch lengths ~ Exp(mean
0.01), random non-reversible 4-state Q, 4 discrete-gamma categories
(shape 0.5), 2000 site patterns simulated down the tree, weights ~ U{1..20},
per-node rescaling, gradient for all 1998 branches; FP64.  --workload C5
runs the 20-state workload (N=500, S=3000), C4 the 61-state codon workload
on the split-BF16 matrix-core path.

A step is one full evaluation through the C-ABI device entry point
(transition matrices, post-order pass, root, pre-order pass with the fused
gradient, per-branch reduction) on inputs already resident in HBM.

    python bench.py [--steps K] [--warmup W] [--precision fp64|fp32|split]
                    [--workload C2|C4|C5]

Prints one JSON line: `value` is K evaluations over the wall clock around
them; `eval_time_us` the median / p5 / p95 of per-evaluation HIP-event
durations; ``roofline`` the dominant kernel's bytes per launch (the
accounting of `algorithmic_bytes`, with the on-chip lower bound beside it) over
its mean duration, measured with HIP events recorded by the library on the
stream the kernel runs on; ``cpu_baseline`` the CPU oracle on bounded
samples (see `cpu_baseline`).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "logL+full-gradient evals/sec, N=1000 4-state; p50/p99 served latency"


def algorithmic_bytes(n_tips, n_patterns, n_states, n_cats, elem_bytes):
    """Bytes the method moves per evaluation (the accounting used for `frac`).

    V = K m S elem_bytes is one partial vector, I' = N - 2 internal non-root
    nodes.  Each stored message (P_k p_k) is written once and read twice (by
    the parent in the post-order pass and in the pre-order pass), each
    pre-order vector q is written once and read once, and each pass reads
    the tip codes (N S bytes) and the transition matrices |P|:
        evaluation = 5 I' V + 2 N S + 2 |P|,
        post-order kernel = 2 I' V + N S + |P|  (message write, parent read),
        pre-order kernel  = 3 I' V + N S + |P|  (message read, q write and read).
    """
    V = n_cats * n_states * n_patterns * elem_bytes
    I = n_tips - 2
    P = (2 * n_tips - 2) * n_cats * n_states * n_states * elem_bytes
    tips = n_tips * n_patterns
    return {"post": 2 * I * V + tips + P, "pre": 3 * I * V + tips + P,
            "eval": 5 * I * V + 2 * tips + 2 * P, "V": V, "P": P, "tips": tips}


def onchip_bytes(n_tips, n_patterns, n_states, n_cats, elem_bytes):
    """Lower bound when children's messages and every q stay on chip.

    The messages of one pass do not fit on chip, so the post-order kernel
    writes each once and the pre-order kernel reads each once (I' V each);
    both read the tip codes and |P|, and the pre-order kernel writes one
    gradient partial per branch and tile (8 (2N - 2) K ceil(S / 16) bytes).
    The depth-first clade walks of the 4-state kernels approach this."""
    V = n_cats * n_states * n_patterns * elem_bytes
    I = n_tips - 2
    P = (2 * n_tips - 2) * n_cats * n_states * n_states * elem_bytes
    tips = n_tips * n_patterns
    partials = 8 * (2 * n_tips - 2) * n_cats * ((n_patterns + 15) // 16)
    post = I * V + tips + P
    pre = I * V + tips + P + partials
    return {"post": post, "pre": pre, "eval": post + pre}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_cores():
    """Host cores this process may use, at most 16 (one GPU's CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_args(w, patterns=None):
    masks, weights = w.tip_masks(), w.weights
    if patterns is not None:
        masks, weights = masks[:, patterns], weights[patterns]
    return (w.parent, w.t, w.Q, w.pi, w.rates, w.cat_weights, masks, weights)


def _linear_chunk(job):
    """One worker of the all-core O(N) run: its share of the patterns."""
    from threadpoolctl import threadpool_limits
    import oracle
    w, patterns = job
    with threadpool_limits(1):
        r = oracle.linear_gradient(*_oracle_args(w, patterns))
    return r["logL"], r["grad"]


def _naive_chunk(job):
    """One worker of the all-core naive run: a pruning pass per branch of its share."""
    from threadpoolctl import threadpool_limits
    import oracle
    w, branches = job
    with threadpool_limits(1):
        r = oracle.naive_gradient(*_oracle_args(w), branches=list(branches))
    return r["logL"]


def cpu_baseline(w, budget_s=10.0):
    """The CPU oracle timed on the host cores, on bounded samples.

    Run before the GPU is touched (its all-core leg forks worker processes).
    value: the naive O(N^2) oracle gradient (the parity reference): one
    pruning pass per branch on a sample of branches, scaled to all 2N - 2.
    others: the naive gradient on all cores (a branch sample split over
    worker processes), the paper's O(N) post/pre-order gradient on one core
    and on all cores (patterns split over worker processes), the pruning logL alone on
    one core, and central finite differences (two logL per branch, the
    paper's "Numeric" gradient of Section 5.1) on a sample of branches,
    scaled to all branches.  BLAS threads are held to one per process."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    import oracle
    host = f"{cpu_model()}, os.cpu_count()={os.cpu_count()}"
    B = len(w.t)
    args = _oracle_args(w)
    rng = np.random.default_rng(0)
    out = {}
    with threadpool_limits(1):
        t0 = time.perf_counter()
        oracle.log_likelihood(*args)
        t_logL = time.perf_counter() - t0
        n_naive = int(max(2, min(B, budget_s / max(t_logL, 1e-3))))
        sample = sorted(rng.choice(B, size=n_naive, replace=False).tolist())
        t0 = time.perf_counter()
        oracle.naive_gradient(*args, branches=sample)
        t_naive = time.perf_counter() - t0
        per_eval = t_logL + (t_naive - t_logL) / n_naive * B
        t0 = time.perf_counter()
        oracle.linear_gradient(*args)
        t_lin1 = time.perf_counter() - t0
        n_fd = int(max(1, min(B, 0.5 * budget_s / max(2 * t_logL, 1e-3))))
        fd_sample = sorted(rng.choice(B, size=n_fd, replace=False).tolist())
        h = 1e-6
        t0 = time.perf_counter()
        oracle.central_fd_gradient(*args, h=h, branches=fd_sample)
        t_fd = time.perf_counter() - t0
    cores = cpu_cores()
    chunks = [c for c in np.array_split(np.arange(w.n_patterns), cores) if len(c)]
    ctx = mp.get_context("fork")
    with ctx.Pool(len(chunks)) as pool:
        pool.map(_linear_chunk, [(w, chunks[0][:16])] * len(chunks))  # start the workers
        t0 = time.perf_counter()
        pool.map(_linear_chunk, [(w, c) for c in chunks])
        t_linN = time.perf_counter() - t0
        # naive, all cores: n_per branches per worker, each worker's share
        # costing about a quarter of the budget
        n_per = int(max(2, 0.25 * budget_s / max(t_logL, 1e-3)))
        nv_sample = rng.choice(B, size=min(B, n_per * len(chunks)), replace=False)
        nv_chunks = [c for c in np.array_split(np.sort(nv_sample), len(chunks)) if len(c)]
        t0 = time.perf_counter()
        pool.map(_naive_chunk, [(w, c) for c in nv_chunks])
        t_nvN = time.perf_counter() - t0
    # every worker also runs one unperturbed pruning pass (the logL) besides its branches
    per_eval_N = t_nvN / max(len(c) + 1 for c in nv_chunks) * (B / len(nv_chunks) + 1)
    others = [
        {"kind": "oracle_naive_O(N^2)", "value": 1.0 / per_eval_N, "unit": "evals/s", "cores": len(nv_chunks),
         "sample": f"naive gradient on {len(nv_sample)} of {B} branches split over {len(nv_chunks)} processes "
                   f"({t_nvN:.1f} s), scaled to all branches ({per_eval_N:.0f} s)"},
        {"kind": "oracle_linear_O(N)", "value": round(1.0 / t_lin1, 4), "unit": "evals/s", "cores": 1,
         "sample": f"one full evaluation ({t_lin1:.1f} s)"},
        {"kind": "oracle_linear_O(N)", "value": round(1.0 / t_linN, 4), "unit": "evals/s",
         "cores": len(chunks),
         "sample": f"one full evaluation, {w.n_patterns} patterns split over {len(chunks)} processes "
                   f"({t_linN:.2f} s)"},
        {"kind": "oracle_pruning_logL", "value": round(1.0 / t_logL, 4), "unit": "logL evals/s", "cores": 1,
         "sample": f"one post-order logL ({t_logL:.2f} s)"},
        {"kind": "central_fd_gradient", "value": 1.0 / (t_fd / n_fd * B), "unit": "evals/s", "cores": 1,
         "sample": f"central differences h={h:g} on {n_fd} of {B} branches ({t_fd:.1f} s), "
                   f"scaled to all branches ({t_fd / n_fd * B:.0f} s)"},
    ]
    out = {"value": 1.0 / per_eval, "unit": "evals/s", "cores": 1, "kind": "oracle",
           "sample": f"naive O(N^2) oracle gradient (one pruning pass per branch) on {n_naive} of {B} "
                     f"branches ({t_naive:.1f} s), scaled to one full evaluation ({per_eval:.0f} s)",
           "host": host, "others": others}
    return out


def calibrate_copy():
    """Copy 1 GiB device to device three times and print the copy rate.

    Under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE this gives the counters'
    reading for a known 1 GiB read and 1 GiB write per copy."""
    import torch
    x = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for _ in range(3):
        ev[0].record()
        y.copy_(x)
        ev[1].record()
        torch.cuda.synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    best = min(times)
    print(json.dumps({"copy_bytes": 2 * 2 ** 30, "best_ms": best,
                      "GB_per_s": 2 * 2 ** 30 / (best * 1e-3) / 1e9}), flush=True)


def hbm_reference():
    """Achievable HBM rates on this GPU beside the 8 TB/s specification:
    a 1 GiB device-to-device copy (1 GiB read + 1 GiB written) and a 2 GiB
    write (fill), best of five each, timed with HIP events on the current
    stream."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def best(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            ev[0].record()
            fn()
            ev[1].record()
            torch.cuda.synchronize()
            t.append(ev[0].elapsed_time(ev[1]))
        return min(t) * 1e-3

    x = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    copy = 2 * 2 ** 30 / best(lambda: y.copy_(x)) / 1e9
    del x, y
    z = torch.ones(2 ** 29, dtype=torch.float32, device="cuda")
    write = 2 ** 31 / best(lambda: z.fill_(2.0)) / 1e9
    del z
    torch.cuda.empty_cache()
    return {"copy_GBps": round(copy, 1), "write_GBps": round(write, 1)}


def traffic_record(kernel, precision, workload="C2"):
    """HBM bytes per launch measured with rocprofv3 counters for this kernel
    source (profiles/traffic.json), or None if the source has changed."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_1905_12146_amd", "csrc",
                       "kernels_mfma.hip" if precision == "split" else
                       "kernels_dense.hip" if workload == "C5" else "kernels.hip")
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256", {}).get(os.path.basename(src), rec.get("kernels_hip_sha256")) != digest:
        return None
    entry = rec.get(workload, {}).get(precision, {}).get(kernel)
    return None if entry is None else entry["read_bytes"] + entry["write_bytes"]


def serving_bench(args):
    """Serve a stream of requests (N ~ U{100..2000}, S ~ U{500..5000}, 4-state,
    K = 4, FP32 partials, `calls` dependent gradient calls each) with
    continuous batching and with one request at a time, at arrival rates that
    are multiples of the one-at-a-time capacity.  Prints one JSON line."""
    from paper_1905_12146_amd import binding as B
    from paper_1905_12146_amd.serving import Server, generate_requests, run_stream
    from synth import serving_requests

    specs = serving_requests(args.requests, qps=1.0)
    t0 = time.perf_counter()
    workloads = generate_requests(specs, processes=min(16, os.cpu_count() or 1))
    gen_s = time.perf_counter() - t0
    budget = int(args.budget_gb * (1 << 30))

    def with_rate(qps):
        gaps = [s.arrival_s for s in specs]
        return [type(s)(rid=s.rid, arrival_s=g / qps, n_tips=s.n_tips, n_patterns=s.n_patterns, seed=s.seed)
                for s, g in zip(specs, gaps)]

    # warm-up (kernel loading, allocator) on a few requests
    with Server(0, B.PG_FP32, budget, args.max_sessions) as srv:
        run_stream(srv, with_rate(1e9)[:4], workloads[:4], calls=2)
    # one-at-a-time capacity: all requests queued at t = 0, one admitted at a time
    with Server(0, B.PG_FP32, budget, 1) as srv:
        cap = run_stream(srv, with_rate(1e9), workloads, calls=args.calls)
    capacity = cap["completed"] / cap["wall_s"]

    def serve(qps, slots, budget_bytes):
        with Server(0, B.PG_FP32, budget_bytes, slots) as srv:
            r = run_stream(srv, with_rate(qps), workloads, calls=args.calls)
            st = srv.stats()
        r.pop("results")
        row = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items() if k != "errors"}
        row["errors"] = len(r["errors"])
        row["max_batch"] = st["max_batch"]
        row["peak_gb"] = round(st["peak_bytes"] / 2 ** 30, 2)
        row["peak_held_gb"] = round(st["peak_held"] / 2 ** 30, 2)
        row["max_waiting"] = st["max_waiting"]
        # keeps up: completed requests per second within 10% of the arrival rate
        row["keeps_up"] = bool(r["requests_per_s"] >= 0.9 * qps)
        return row

    # arrival rates rise until the one-at-a-time server falls behind them,
    # then one more
    runs = []
    behind = 0
    for f in [float(x) for x in args.qps_factors.split(",") if x]:
        qps = f * capacity
        row = {"qps_factor": f, "qps": round(qps, 2),
               "batched": serve(qps, args.max_sessions, budget),
               "one_at_a_time": serve(qps, 1, budget)}
        runs.append(row)
        print(json.dumps({"serving_progress": row["qps_factor"],
                          "one_at_a_time_keeps_up": row["one_at_a_time"]["keeps_up"],
                          "batched_keeps_up": row["batched"]["keeps_up"]}), file=sys.stderr, flush=True)
        if not row["one_at_a_time"]["keeps_up"]:
            behind += 1
            if behind >= 2:
                break
    # admission that binds: a budget that holds only a few sessions at once,
    # at the highest arrival rate
    tight_gb = args.tight_budget_gb
    tight = {"budget_gb": tight_gb, "qps": runs[-1]["qps"],
             "batched": serve(runs[-1]["qps"], args.max_sessions, int(tight_gb * (1 << 30)))}
    out = {"metric": "served gradient calls: p50/p99 request latency and throughput",
           "workload": f"{args.requests} requests, N~U{{100..2000}}, S~U{{500..5000}}, 4-state, K=4, FP32, "
                       f"{args.calls} calls each, Poisson arrivals",
           "budget_gb": args.budget_gb, "max_sessions": args.max_sessions,
           "one_at_a_time_capacity_req_per_s": round(capacity, 2),
           "capacity_run": {"wall_s": round(cap["wall_s"], 3), "calls_per_s": round(cap["calls_per_s"], 1)},
           "generation_s": round(gen_s, 1), "runs": runs, "tight_budget": tight}
    print(json.dumps(out), flush=True)


def update_bench(args):
    """Partial re-evaluation on the C2 workload: one logL after changing one
    branch length (pg_logL_update: its transition matrices and the post-order
    nodes on its path to the root), against a full logL-only evaluation
    (pg_logL), both through the host entry points; prints one JSON line."""
    from paper_1905_12146_amd import binding as B
    from synth import make_workload

    w = make_workload("C2")
    prec = B.PG_FP64 if (args.precision or "fp64") == "fp64" else B.PG_FP32
    rng = np.random.default_rng(5)
    ctx = B.Context(0, prec)
    ctx.set_workload(w)
    t = w.t.copy()
    for _ in range(5):
        ctx.logL(t)
    n = max(args.steps, 20)
    t0 = time.perf_counter()
    for _ in range(n):
        ctx.logL(t)
    full_us = (time.perf_counter() - t0) / n * 1e6
    ctx.logL_update([0], [t[0]])  # switches on exponent storage (one full pass)
    picks = rng.integers(0, len(t), size=n)
    vals = t[picks] * np.exp(rng.normal(0.0, 0.1, size=n))
    t0 = time.perf_counter()
    for b, v in zip(picks, vals):
        ctx.logL_update([int(b)], [float(v)])
    upd_us = (time.perf_counter() - t0) / n * 1e6
    ctx.close()
    print(json.dumps({"metric": "single-branch logL update vs full logL (host entry points)",
                      "workload": "C2: Yule N=1000, 4-state, K=4, S=2000", "precision": "fp64" if prec == B.PG_FP64 else "fp32",
                      "full_logL_us": round(full_us, 1), "update_logL_us": round(upd_us, 1),
                      "speedup": round(full_us / upd_us, 2), "calls": n}), flush=True)


def hmc_bench(args):
    """Vanilla HMC against HMC with the adaptive Hessian-informed diagonal
    mass matrix (Section 3.2.1) on a random-effects clock (log rate of every
    branch, t_b = exp(theta_b) tau_b, theta_b ~ N(0, 0.5^2)), with the
    gradient and the Hessian diagonal from the GPU.  Each sampler tunes its
    step size for about 70% acceptance in a warm-up, then runs the same
    number of iterations; ESS per second (min and median over the branches)
    is reported for both.  Prints one JSON line."""
    from paper_1905_12146_amd import binding as B
    from paper_1905_12146_amd.inference import RandomEffectsClock, adaptive_hmc, ess, hmc
    from synth import make_workload

    w = make_workload("C5", n_states=4, n_tips=args.hmc_tips, n_patterns=1000)
    ctx = B.Context(0, B.PG_FP64)
    ctx.set_workload(w)
    model = RandomEffectsClock(ctx, w.tau.copy(), sigma=0.5)
    d = len(w.t)
    n_leap, n_warm, n_iter = 10, args.hmc_warmup, args.hmc_iters

    def run(kind, seed):
        x, step = np.zeros(d), 0.02
        state = {"mass": np.ones(d), "h_sum": np.zeros(d), "n": 0}
        # warm-up in blocks of 10 iterations: adjust the step towards 70%
        # acceptance (pHMC also adapts its mass matrix meanwhile)
        t0 = time.perf_counter()
        for blk in range(n_warm // 10):
            if kind == "vhmc":
                r = hmc(model, x, 10, step, n_leap, seed=seed + blk)
            else:
                r = adaptive_hmc(model, model.neg_hess_diag, x, 10, step, n_leap, k=10, seed=seed + blk,
                                 init=(state["h_sum"], state["n"]))
                state["h_sum"], state["n"] = r.h_sum, r.n_updates
            x = r.samples[-1]
            step *= float(np.exp(0.5 * (r.accept_rate - 0.7)))
        t_warm = time.perf_counter() - t0
        t0 = time.perf_counter()
        if kind == "vhmc":
            r = hmc(model, x, n_iter, step, n_leap, seed=seed + 999)
        else:
            r = adaptive_hmc(model, model.neg_hess_diag, x, n_iter, step, n_leap, k=10, seed=seed + 999,
                             init=(state["h_sum"], state["n"]))
        el = time.perf_counter() - t0
        e = np.array([ess(r.samples[:, i]) for i in range(d)])
        return {"step": round(step, 5), "accept": round(r.accept_rate, 3), "seconds": round(el, 2),
                "warmup_seconds": round(t_warm, 2), "ess_min": round(float(e.min()), 1),
                "ess_median": round(float(np.median(e)), 1), "ess_per_s_min": round(float(e.min()) / el, 2),
                "ess_per_s_median": round(float(np.median(e)) / el, 2)}

    v = run("vhmc", 100)
    ph = run("phmc", 200)
    ctx.close()
    print(json.dumps({"metric": "ESS/s of HMC on a random-effects clock: vanilla vs adaptive preconditioned",
                      "workload": f"Yule N={w.n_tips}, 4-state, K=4, S=1000 simulated, {d} branch rates, "
                                  f"{n_leap} leapfrog steps, {n_iter} iterations after {n_warm} warm-up",
                      "vhmc": v, "phmc": ph,
                      "speedup_min": round(ph["ess_per_s_min"] / max(v["ess_per_s_min"], 1e-12), 2),
                      "speedup_median": round(ph["ess_per_s_median"] / max(v["ess_per_s_median"], 1e-12), 2)}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp64", "fp32", "split"], default=None,
                    help="fp64 / fp32 (default fp64 for C2), split = split-BF16 matrix cores (C4)")
    ap.add_argument("--workload", choices=["C2", "C4", "C5"], default="C2",
                    help="C2: N=1000 4-state (headline); C4: N=256 61-state codon, split-BF16; "
                         "C5: N=500 20-state, 3000 patterns")
    ap.add_argument("--timing-steps", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="CPU work per sampled oracle leg (0 disables the CPU baseline)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB device buffer 3 times (HBM counter calibration)")
    ap.add_argument("--serving", action="store_true",
                    help="serving benchmark: a Poisson stream of gradient sessions (continuous batching "
                         "vs one request at a time)")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--calls", type=int, default=10)
    ap.add_argument("--qps-factors", default="0.5,1,1.5,2,3,4,6,8,12",
                    help="arrival rates as multiples of the one-at-a-time capacity (the sweep "
                         "stops after the one-at-a-time server has fallen behind twice)")
    ap.add_argument("--tight-budget-gb", type=float, default=2.0,
                    help="HBM budget of the extra run in which admission binds")
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--max-sessions", type=int, default=64)
    ap.add_argument("--hmc", action="store_true",
                    help="ESS/s of vanilla vs adaptive preconditioned HMC on a random-effects clock")
    ap.add_argument("--hmc-tips", type=int, default=150)
    ap.add_argument("--hmc-iters", type=int, default=1500)
    ap.add_argument("--hmc-warmup", type=int, default=300)
    ap.add_argument("--updates", action="store_true",
                    help="partial re-evaluation: single-branch logL updates against full logL (C2)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.serving:
        serving_bench(args)
        return
    if args.updates:
        update_bench(args)
        return
    if args.hmc:
        hmc_bench(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the pattern-sharded multi-GPU layout is a design, not built)", file=sys.stderr)
        sys.exit(2)

    from synth import make_workload

    if args.precision is None:
        args.precision = "split" if args.workload == "C4" else "fp64"
    w = make_workload(args.workload)
    # the CPU legs run first: the all-core leg forks, which must happen
    # before this process touches the GPU
    cpu = cpu_baseline(w, args.cpu_seconds) if args.cpu_seconds > 0 else None

    import torch

    from paper_1905_12146_amd import binding as B

    N, S, m, K = w.n_tips, w.n_patterns, w.n_states, w.n_cats
    prec = {"fp64": B.PG_FP64, "fp32": B.PG_FP32, "split": B.PG_SPLIT_BF16}[args.precision]
    es = 8 if prec == B.PG_FP64 else 4

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    ctx = B.Context(0, prec)
    ctx.set_workload(w)
    ctx.set_stream(stream.cuda_stream)
    d_t = torch.tensor(w.t, device=dev, dtype=torch.float64)
    d_l = torch.zeros(1, device=dev, dtype=torch.float64)
    d_g = torch.zeros(len(w.t), device=dev, dtype=torch.float64)

    def step():
        ctx.logL_and_grad_device(d_t.data_ptr(), d_l.data_ptr(), d_g.data_ptr())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if ctx.status() != B.PG_OK:
        raise RuntimeError("evaluation failed: " + B.pg_last_error(ctx.handle))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed

    # per-evaluation durations: a HIP event pair around each evaluation on
    # the context's stream (torch's current stream here)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    ev_us = np.array([e0.elapsed_time(e1) * 1e3 for e0, e1 in evs])
    eval_us = {"median": round(float(np.median(ev_us)), 2), "p5": round(float(np.percentile(ev_us, 5)), 2),
               "p95": round(float(np.percentile(ev_us, 95)), 2), "n": len(ev_us)}

    # per-kernel durations: HIP events recorded by the library on the
    # context's stream, one pair per kernel launch
    ctx.set_timing(True)
    for _ in range(args.timing_steps):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(False)
    times = ctx.timing()
    avg_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in times.items()}
    sb = algorithmic_bytes(N, S, m, K, es)
    ob = onchip_bytes(N, S, m, K, es)
    dom = max(("post", "pre"), key=lambda k: avg_ms[k])

    def rate(nbytes, ms):
        return nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0

    achieved = rate(sb[dom], avg_ms[dom])
    med_ms = eval_us["median"] * 1e-3
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_record(dom, args.precision, args.workload),
                "byte_model": "5 I'V + 2 N S + 2 |P| per evaluation; post 2 I'V + N S + |P|, "
                              "pre 3 I'V + N S + |P|",
                "bytes_per_launch": sb[dom], "avg_us": round(avg_ms[dom] * 1e3, 2),
                "kernels_avg_us": {k: round(v * 1e3, 2) for k, v in avg_ms.items()},
                "kernels_frac": {k: round(rate(sb[k], avg_ms[k]) / HBM_PEAK_GBS, 4) for k in ("post", "pre")},
                "eval_bytes": sb["eval"],
                "eval_frac": round(rate(sb["eval"], med_ms) / HBM_PEAK_GBS, 4),
                "onchip_model": {"what": "lower bound with children's messages and q kept on chip",
                                 "bytes_per_launch": {k: ob[k] for k in ("post", "pre")},
                                 "frac": round(rate(ob[dom], avg_ms[dom]) / HBM_PEAK_GBS, 4),
                                 "eval_bytes": ob["eval"],
                                 "eval_frac": round(rate(ob["eval"], med_ms) / HBM_PEAK_GBS, 4)}}
    # what plain copies, reads and writes achieve on this GPU, beside the
    # dominant kernel's counter-measured bytes over its measured time
    ref = hbm_reference()
    if roofline["traffic"]:
        ref["kernel_traffic_GBps"] = round(rate(roofline["traffic"], avg_ms[dom]), 1)
    roofline["measured_hbm"] = ref

    if prec == B.PG_SPLIT_BF16:
        # executed BF16 matrix-core work of the dominant kernel: 16x16x32
        # MFMAs (16384 flops each) per tile of 16 patterns of one category;
        # a product with a 64 x 64 matrix is 6 part products x 8 MFMAs: per
        # internal non-root node one (post: F p); per child in the pre-order
        # one for Q m plus one for F^T u if the child is internal
        n_tiles = K * ((S + 15) // 16)
        n_int = N - 2
        mf = {"post": 48 * n_int, "pre": 48 * (2 * N - 2) + 48 * n_int}
        fl = mf[dom] * n_tiles * 16384
        tf = fl / (avg_ms[dom] * 1e-3) / 1e12 if avg_ms[dom] > 0 else 0.0
        roofline["mfma"] = {"kernel": dom, "bf16_flops_per_launch": fl, "achieved": round(tf, 2),
                            "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tf / 2500.0, 4)}

    if m == 20 and prec != B.PG_SPLIT_BF16:
        # executed matrix-core work of the dense-state kernels: 16x16x4 MFMAs
        # (2048 flops each, FP64 or FP32) per tile; a 20 x 20 product is 2
        # row blocks x 5 k-steps = 10 MFMAs (62.5% of the issued work is the
        # 20 x 20 product itself); post: one per internal non-root node (P p),
        # pre: one per child (Q m) plus one per internal child (P^T u)
        n_tiles = K * ((S + 15) // 16)
        n_int = N - 2
        mf = {"post": 10 * n_int, "pre": 10 * (2 * N - 2) + 10 * n_int}
        peak = 78.6 if prec == B.PG_FP64 else 157.3
        fl = mf[dom] * n_tiles * 2048
        tf = fl / (avg_ms[dom] * 1e-3) / 1e12 if avg_ms[dom] > 0 else 0.0
        roofline["mfma"] = {"kernel": dom, "flops_per_launch": fl, "achieved": round(tf, 2),
                            "peak": peak, "unit": "TFLOP/s", "frac": round(tf / peak, 4)}

    out = {"metric": METRIC, "value": round(value, 2), "unit": "evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {B.PG_FP64: "f64", B.PG_FP32: "f32", B.PG_SPLIT_BF16: "bf16x3-f32acc"}[prec],
           "data": "synthetic (seeded Yule tree, random non-reversible "
                   + ("codon " if m == 61 else "") + "Q, simulated sites)",
           "config": {"workload": f"Yule N={N}, {m}-state non-reversible CTMC, K={K} gamma(0.5) "
                                  f"categories, S={S} simulated patterns, rescaling on, "
                                  f"{len(w.t)} branch gradients",
                      "n_tips": N, "n_patterns": S, "n_states": m, "n_cats": K,
                      "precision": args.precision},
           "eval_time_us": eval_us,
           "roofline": roofline}
    ctx.close()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
