"""Benchmark of the PLUGIN bandwidth selector's hot path on one MI355X.

One step = one complete bandwidth selection (Algorithm 1, Steps I-VII: the
moment reduction, the Step IV and Step VI pair sums over all n(n-1)/2 pairs
each, and the scalar stages) for one sample already resident in HBM, through
the C ABI (kde_plugin_bandwidth_ex on a device pointer).  The default
workload is the large single-dataset configuration: n = 2^20 draws
x = 1e3 exp(Z) - 5e2, Z ~ N(0, 1), seed 2 (heavy right tail, large offset),
FP32 pair arithmetic with compensated sums (FP64 plain is timed beside it).

value      = pair evaluations per second, n(n-1) per selection (the diagonal is
             added analytically and not counted)
roofline   = the persistent kernel's algorithmic FP32 FLOP rate (10 FLOP per
             pair at r = 6, 8 at r = 4; FMA = 2, exp2 = 1) against the FP32
             vector peak of 157.3 TFLOP/s; its duration comes from HIP events
             recorded by the library on the launch stream around every launch
cpu_baseline = the FP64 oracle (plain C + OpenMP, all host cores) on the same
             sample: one full selection up to n = 2^17, else both pair stages
             over the first 16384 rows against all later columns (at the
             oracle's g1 and g2 from its stored record), the fraction stated
rel_err_vs_oracle = against the oracle's stored record of the same sample
             (tests/golden/full_size_records.json, matched by SHA-256), or a
             full oracle run for small samples

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|fp32x|fp32poly|q32|fp64]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3      # MI355X datasheet, packed FP32 vector
FP32_NONPACKED_PEAK_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
FP64_VECTOR_PEAK_TFLOPS = 78.6       # MI355X datasheet, FP64 vector
FLOP_PER_PAIR = {6: 10, 4: 8}
EVAL_FLOP_PER_PAIR = 4            # density evaluation: sub, square, exp2, add

WORKLOADS = {
    "normal1024": dict(desc="single dataset n=1024, N(0,1), seed 0", n=1024, kind="normal", seed=0),
    "bimodal65536": dict(desc="single dataset n=65536, 0.5N(-1,(2/3)^2)+0.5N(1,(2/3)^2), seed 1",
                         n=65536, kind="bimodal", seed=1),
    "lognormal1m": dict(desc="single dataset n=2^20, 1e3*exp(Z)-5e2, Z~N(0,1), seed 2",
                        n=1 << 20, kind="lognormal", seed=2),
}


# Samples up to this size get one full oracle selection as the CPU baseline;
# larger ones a bounded part of it (both pair stages over the first rows).
FULL_ORACLE_MAX_N = 1 << 17
CPU_BASELINE_ROWS = 16384
GOLDEN_FULL = os.path.join(ROOT, "tests", "golden", "full_size_records.json")


def stored_oracle_record(workload, x):
    """The FP64 oracle's Algorithm 1 record for this workload's sample, as
    written by tests/golden/make_full_size.py (oracle only), if present and
    made from the same bytes."""
    if not os.path.exists(GOLDEN_FULL):
        return None
    with open(GOLDEN_FULL) as f:
        recs = json.load(f)
    rec = recs.get(workload)
    if not rec:
        return None
    from paper_1505_02100_amd import synth
    if rec["sha256"] != synth.sha256(x):
        return None
    return {k: float.fromhex(v) for k, v in rec["plugin"].items()}


def stored_batch_records(xs):
    """The FP64 oracle's records of the 512-sample batch (tests/golden), in
    sample order, if present and made from the same bytes; else None."""
    if not os.path.exists(GOLDEN_FULL):
        return None
    with open(GOLDEN_FULL) as f:
        rec = json.load(f).get("batch512")
    from paper_1505_02100_amd import synth
    if not rec or len(rec["samples"]) != len(xs):
        return None
    out = []
    for r, x in zip(rec["samples"], xs):
        if r["sha256"] != synth.sha256(x):
            return None
        out.append({k: float.fromhex(v) for k, v in r["plugin"].items()})
    return out


def run_env():
    """The versions and devices a line was measured with."""
    import platform
    import torch
    prop = torch.cuda.get_device_properties(0)
    from paper_1505_02100_amd import kdeplugin as kp
    return {"device": prop.name, "gcn_arch": getattr(prop, "gcnArchName", None),
            "compute_units": prop.multi_processor_count, "library": kp.kde_version(),
            "torch": torch.__version__, "hip": torch.version.hip, "python": platform.python_version(),
            "host_cpus": os.cpu_count()}


def synth_sha256(x):
    from paper_1505_02100_amd import synth
    return synth.sha256(x)


def make_sample(w):
    from paper_1505_02100_amd import synth
    if w["kind"] == "normal":
        return synth.workload_single_normal(w["n"], w["seed"])
    if w["kind"] == "bimodal":
        return synth.workload_single_bimodal(w["n"], w["seed"])
    return synth.workload_single_lognormal(w["n"], w["seed"])


# The persistent kernel and the host code that builds its work list: a change
# to any of them can change the traffic the counters measured.
KERNEL_SOURCES = ("kde_device.hip", "kde_internal.h", "kde_exp2_poly.h", "kde_runtime.h", "kde_host.cpp")


def kernel_source_sha256():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1505_02100_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, precision):
    """HBM bytes per launch of the persistent kernel from the committed
    rocprofv3 counter summary, or None if absent or taken on other code."""
    p = os.path.join(ROOT, "profiles", f"traffic_k_persistent_{workload}_{precision}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    return t.get("hbm_bytes_per_launch")


def calib_copy(steps):
    """A plain device copy of known size, for scaling FETCH_SIZE/WRITE_SIZE."""
    import torch
    nbytes = 256 << 20
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(steps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read": nbytes, "calib_copy_bytes_written": nbytes,
                      "launches": steps}))


def bench_batch(args):
    """512 samples, n log-uniform in [256, 65536], normal / bimodal / t3 mixed:
    one call = one persistent launch over all of them (graph replay), against
    512 sequential single-sample calls (FP64 plain and the measured precision)."""
    import numpy as np
    import tempfile
    import torch
    from paper_1505_02100_amd import kdeplugin as kp
    from paper_1505_02100_amd import synth
    prec = {"fp32": kp.KDE_FP32_COMP, "fp32x": kp.KDE_FP32_COMP_EXACT, "fp32poly": kp.KDE_FP32_POLYEXP,
            "q32": kp.KDE_Q32_32, "fp64": kp.KDE_FP64_PLAIN}
    xs, names = synth.workload_batch(512, 3)
    xds = [torch.from_numpy(x).cuda() for x in xs]
    pairs = sum(x.size * (x.size - 1) for x in xs)
    torch.cuda.synchronize()
    table = args.tune_table
    tuned = None
    if not table:
        table = os.path.join(tempfile.gettempdir(), f"kde_tune_{args.precision}.json")
        t0 = time.perf_counter()
        tuned = kp.kde_autotune(prec[args.precision], [x.size for x in xs], table,
                                mode=kp.KDE_TUNE_BATCH, reps=3)
        tuned["seconds"] = round(time.perf_counter() - t0, 2)
    ctx = kp.Context(prec[args.precision], tune_table=table)
    ctx.plugin_bandwidth_batch(xds)
    torch.cuda.synchronize()
    dev = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.plugin_bandwidth_batch(xds)
        dev.append(ctx.last_device_ms())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = (t1 - t0) / args.steps
    dev_ms = float(np.mean(dev))
    flop = sum(FLOP_PER_PAIR.values()) * sum(x.size * (x.size - 1) // 2 for x in xs)
    achieved = flop / (dev_ms * 1e-3) / 1e12

    def sequential(p, tt=None):
        c = kp.Context(p, tune_table=tt) if tt else kp.Context(p)
        for xd in xds[:4]:
            c.plugin_bandwidth(xd)
        torch.cuda.synchronize()
        a = time.perf_counter()
        hs = [c.plugin_bandwidth(xd).h for xd in xds]
        torch.cuda.synchronize()
        b = time.perf_counter()
        c.close()
        return b - a, hs

    recs = stored_batch_records(xs)
    err = None
    if recs:
        err = {k: max(abs(getattr(r, k) - q[k]) / abs(q[k]) for r, q in zip(res, recs)) for k in ("h", "psi6", "psi4")}
        err["source"] = "stored FP64 oracle records of all 512 samples (tests/golden/full_size_records.json)"
    seq64_s, h64 = sequential(kp.KDE_FP64_PLAIN)
    seq_s, hseq = sequential(prec[args.precision], table)
    worst64 = max(abs(r.h - h) / h for r, h in zip(res, h64))
    same = all(r.h == h for r, h in zip(res, hseq))
    out = {"metric": "pair-evals/s & %FP32 VALU peak; selections/s, p50/p99 latency vs FP64 plain",
           "value": pairs / per, "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 1, "ms_per_step": round(per * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
           "config": {"workload": "batch of 512 samples, n log-uniform in [256, 65536], N(0,1) / bimodal / t3 "
                                  "with equal probability, one persistent launch per batch (graph replay)",
                      "samples": len(xs), "sum_n": int(sum(x.size for x in xs)),
                      "pairs_per_batch": int(pairs), "precision": args.precision,
                      "tile": ctx.config(), "launch": ctx.last_launch(), "tune_table": tuned},
           "selections_per_s": round(len(xs) / per, 1),
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                        "traffic": None, "kernel": "kde::k_persistent", "kernel_ms_avg": round(dev_ms, 4)},
           "sequential_fp64_plain": {"seconds": round(seq64_s, 4),
                                     "selections_per_s": round(len(xs) / seq64_s, 1),
                                     "speedup_of_batch": round(seq64_s / per, 2),
                                     "max_rel_diff_h": worst64},
           "max_rel_err_vs_oracle": err,
           "sequential_same_precision": {"seconds": round(seq_s, 4),
                                         "selections_per_s": round(len(xs) / seq_s, 1),
                                         "speedup_of_batch": round(seq_s / per, 2),
                                         "bitwise_equal_h": same}}
    ctx.close()
    print(json.dumps(out))


def bench_eval(args):
    """Density evaluation (equation (1)) with the selected bandwidth.
    eval4096: the n = 2^20 lognormal workload sample on a grid of 4096
    points spanning its 0.1% to 99.9% quantiles (evenly spaced runs).
    eval-samples: the n = 2^18 lognormal sample at its own samples, in the
    order drawn (unsorted, so the per-point path with FP64 differences).
    One step = one evaluation of all m points (n m pair evaluations), sample
    and points resident in HBM."""
    import numpy as np
    import torch
    from paper_1505_02100_amd import kdeplugin as kp
    from paper_1505_02100_amd import synth
    prec = {"fp32": kp.KDE_FP32_COMP, "fp32x": kp.KDE_FP32_COMP_EXACT, "fp32poly": kp.KDE_FP32_POLYEXP,
            "q32": kp.KDE_Q32_32, "fp64": kp.KDE_FP64_PLAIN}
    at_samples = args.workload == "eval-samples"
    x = synth.workload_single_lognormal(1 << 18 if at_samples else 1 << 20, 2)
    n = x.size
    m = n if at_samples else 4096
    xd = torch.from_numpy(x).cuda()
    ctx = kp.Context(prec[args.precision])
    h = ctx.plugin_bandwidth(xd).h
    y = x.copy() if at_samples else np.linspace(np.quantile(x, 0.001), np.quantile(x, 0.999), m)
    yd = torch.from_numpy(y).cuda()
    for _ in range(max(1, args.warmup)):
        ctx.eval(xd, yd, h)
    torch.cuda.synchronize()
    dev = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f = ctx.eval(xd, yd, h)
        dev.append(ctx.last_device_ms())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = (t1 - t0) / args.steps
    dev_ms = float(np.mean(dev))
    pairs = n * m
    achieved = EVAL_FLOP_PER_PAIR * pairs / (dev_ms * 1e-3) / 1e12
    out = {"metric": "pair-evals/s & %FP32 VALU peak; selections/s, p50/p99 latency vs FP64 plain",
           "value": pairs / per, "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(per * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
           "config": {"workload": ("density evaluation f(x_k; h) at the n=2^18 lognormal sample's own "
                                   "points, unsorted (1e3*exp(Z)-5e2, seed 2), with its selected h" if at_samples else
                                   "density evaluation f(y; h) on a 4096-point grid for the n=2^20 "
                                   "lognormal sample (1e3*exp(Z)-5e2, seed 2) with its selected h"),
                      "n": n, "m": m, "h": h, "precision": args.precision},
           "device_ms": {q: round(float(np.percentile(dev, p)), 4) for q, p in (("p10", 10), ("p50", 50), ("p90", 90))},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                        "kernel": ("kde::eval::k_eval64" if args.precision == "fp64" else "kde::eval::k_eval32") + " + k_eval_reduce",
                        "kernel_ms_avg": round(dev_ms, 4),
                        "flop_per_launch": EVAL_FLOP_PER_PAIR * pairs}}
    if not args.no_cpu_baseline:
        import oracle
        k = 64
        pick = np.linspace(0, m - 1, k).astype(int)
        a = time.perf_counter()
        ref = oracle.kde_eval(x, h, y[pick])
        b = time.perf_counter()
        got = f.cpu().numpy()[pick]
        out["cpu_baseline"] = {"value": n * k / (b - a), "unit": "pair-evals/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"{k} of the {m} points against all n samples ({b - a:.2f} s)"}
        out["max_rel_err_vs_oracle"] = float(np.max(np.abs(got - ref) / ref))
    ctx.close()
    print(json.dumps(out))


def bench_serve(args):
    """Poisson arrivals (rate args.rate per s for args.duration s), n log-uniform
    in [1e3, 4e6], normal / bimodal / t3 mixed, samples drawn in device memory,
    admission capped by an 8 GiB budget; FP32 path.  Reports served throughput,
    selections/s and latency from arrival, then re-runs a sample of completed
    requests alone (bitwise check) and the oracle on the small ones."""
    import numpy as np
    import torch
    from paper_1505_02100_amd import kdeplugin as kp
    from paper_1505_02100_amd import synth
    from paper_1505_02100_amd.server import serve_trace
    prec = {"fp32": kp.KDE_FP32_COMP, "fp32x": kp.KDE_FP32_COMP_EXACT, "fp32poly": kp.KDE_FP32_POLYEXP,
            "q32": kp.KDE_Q32_32, "fp64": kp.KDE_FP64_PLAIN}
    trace = synth.serving_trace(rate=args.rate, duration=args.duration, master=4)
    # items of about 2^pair_budget_log2 pairs for every request size: a step of
    # 2^36 pairs then holds thousands of items from many requests
    ctx = kp.Context(prec[args.precision], pair_budget=1 << args.pair_budget_log2)
    ctx.plugin_bandwidth(synth.normal(4096, 1))
    rep = serve_trace(ctx, trace, duration_s=args.duration, mem_budget=8 << 30, max_active=args.max_active,
                      step_pairs=1 << 36, policy=args.policy, aging_ms=args.aging_ms, fill=args.fill,
                      keep_samples=True,
                      drain=args.drain, log=lambda m: print(m, file=sys.stderr, flush=True))
    done = rep["completions"]
    # alone re-runs of up to 50 completed requests, oracle on those with n <= 2^17
    rng = np.random.default_rng(0)
    pick = rng.choice(len(done), size=min(50, len(done)), replace=False) if done else []
    same, worst, oracle_checked = 0, 0.0, 0
    import oracle
    for k in pick:
        c = done[int(k)]
        x = rep["samples"][c.id]
        a = ctx.plugin_bandwidth(x)
        same += int(a.h == c.h)
        if c.n <= (1 << 17):
            ref = oracle.plugin(x.cpu().numpy())
            worst = max(worst, abs(c.h - ref.h) / ref.h)
            oracle_checked += 1
    ns = np.array([c.n for c in done]) if done else np.zeros(0)
    out = {"metric": "pair-evals/s & %FP32 VALU peak; selections/s, p50/p99 latency vs FP64 plain",
           "value": rep["completed_pair_evals_per_s"], "unit": "pair-evals/s", "n_gpus": 1,
           "steps": len(done), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
           "config": {"workload": f"serving: Poisson arrivals {args.rate}/s for {args.duration}s, n log-uniform "
                                  "in [1e3, 4e6], N(0,1)/bimodal/t3, samples resident on device, admission "
                                  "capped at 8 GiB", "policy": args.policy, "aging_ms": args.aging_ms, "fill": args.fill,
                      "pair_budget_log2": args.pair_budget_log2,
                      "max_active": args.max_active, "precision": args.precision, "drain": args.drain},
           "value_is": "pair evaluations of completed requests per second of the run",
           "selections_per_s": round(rep["selections_per_s"], 3),
           "latency_ms_all_arrivals": rep["latency_ms_all_arrivals"],
           "latency_ms_completed_only": rep["latency_ms"],
           "window_s": round(rep["window_s"], 2),
           "arrived": rep["arrived"], "completed": len(done), "unfinished": rep["unfinished"],
           "failed": rep["failed"], "failed_steps": rep["failed_steps"], "by_size": rep["by_size"],
           "completed_n_median": float(np.median(ns)) if len(ns) else None,
           "offered_pair_evals_per_s": rep["offered_pair_evals_per_s"],
           "completed_pair_evals_per_s": rep["completed_pair_evals_per_s"],
           "issued_pair_evals_per_s": rep["device_pair_evals_per_s"],
           "issued_over_offered": rep["device_pair_evals_per_s"] / max(rep["offered_pair_evals_per_s"], 1),
           "backlog_at_end": rep["backlog"],
           "alone_vs_mix": {"checked": len(pick), "bitwise_equal": same},
           "oracle": {"checked": oracle_checked, "max_rel_err_h": worst}}
    print(json.dumps(out))


def bench_issue_rate(args):
    """Issue rates of the pair stages' instructions (paper_1505_02100_amd/probes/
    issue_rate, built by build()): FP32 fma/mul/sub, v_exp_f32, and the Step IV
    and Step VI per-pair sequences in register-only loops at 2, 3, 4 and 8 waves
    per SIMD, with the shader clock measured under that load.  The pair
    sequences' rates are the ceiling of the pair kernels' instruction mix."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1505_02100_amd", "probes", "issue_rate")
    if not os.path.exists(exe):
        raise SystemExit(f"{exe} is not built: run __graft_entry__.build()")
    r = subprocess.run([exe], capture_output=True, text=True, check=True)
    probe = json.loads(r.stdout)
    res = probe["results"]
    best = {}
    for row in res:
        if row["op"] not in best or row["lane_steps_per_s"] > best[row["op"]]["lane_steps_per_s"]:
            best[row["op"]] = row
    pair = (best["pair_r6"]["lane_steps_per_s"] + best["pair_r4"]["lane_steps_per_s"]) / 2
    tflops = sum(FLOP_PER_PAIR.values()) / 2 * pair / 1e12
    out = {"metric": "issue rates of the pair-stage instruction mix (microbenchmark)",
           "value": pair, "unit": "pair-evals/s", "n_gpus": 1, "steps": 5, "warmup": 1,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "register-only loops of the Step IV / Step VI per-pair sequences and of "
                                  "single FP32 instructions, 8 independent chains per lane"},
           "pair_mix_ceiling": {"pair_evals_per_s": pair, "tflops_algorithmic": round(tflops, 2),
                                "frac_of_157_3": round(tflops / FP32_VECTOR_PEAK_TFLOPS, 4)},
           "best_by_op": {k: {q: v[q] for q in ("waves_per_simd", "lane_insts_per_s", "insts_per_cu_cycle",
                                                "sclk_mhz")} for k, v in best.items()},
           "probe": probe}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["fp32", "fp32x", "fp32poly", "q32", "fp64"], default="fp32")
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["batch512", "serve", "eval4096", "eval-samples",
                                                               "issue-rate"],
                    default="lognormal1m")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: arrival window in seconds")
    ap.add_argument("--policy", choices=["fcfs", "sjf"], default="sjf", help="serve: admission order")
    ap.add_argument("--max-active", type=int, default=256, help="serve: requests on the device at once")
    ap.add_argument("--aging-ms", type=int, default=10000,
                    help="serve, sjf: a queued request's key drops by one (a halving of its pair count) per "
                         "this many ms of waiting; 0 = pure smallest first")
    ap.add_argument("--drain", action="store_true", help="serve: run until every arrival has finished")
    ap.add_argument("--pair-budget-log2", type=int, default=22,
                    help="serve: work items of about 2^this many pairs (the step holds 2^36)")
    ap.add_argument("--fill", choices=["share", "priority"], default="priority",
                    help="serve: a step's pair budget round-robin over the active requests, or in key order")
    ap.add_argument("--tune-table", default=None, help="autotune table for the batch workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a 256 MiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); multi-GPU sharding is described in DESIGN.md but not built",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.calib_copy:
        calib_copy(args.steps)
        return

    if args.workload == "batch512":
        bench_batch(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload in ("eval4096", "eval-samples"):
        bench_eval(args)
        return
    if args.workload == "issue-rate":
        bench_issue_rate(args)
        return

    from paper_1505_02100_amd import kdeplugin as kp

    prec_code = {"fp32": kp.KDE_FP32_COMP, "fp32x": kp.KDE_FP32_COMP_EXACT, "fp32poly": kp.KDE_FP32_POLYEXP,
                 "q32": kp.KDE_Q32_32, "fp64": kp.KDE_FP64_PLAIN}[args.precision]
    w = WORKLOADS[args.workload]
    x = make_sample(w)
    n = x.size
    pairs = n * (n - 1)             # pair evaluations per selection (both Psi stages)
    flop = sum(FLOP_PER_PAIR.values()) * (n * (n - 1) // 2)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    torch.cuda.synchronize()

    ctx = kp.Context(prec_code)
    for _ in range(max(1, args.warmup)):
        ctx.plugin_bandwidth(xd)
    torch.cuda.synchronize()
    dev_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.plugin_bandwidth(xd)
        dev_ms.append(ctx.last_device_ms())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = pairs / ((t1 - t0) / args.steps)
    timeline = ctx.last_timeline(0)
    cfg = ctx.config()
    cfg["launch"] = ctx.last_launch()   # blocks and waves per SIMD of the timed kernel
    dev_ms_avg = float(np.mean(dev_ms))

    achieved = flop / (dev_ms_avg * 1e-3) / 1e12
    traffic = measured_traffic(args.workload, args.precision)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": traffic,
                "kernel": "kde::k_persistent", "kernel_ms_avg": round(dev_ms_avg, 4),
                "flop_per_launch": flop,
                "frac_of_nonpacked_fp32": round(achieved / FP32_NONPACKED_PEAK_TFLOPS, 4)}

    out = {"metric": "pair-evals/s & %FP32 VALU peak; selections/s, p50/p99 latency vs FP64 plain",
           "value": value, "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp64": "f64", "q32": "q32.32"}.get(args.precision, "f32"), "data": "synthetic",
           "config": {"workload": w["desc"] + ", Steps I-VII per step, samples resident in HBM",
                      "n": n, "precision": args.precision, "pairs_per_selection": pairs,
                      "tile": cfg},
           "selections_per_s": round(1e3 / ms_per_step, 3),
           "device_ms_per_selection": {q: round(float(np.percentile(dev_ms, p)), 4)
                                       for q, p in (("p10", 10), ("p50", 50), ("p90", 90))},
           "stage_timeline_ms": [round(t, 4) for t in timeline],
           "exp2_per_s_device": pairs / (dev_ms_avg * 1e-3),
           "roofline": roofline,
           "env": run_env(), "dataset_sha256": synth_sha256(x)}

    if not args.no_fp64_compare and args.precision != "fp64":
        ctx64 = kp.Context(kp.KDE_FP64_PLAIN)
        ctx64.plugin_bandwidth(xd)
        k64 = max(3, args.steps // 10)
        torch.cuda.synchronize()
        dev64 = []
        a = time.perf_counter()
        for _ in range(k64):
            r64 = ctx64.plugin_bandwidth(xd)
            dev64.append(ctx64.last_device_ms())
        torch.cuda.synchronize()
        b = time.perf_counter()
        ach64 = flop / (float(np.mean(dev64)) * 1e-3) / 1e12
        out["fp64_plain"] = {"pair_evals_per_s": pairs / ((b - a) / k64),
                             "selections_per_s": round(k64 / (b - a), 3),
                             "ms_per_step": round((b - a) * 1e3 / k64, 4),
                             "kernel_ms_avg": round(float(np.mean(dev64)), 4),
                             "achieved_tflops": round(ach64, 3),
                             "frac_of_fp64_peak": round(ach64 / FP64_VECTOR_PEAK_TFLOPS, 4),
                             "speedup_of_measured_path": round(value / (pairs / ((b - a) / k64)), 3),
                             "rel_diff_h": abs(res.h - r64.h) / r64.h}
        ctx64.close()

    record = stored_oracle_record(args.workload, x)
    if record is not None:
        out["rel_err_vs_oracle"] = {k: abs(getattr(res, k) - v) / abs(v) for k, v in record.items()
                                    if k in ("h", "psi6", "psi4", "g2", "g1", "sigma", "psi8")}
        out["rel_err_vs_oracle"]["source"] = "stored FP64 oracle record (tests/golden/full_size_records.json)"
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.num_threads()
        if n <= FULL_ORACLE_MAX_N:
            a = time.perf_counter()
            ref = oracle.plugin(x)
            b = time.perf_counter()
            out["cpu_baseline"] = {"value": pairs / (b - a), "unit": "pair-evals/s", "cores": threads,
                                   "kind": "oracle",
                                   "sample": f"one full selection of the same n={n} sample "
                                             f"({pairs} pair evaluations, {b - a:.2f} s)"}
            if record is None:
                out["rel_err_vs_oracle"] = {k: abs(getattr(res, k) - getattr(ref, k)) / abs(getattr(ref, k))
                                            for k in ("h", "psi6", "psi4", "g2")}
        elif record is not None:
            # both pair stages of the oracle over the first rows against all
            # later columns, at the oracle's own g1 and g2 from the stored record
            rows = min(n, CPU_BASELINE_ROWS)
            a = time.perf_counter()
            oracle.block_sum(x, 6, record["g1"], 0, rows, 0, n)
            oracle.block_sum(x, 4, record["g2"], 0, rows, 0, n)
            b = time.perf_counter()
            p_part = 2 * (rows * (n - 1) - rows * (rows - 1) // 2)
            out["cpu_baseline"] = {"value": p_part / (b - a), "unit": "pair-evals/s", "cores": threads,
                                   "kind": "oracle",
                                   "sample": f"Step IV and Step VI pair sums of rows 0..{rows - 1} against all "
                                             f"later columns of the same n={n} sample ({p_part} pair evaluations, "
                                             f"{p_part / pairs:.4f} of a selection, {b - a:.2f} s); a full "
                                             f"selection at this rate: {pairs / p_part * (b - a):.0f} s"}
        g1 = ref.g1 if n <= FULL_ORACLE_MAX_N else (record or {}).get("g1")
        if g1:
            # one host core on a bounded part of the same work: the Step IV pair
            # sum of the first rows against all later columns, at the oracle's g1
            rows = max(1, min(n, (1 << 26) // max(1, n)))
            oracle.set_num_threads(1)
            try:
                a = time.perf_counter()
                oracle.block_sum(x, 6, g1, 0, rows, 0, n)
                b = time.perf_counter()
            finally:
                oracle.set_num_threads(threads)
            p1 = rows * (n - 1) - rows * (rows - 1) // 2
            out["cpu_baseline_1core"] = {"value": p1 / (b - a), "unit": "pair-evals/s", "cores": 1,
                                         "kind": "oracle",
                                         "sample": f"Step IV pair sum of rows 0..{rows - 1} against all later "
                                                   f"columns ({p1} pair evaluations, {b - a:.2f} s)"}
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
