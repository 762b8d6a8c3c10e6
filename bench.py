"""Benchmark: neutron histories per second on one MI355X.

Workload (the headline metric's configuration): the biased powder-sample
problem, 1e7 histories per step: monochromatic 1.8 A pencil beam on a solid
cylinder (r=5 mm, h=20 mm, axis y) of a synthetic fcc powder (a=4.0 A, 26
reflection families, sigma_inc=5 b, sigma_abs=2 b at 1.798 A), scattering
cross section biased by 4 with the probability-conserving weight correction;
tallies: 2theta(1800) x lambda(100) of scattered escapes, transmitted counter,
absorbed counter.  One step = one pr_run_histories call over 1e7 histories
(source, flights, collisions, scoring all inside the timed kernel) with the
inputs already resident on the GPU.

The FP32-mixed policy is the headline value; the FP64-plain policy and the
persistent FP64 policy (the same FP64 histories, bit for bit) are timed beside
it.  The oracle is timed on the host's cores on a bounded sample.  The
mixed policy runs with the launch tuning stored per workload (measured with
pr_autotune on MI355X); --autotune measures it afresh before timing.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "neutron histories/sec on 1 MI355X, FP32-mixed & batched vs FP64 plain, at tally match"

# Algorithmic VALU lane-operations per event of the FP32 history loop, with their
# derivation (printed in the JSON line): the operations the algorithm itself
# needs, as FP32/integer lane instructions, not the instructions the kernel
# happens to execute (divergence, refill and bookkeeping excluded).
OPS_MODEL = {
    "draw": (43, "Philox4x32-10 block: 10 rounds x (2 32x32->64-bit multiply-adds + 2 three-input xors "
                 "+ 2 key adds) = 80 ops per 2 uniforms, + 3 for the conversion to a uniform"),
    "step": (96, "ray-cylinder (24) and ray-sphere (18) slab/quadratic intersection, flight -ln(u)/Sigma_g "
                 "(log 8, reciprocal 2, 2), move and time (8), weight exp((Sigma_g - Sigma) x) (8) and FP64 product "
                 "(4), boundary/collision decision and region update (22)"),
    "scatter": (48, "process choice (4), 1/g weight factor (2), Bragg family search (12) or isotropic mu (2), "
                    "sqrt (2), sin/cos (6), frame e1, e2 (12), rotation (8)"),
    "history": (60, "source position and direction (10), cross sections at lambda: edge search and C(lambda) "
                    "(16), 2theta = acos(u.b) (12), two bin indices (10), end-of-history bookkeeping (12)"),
}
# VALU issue peak: 256 CUs x 64 lanes x 2.4 GHz, one lane-instruction per lane per clock
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernels from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (scaled by a 256 MiB copy: fetch x2.000, write x1.000), valid
# only for the kernel build they were taken on (hash of transport.hip, device.h and
# the compiler flags); the profiles/ summaries hold them.
MEASURED_TRAFFIC = {
    "source_hash": "345ad6539fa884ad",
    # profiles/k_mixed_biased_sample_1e7.txt, k_mixed_vessel_1e8.txt, k_mixed_guide_1e8_4e8bins.txt
    "k_mixed<float>:sample": 1.84289e7,
    "k_mixed<float>:vessel": 1.854e9,
    "k_mixed<float>:guide": 2.75813e9,
}


def kernel_source_hash() -> str:
    """Hash of the kernel sources and the compiler flags they are built with."""
    import hashlib
    from paper_2304_06226_amd.build import HIPCC_FLAGS
    h = hashlib.sha256()
    for f in ("paper_2304_06226_amd/csrc/transport.hip", "paper_2304_06226_amd/csrc/device.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    if kernel_source_hash() != MEASURED_TRAFFIC.get("source_hash"):
        return None
    return MEASURED_TRAFFIC.get(kernel)


def algorithmic_ops(stats: dict) -> float:
    return (OPS_MODEL["draw"][0] * stats["draws"] + OPS_MODEL["step"][0] * stats["steps"]
            + OPS_MODEL["scatter"][0] * stats["scatters"] + OPS_MODEL["history"][0] * stats["histories"])


def alu_roofline(stats: dict, n: int, ms: float, kernel: str, workload: str) -> dict:
    """The ALU roofline of one launch of `kernel` on `workload` (the key of its
    measured traffic)."""
    per_launch = algorithmic_ops(stats) / max(1, stats["histories"]) * n
    achieved = per_launch / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(kernel + ":" + workload),
            "traffic_unit": "bytes per launch", "kernel": kernel, "ops_per_history": per_launch / n}


def cpu_info() -> dict:
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if info:
                        break
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("vendor_id", "model name", "cpu family", "model", "stepping", "cpu MHz", "cache size") \
                        and k not in info:
                    info[k] = v
    except OSError:
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    info["nproc"] = os.cpu_count()
    return info


def cpu_baseline(prob, seconds: float, runs: int = 3) -> dict:
    """The oracle on the host's cores: a bounded sample of the workload (about
    `seconds` per run), timed `runs` times; the median rate is the value."""
    from oracle import oracle as O
    info = cpu_info()
    threads = min(info.get("affinity_cpus") or os.cpu_count() or 1, 64)
    t0 = time.perf_counter()
    O.run(prob, first=0, n=20_000, threads=1)
    rate1 = 20_000 / max(time.perf_counter() - t0, 1e-6)
    n = int(min(max(rate1 * threads * seconds, 1e5), 5e8))
    rates = []
    for _ in range(runs):
        t0 = time.perf_counter()
        O.run(prob, first=0, n=n, threads=threads)
        rates.append(n / (time.perf_counter() - t0))
    return {"value": statistics.median(rates), "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} histories of the same workload (FP64 oracle, {threads} threads), median of {runs} "
                      f"runs of about {seconds:.0f} s",
            "runs": rates, "single_thread_value": rate1, "single_thread_sample": "first 20000 histories, 1 thread",
            "cpu": info}


def time_steps(torch, step, steps: int, warmup: int, after_warmup=None):
    """`warmup` untimed steps, then `steps` steps, each between two HIP events on
    the current stream (the stream the library launches on), with the device
    synchronised before and after; returns (median ms, mean ms, per-step ms)."""
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    if after_warmup is not None:
        after_warmup()
        torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record()
        step(warmup + k)
        ev[k][1].record()
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in ev]
    return statistics.median(ms), statistics.mean(ms), ms


def time_policy(torch, sim, n, precision, steps, warmup):
    """Median-of-steps timing of one policy over fresh history ranges, and the run
    statistics of the timed steps."""
    med, mean, ms = time_steps(torch, lambda k: sim.run(first=(k + 1) * n, n=n, precision=precision), steps, warmup,
                               after_warmup=sim.ctx.reset_stats)
    return med, mean, sim.ctx.read_stats()


def time_one_by_one(torch, ctx, br, precision, shift, steps, tunings=None):
    """The batch's simulations launched one after another with pr_run_histories
    (history ids shifted by `shift`, then by the batch's span each step); median ms per pass."""
    def one_pass(k):
        for j, (s, o) in enumerate(zip(br.sims, br.offsets)):
            if tunings is not None:
                ctx.set_tuning(**tunings[j])
            s.run(first=o + shift + k * br.span, n=s.prob.n_histories, precision=precision)
    med, _, _ = time_steps(torch, one_pass, steps, 1)
    return med


def config_leg(torch, B, ctx, prob, tuning, steps, fp64_steps, plain_steps, kernel, hbm_bytes_per_score=None):
    """One more workload at its full size: FP32 mixed (median of `steps`), FP64
    persistent and FP64 plain (medians), with its own rooflines."""
    from paper_2304_06226_amd.tuning import TUNED, TUNED_FP64_PERSISTENT
    n = prob.n_histories
    sim = B.Simulation(ctx, prob)
    ctx.set_tuning(**TUNED[tuning])
    med, mean, st = time_policy(torch, sim, n, "fp32", steps, 1)
    leg = {"histories_per_step": n, "value": n / med * 1e3, "unit": "histories/s", "ms_per_step": med,
           "mean_ms_per_step": mean, "steps": steps, "tuning": ctx.get_tuning(),
           "steps_per_history": st["steps"] / max(1, st["histories"]),
           "roofline": alu_roofline(st, n, med, kernel, tuning)}
    if hbm_bytes_per_score is not None:
        # tally traffic: one (sum w, sum w^2) pair per scored history into a tally far
        # larger than the caches, the bytes the algorithm must move at least
        scored = st["escaped"] + st["detected"] + st["absorbed"]
        per_launch = hbm_bytes_per_score * scored / max(1, st["histories"]) * n
        achieved = per_launch / (med * 1e-3) / 1e9
        leg["roofline_hbm"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kernel + ":" + tuning),
                               "algorithmic_bytes_per_launch": per_launch,
                               "note": f"{hbm_bytes_per_score} B (sum w, sum w^2) per scored history"}
    print(f"[bench] {prob.name} fp32 {med:.3f} ms/step, {n / med * 1e3:.4g} histories/s", file=sys.stderr, flush=True)
    if tuning in TUNED_FP64_PERSISTENT:
        ctx.set_tuning(**TUNED_FP64_PERSISTENT[tuning])
    med_p, _, _ = time_policy(torch, sim, n, "fp64_persistent", fp64_steps, 1)
    leg["fp64_persistent"] = {"value": n / med_p * 1e3, "ms_per_step": med_p, "steps": fp64_steps}
    med64, _, _ = time_policy(torch, sim, n, "fp64", plain_steps, 1)
    leg["fp64_plain"] = {"value": n / med64 * 1e3, "ms_per_step": med64, "steps": plain_steps}
    leg["speedup_vs_fp64_plain"] = med64 / med
    leg["speedup_vs_fp64_persistent"] = med_p / med
    print(f"[bench] {prob.name} fp64-persistent {med_p:.3f} ms, fp64-plain {med64:.3f} ms", file=sys.stderr, flush=True)
    return leg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--histories", type=int, default=10_000_000)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=5.0)
    ap.add_argument("--cpu-runs", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp32", "fp64", "both"], default="both")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the vessel (1e8) and guide (1e8, 4e8-bin tally) legs")
    ap.add_argument("--config-steps", type=int, default=5)
    ap.add_argument("--paper-guide", action="store_true",
                    help="also time the paper's guide benchmark (1e8 neutrons; same kernel as the headline)")
    ap.add_argument("--autotune", action="store_true", help="re-measure the launch tuning before timing")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--one-by-one-steps", type=int, default=1,
                    help="steps of the batch's simulations launched one by one (FP64 plain, FP32 mixed, "
                         "FP64 persistent); 0 skips")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the history range would be "
              "sharded across GPUs with a final tally sum, which this program does not do.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_06226_amd import binding as B
    from paper_2304_06226_amd import workloads as W
    from paper_2304_06226_amd.tuning import TUNED, TUNED_FP64_PERSISTENT

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n = args.histories
    prob = W.biased_sample(n=n)
    ctx = B.Context(device=0, seed=W.RUN_SEED)
    sim = B.Simulation(ctx, prob)

    out = {"metric": METRIC, "unit": "histories/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic",
           "config": {"workload": "biased powder cylinder (scatter bias 4), 1.8 A pencil beam, "
                                  "2theta(1800) x lambda(100) + transmitted + absorbed tallies",
                      "histories_per_step": n, "seed": W.RUN_SEED},
           "timing": "HIP events around each step on the launch stream; ms_per_step is the median over the timed "
                     "steps, mean_ms_per_step their mean"}
    fp32 = fp64 = None
    if args.autotune:
        out["tuning"] = ctx.autotune([(sim.geom, sim.src, sim.tallies, 1 << 44, n)], sample_fraction=1.0)
    else:
        ctx.set_tuning(**TUNED["sample"])
        out["tuning"] = ctx.get_tuning()
    if args.only in ("fp32", "both"):
        med, mean, st = time_policy(torch, sim, n, "fp32", args.steps, args.warmup)
        fp32 = (med, mean, st)
        print(f"[bench] fp32-mixed {med:.3f} ms/step (median), {n / med * 1e3:.4g} histories/s", file=sys.stderr,
              flush=True)
    fp64p = None
    if args.only in ("fp64", "both"):
        med64, mean64, st64 = time_policy(torch, sim, n, "fp64", args.fp64_steps, 1)
        fp64 = (med64, mean64, st64)
        print(f"[bench] fp64-plain {med64:.3f} ms/step, {n / med64 * 1e3:.4g} histories/s", file=sys.stderr, flush=True)
        # the same FP64 histories (identical records) on persistent lanes with LDS tallies,
        # with that policy's stored tuning
        if not args.autotune:
            ctx.set_tuning(**TUNED_FP64_PERSISTENT["sample"])
        fp64p_tuning = ctx.get_tuning()
        med64p, _, _ = time_policy(torch, sim, n, "fp64_persistent", args.fp64_steps, 1)
        fp64p = med64p
        ctx.set_tuning(**out["tuning"])
        print(f"[bench] fp64-persistent {med64p:.3f} ms/step, {n / med64p * 1e3:.4g} histories/s", file=sys.stderr,
              flush=True)

    head_ms, head_mean, head_st = fp32 if fp32 else fp64
    out["value"] = n / head_ms * 1e3
    out["ms_per_step"] = head_ms
    out["mean_ms_per_step"] = head_mean
    out["dtype"] = "f32" if fp32 else "f64"
    out["roofline"] = alu_roofline(head_st, n, head_ms, "k_mixed<float>" if fp32 else "k_plain", "sample")
    out["ops_model"] = {k: {"ops": v[0], "derivation": v[1]} for k, v in OPS_MODEL.items()}
    if fp32 and fp64:
        out["fp64_plain"] = {"value": n / fp64[0] * 1e3, "ms_per_step": fp64[0], "steps": args.fp64_steps}
        out["speedup_vs_fp64_plain"] = fp64[0] / fp32[0]
        out["fp64_persistent"] = {"value": n / fp64p * 1e3, "ms_per_step": fp64p, "steps": args.fp64_steps,
                                  "tuning": fp64p_tuning,
                                  "note": "the plain kernel's FP64 step on persistent lanes with LDS tallies; "
                                          "records identical to FP64 plain"}
        out["speedup_vs_fp64_persistent"] = fp64p / fp32[0]
    out["events_per_history"] = {"steps": head_st["steps"] / head_st["histories"],
                                 "draws": head_st["draws"] / head_st["histories"],
                                 "scatters": head_st["scatters"] / head_st["histories"]}
    if not args.no_batch:
        # the batched workload: 256 uneven powder simulations + the 1000-box imaging setup,
        # prepared once and stepped by replaying a HIP graph of one prepared run
        batch = W.sample_batch()
        br = B.BatchRun(ctx, batch, base=1 << 40)
        if args.autotune:
            tuned = ctx.autotune(br.descriptors(shift=8 * br.span), sample_fraction=1.0)
        else:
            ctx.set_tuning(**TUNED["batch"])
            tuned = ctx.get_tuning()
        # host cost of one unprepared call, for comparison
        br.run()
        torch.cuda.synchronize()
        h0 = time.perf_counter()
        br.run(shift=br.span)
        h_run_batch = (time.perf_counter() - h0) * 1e3
        torch.cuda.synchronize()
        pid = ctx.prepare_batch(br.descriptors(shift=2 * br.span), stride=br.span)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            ctx.run_prepared(pid)
        h0 = time.perf_counter()
        bms, bmean, _ = time_steps(torch, lambda k: graph.replay(), args.batch_steps, 1, after_warmup=ctx.reset_stats)
        h_graph = (time.perf_counter() - h0) * 1e3 / (args.batch_steps + 1)
        bst = ctx.read_stats()
        ctx.release_batch(pid)
        ops = algorithmic_ops(bst) / args.batch_steps
        out["batched"] = {"value": batch.total_histories / bms * 1e3, "unit": "histories/s", "ms_per_step": bms,
                          "mean_ms_per_step": bmean, "steps": args.batch_steps,
                          "histories_per_step": batch.total_histories, "simulations": len(batch.problems),
                          "steps_per_history": bst["steps"] / max(1, bst["histories"]), "tuning": tuned,
                          "roofline": {"bound": "alu", "unit": "TOP/s", "peak": VALU_PEAK_TOPS,
                                       "achieved": ops / (bms * 1e-3) / 1e12,
                                       "frac": ops / (bms * 1e-3) / 1e12 / VALU_PEAK_TOPS, "kernel": "k_batch"},
                          "step": "HIP graph replay of a prepared batch run",
                          "host_ms_per_step": {"graph_replay": h_graph, "pr_run_batch": h_run_batch},
                          "workload": "256 powder simulations (r 1-20 mm, a 3.5-6 A, lambda 1-5 A, bias 1/2/4/8, "
                                      "1e4-1e6 histories each, odd ones in a vessel) + 1000-box imaging, 1e7 histories"}
        print(f"[bench] batched {bms:.3f} ms/step, {batch.total_histories / bms * 1e3:.4g} histories/s",
              file=sys.stderr, flush=True)
        if args.one_by_one_steps > 0:
            # the same simulations, one launch each: FP64 plain (the batch's precision
            # baseline), FP32 mixed with each workload's stored tuning (the gain of batching)
            # and persistent FP64 with its own stored tunings
            shift = 4 * br.span
            ms64 = time_one_by_one(torch, ctx, br, "fp64", shift, args.one_by_one_steps)
            shift += (args.one_by_one_steps + 1) * br.span
            # each launch gets its workload's stored tuning, with the claim size scaled
            # down for small simulations so that every wave of the grid gets work
            tunings = [TUNED["imaging"] if p.name.startswith("imaging") else
                       dict(TUNED["sample"], chunk=int(min(TUNED["sample"]["chunk"], max(64, p.n_histories // 8192))))
                       for p in batch.problems]
            ms32 = time_one_by_one(torch, ctx, br, "fp32", shift, args.one_by_one_steps, tunings)
            shift += (args.one_by_one_steps + 1) * br.span
            tunings64 = [TUNED_FP64_PERSISTENT["imaging"] if p.name.startswith("imaging") else
                         dict(TUNED_FP64_PERSISTENT["sample"],
                              chunk=int(min(TUNED_FP64_PERSISTENT["sample"]["chunk"], max(64, p.n_histories // 8192))))
                         for p in batch.problems]
            ms64p = time_one_by_one(torch, ctx, br, "fp64_persistent", shift, args.one_by_one_steps, tunings64)
            out["batched"]["one_by_one"] = {
                "fp64_plain": {"value": batch.total_histories / ms64 * 1e3, "ms_per_step": ms64},
                "fp64_persistent": {"value": batch.total_histories / ms64p * 1e3, "ms_per_step": ms64p},
                "fp32_mixed": {"value": batch.total_histories / ms32 * 1e3, "ms_per_step": ms32},
                "launches_per_step": len(batch.problems)}
            out["batched"]["speedup_vs_fp64_plain"] = ms64 / bms
            out["batched"]["speedup_vs_fp64_persistent"] = ms64p / bms
            print(f"[bench] one by one: fp64-plain {ms64:.3f} ms, fp64-persistent {ms64p:.3f} ms, "
                  f"fp32-mixed {ms32:.3f} ms per step", file=sys.stderr, flush=True)
    if not args.no_configs:
        # the powder diffractometer with its vessel (1e8, 2theta(3600) x lambda(1000)) and the
        # m = 3 guide (1e8, 4e8-bin exit tally), at their full sizes
        out["configs"] = {
            "vessel": dict(config_leg(torch, B, ctx, W.vessel_sample(), "vessel", args.config_steps, 3, 2,
                                      "k_mixed<float>"),
                           workload="sample (bias 2) in an Al-like vessel shell, 300 K Maxwellian 0.5-5 A over "
                                    "10x10 mm, 2theta(3600) x lambda(1000), 1e8 histories"),
            "guide": dict(config_leg(torch, B, ctx, W.m3_guide(), "guide", args.config_steps, 3, 3, "k_mixed<float>",
                                     hbm_bytes_per_score=16),
                          workload="10 m m=3 straight guide, +-1 deg divergent source, lambda 1-10 A, exit "
                                   "x,y(200x200) x div_x,div_y(100x100) = 4e8 bins (6.4 GB), 1e8 histories"),
        }
    if args.paper_guide:
        # the paper's m = 1 guide benchmark at its own size (1e8 neutrons), for context
        # with the paper's only timing (about 140 s on a laptop)
        pg = W.paper_guide()
        ctx.set_tuning(**TUNED["paper_guide"])
        gsim = B.Simulation(ctx, pg)
        gms, _, _ = time_policy(torch, gsim, pg.n_histories, "fp32", 3, 1)
        out["paper_guide"] = {"histories": pg.n_histories, "ms": gms, "histories_per_s": pg.n_histories / gms * 1e3,
                              "paper_laptop_s": 140.0, "note": "the paper's timing is on other hardware: context only"}
        print(f"[bench] paper guide 1e8: {gms:.3f} ms", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host cores", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds, args.cpu_runs)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
