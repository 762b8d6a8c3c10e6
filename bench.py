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
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "neutron histories/sec on 1 MI355X, FP32-mixed & batched vs FP64 plain, at tally match"

# Minimal VALU lane-instruction counts of the algorithm's steps in FP32 (see the
# roofline section of the design notes): per random draw (a Philox4x32-10 block
# of 2 x 4 32-bit multiplies, 2 three-way xors and 2 key adds per round,
# amortised over its two draws, plus the conversion), per transport step
# (ray-cylinder and ray-sphere intersection, log, reciprocal, move, exp and the
# weight product), per scattering (sqrt, sin/cos, frame, rotation, family
# search) and per history (source, cross sections, tally angle and binning).
OPS_PER_DRAW = 43
OPS_PER_STEP = 96
OPS_PER_SCATTER = 48
OPS_PER_HISTORY = 60
# VALU issue peak: 256 CUs x 64 lanes x 2.4 GHz, one lane-instruction per lane per clock
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# HBM bytes per launch of the dominant kernels from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (scaled by a 256 MiB copy: fetch x2.000, write x1.000), valid
# only for the kernel build they were taken on (hash of transport.hip, device.h and
# the compiler flags);
# profiles/k_mixed_biased_sample_1e7.txt holds the summary.  Nearly all of it is
# the 32-byte memory-side writes of FP64 tally atomics.
MEASURED_TRAFFIC = {"source_hash": "8be0601b45afebbb",
                    "k_mixed<float>": 0.459e6 + 354.922e6, "k_plain": 0.492e6 + 669.999e6}


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


def algorithmic_ops(stats: dict) -> float:
    return (OPS_PER_DRAW * stats["draws"] + OPS_PER_STEP * stats["steps"] + OPS_PER_SCATTER * stats["scatters"]
            + OPS_PER_HISTORY * stats["histories"])


def cpu_baseline(prob, seconds: float) -> dict:
    from oracle import oracle as O
    threads = min(os.cpu_count() or 1, 64)
    t0 = time.perf_counter()
    O.run(prob, first=0, n=20_000, threads=1)
    rate1 = 20_000 / max(time.perf_counter() - t0, 1e-6)
    n = int(min(max(rate1 * threads * seconds, 1e5), 5e8))
    t0 = time.perf_counter()
    O.run(prob, first=0, n=n, threads=threads)
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": n / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} histories of the same workload (FP64 oracle, {threads} threads, {dt:.1f} s)",
            "single_thread_value": rate1, "single_thread_sample": "first 20000 histories, 1 thread",
            "cpu_model": cpu, "nproc": os.cpu_count()}


def time_policy(torch, sim, n, precision, steps, warmup):
    for _ in range(warmup):
        sim.run(first=0, n=n, precision=precision)
    torch.cuda.synchronize()
    sim.ctx.reset_stats()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for k in range(steps):
        sim.run(first=(k + 1) * n, n=n, precision=precision)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    stats = sim.ctx.read_stats()
    return ms, stats


def time_one_by_one(torch, ctx, br, precision, shift, steps, tunings=None):
    """The batch's simulations launched one after another with pr_run_histories
    (history ids shifted by `shift`, then by the batch's span each step)."""
    def one_pass(sh):
        for k, (s, o) in enumerate(zip(br.sims, br.offsets)):
            if tunings is not None:
                ctx.set_tuning(**tunings[k])
            s.run(first=o + sh, n=s.prob.n_histories, precision=precision)
    one_pass(shift)   # warm-up
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for k in range(steps):
        one_pass(shift + (k + 1) * br.span)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--histories", type=int, default=10_000_000)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp32", "fp64", "both"], default="both")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--paper-guide", action="store_true",
                    help="also time the paper's guide benchmark (1e8 neutrons; same kernel as the headline)")
    ap.add_argument("--autotune", action="store_true", help="re-measure the launch tuning before timing")
    ap.add_argument("--batch-steps", type=int, default=3)
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
                      "histories_per_step": n, "seed": W.RUN_SEED}}
    fp32 = fp64 = None
    if args.autotune:
        out["tuning"] = ctx.autotune([(sim.geom, sim.src, sim.tallies, 1 << 44, n)], sample_fraction=1.0)
    else:
        ctx.set_tuning(**TUNED["sample"])
        out["tuning"] = ctx.get_tuning()
    if args.only in ("fp32", "both"):
        ms, st = time_policy(torch, sim, n, "fp32", args.steps, args.warmup)
        fp32 = (ms, st)
        print(f"[bench] fp32-mixed {ms:.3f} ms/step, {n / ms * 1e3:.4g} histories/s", file=sys.stderr, flush=True)
    fp64p = None
    if args.only in ("fp64", "both"):
        ms64, st64 = time_policy(torch, sim, n, "fp64", args.fp64_steps, 1)
        fp64 = (ms64, st64)
        print(f"[bench] fp64-plain {ms64:.3f} ms/step, {n / ms64 * 1e3:.4g} histories/s", file=sys.stderr, flush=True)
        # the same FP64 histories (identical records) on persistent lanes with LDS tallies,
        # with that policy's stored tuning
        if not args.autotune:
            ctx.set_tuning(**TUNED_FP64_PERSISTENT["sample"])
        fp64p_tuning = ctx.get_tuning()
        ms64p, _ = time_policy(torch, sim, n, "fp64_persistent", args.fp64_steps, 1)
        fp64p = ms64p
        ctx.set_tuning(**out["tuning"])
        print(f"[bench] fp64-persistent {ms64p:.3f} ms/step, {n / ms64p * 1e3:.4g} histories/s", file=sys.stderr,
              flush=True)

    head_ms, head_st = fp32 if fp32 else fp64
    out["value"] = n / head_ms * 1e3
    out["ms_per_step"] = head_ms
    out["dtype"] = "f32" if fp32 else "f64"
    per_launch_ops = algorithmic_ops(head_st) / max(1, head_st["histories"]) * n
    achieved = per_launch_ops / (head_ms * 1e-3) / 1e12
    kname = "k_mixed<float>" if fp32 else "k_plain"
    traffic = MEASURED_TRAFFIC[kname] if kernel_source_hash() == MEASURED_TRAFFIC["source_hash"] else None
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                       "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic, "traffic_unit": "bytes per launch",
                       "kernel": kname, "ops_per_history": per_launch_ops / n}
    if fp32 and fp64:
        out["fp64_plain"] = {"value": n / fp64[0] * 1e3, "ms_per_step": fp64[0]}
        out["speedup_vs_fp64_plain"] = fp64[0] / fp32[0]
        out["fp64_persistent"] = {"value": n / fp64p * 1e3, "ms_per_step": fp64p, "tuning": fp64p_tuning,
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
        graph.replay()   # warm-up step
        torch.cuda.synchronize()
        ctx.reset_stats()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        h0 = time.perf_counter()
        t0.record()
        for _ in range(args.batch_steps):
            graph.replay()
        t1.record()
        h_graph = (time.perf_counter() - h0) * 1e3 / args.batch_steps
        torch.cuda.synchronize()
        bms = t0.elapsed_time(t1) / args.batch_steps
        bst = ctx.read_stats()
        ctx.release_batch(pid)
        out["batched"] = {"value": batch.total_histories / bms * 1e3, "unit": "histories/s", "ms_per_step": bms,
                          "histories_per_step": batch.total_histories, "simulations": len(batch.problems),
                          "steps_per_history": bst["steps"] / max(1, bst["histories"]), "tuning": tuned,
                          "roofline": {"bound": "alu", "unit": "TOP/s", "peak": VALU_PEAK_TOPS,
                                       "achieved": algorithmic_ops(bst) / (args.batch_steps * bms * 1e-3) / 1e12,
                                       "frac": algorithmic_ops(bst) / (args.batch_steps * bms * 1e-3) / 1e12
                                       / VALU_PEAK_TOPS, "kernel": "k_batch"},
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
    if args.paper_guide:
        # the paper's m = 1 guide benchmark at its own size (1e8 neutrons), for context
        # with the paper's only timing (about 140 s on a laptop)
        pg = W.paper_guide()
        ctx.set_tuning(**TUNED["paper_guide"])
        gsim = B.Simulation(ctx, pg)
        gms, _ = time_policy(torch, gsim, pg.n_histories, "fp32", 2, 1)
        out["paper_guide"] = {"histories": pg.n_histories, "ms": gms, "histories_per_s": pg.n_histories / gms * 1e3,
                              "paper_laptop_s": 140.0, "note": "the paper's timing is on other hardware: context only"}
        print(f"[bench] paper guide 1e8: {gms:.3f} ms", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host cores", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
