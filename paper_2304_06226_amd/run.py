"""Run a named workload through the GPU library and print one JSON line of timings.

    python -m paper_2304_06226_amd.run --workload guide --histories 1e8 --precision fp32 --repeat 3

Workloads: sample (biased powder sample), vessel, guide, imaging, paper_guide
(the paper's m = 1 guide benchmark, 1e8 neutrons), batch
(the 256-simulation + imaging batch; always FP32-mixed).  The mixed policy uses
the workload's stored launch tuning (--autotune re-measures it).  One warm-up
run, then `repeat` timed runs on disjoint history ranges (HIP events on the
current stream).  Useful under rocprofv3 to profile one workload's kernels.
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["sample", "vessel", "guide", "imaging", "paper_guide", "paper_chopper",
                                           "batch"],
                    default="sample")
    ap.add_argument("--histories", type=float, default=None)
    ap.add_argument("--precision", choices=["fp32", "fp64", "fp64_persistent"], default="fp32")
    ap.add_argument("--repeat", type=int, default=3)
    ap.add_argument("--autotune", action="store_true")
    args = ap.parse_args(argv)

    import torch
    from . import binding as B
    from . import workloads as W
    from .tuning import TUNED, TUNED_FP64_PERSISTENT

    torch.cuda.set_device(0)
    ctx = B.Context(0, seed=W.RUN_SEED)
    stored = TUNED_FP64_PERSISTENT if args.precision == "fp64_persistent" else TUNED
    if args.workload in stored:
        ctx.set_tuning(**stored[args.workload])
    if args.workload == "batch":
        batch = W.sample_batch()
        br = B.BatchRun(ctx, batch)
        n = batch.total_histories
        if args.autotune:
            ctx.autotune(br.descriptors(), sample_fraction=1.0)

        def go(k):
            br.run(shift=k * br.span)
    else:
        prob = {"sample": W.biased_sample, "vessel": W.vessel_sample, "guide": W.m3_guide, "imaging": W.imaging_problem,
                "paper_guide": W.paper_guide, "paper_chopper": W.paper_chopper}[args.workload]()
        n = int(args.histories) if args.histories else prob.n_histories
        sim = B.Simulation(ctx, prob)
        if args.autotune and args.precision == "fp32":
            ctx.autotune([(sim.geom, sim.src, sim.tallies, 1 << 44, n)], sample_fraction=1.0)

        def go(k):
            sim.run(first=k * n, n=n, precision=args.precision)
    go(0)
    torch.cuda.synchronize()
    ctx.reset_stats()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for k in range(args.repeat):
        go(k + 1)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.repeat
    st = ctx.read_stats()
    out = {"workload": args.workload, "precision": args.precision if args.workload != "batch" else "fp32",
           "histories": n, "ms": ms, "histories_per_s": n / ms * 1e3,
           "steps_per_history": st["steps"] / max(1, st["histories"]), "tuning": ctx.get_tuning()}
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    sys.exit(main())
