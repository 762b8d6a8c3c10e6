"""Launch tunings of the PR_FP32_MIXED policy measured on one MI355X with
pr_autotune (coordinate descent over the pr_tuning knobs, HIP-event timed), per
named workload.  Results do not depend on them beyond floating-point summation
order; Context.autotune re-measures them.  Workloads whose large tallies are hit
at random bins (guide, vessel, imaging) run without the LDS bin cache: it would
rarely hit and every score would pay its probes.  The sample and batch entries
were re-measured at full size: the autotuner's reduced samples shift where the
last claims of a launch fall, which is what decides the best chunk there.
waves_per_simd 5 (kernels held to 96 VGPRs) is faster for the vessel, the
paper's guide and the batch's powder simulations, slower for the others.  In
the batch the imaging class (a daughter grid) claims 128 histories at a time
and the powder class 512 (-2 % against 256 for both).  Blocks of 1024 lanes
(16 waves sharing one LDS tally) take 0.5 % off the sample and 1.3 % off the
guide.  Grid walks paused after 3 cells (grid_walk_cells) take the imaging
scene from 8.65 to 6.55 ms per 1e7 histories and the batch from 18.3 to 16.4 ms
per step: a wave no longer waits for its lanes' longest walk.  Runs whose
tallies score straight into global memory (guide, vessel, paper's guide) score
as a wave with paired-lane atomics; for the guide that moved the best refill
threshold from 16 to 48 idle lanes (7.56 -> 6.22 ms per 1e8 histories).  Cheaper
tally binning moved the biased sample's from 32 to 16 (512-id claims: 1.237 ->
1.221 ms); taking a newborn history's first vacuum step in the refill pass moved
it to 28 (1.086 -> 1.000 ms; 24 to 32 are within 0.5 %); starting a pencil
beam's newborns from the first newborn's state after its first step made refills
cheaper and 1024-id claims best (fewer claim atomics; 24 idle lanes, 0.907 ms)."""

# workload name -> pr_tuning fields
TUNED = {
    "sample": {"block": 1024, "blocks_per_cu": 0, "refill_threshold": 24, "lds_tally_bytes": 32768,
               "bin_cache_slots": 256, "chunk": 1024, "waves_per_simd": 4,
               "grid_chunk": 0, "grid_walk_cells": 0, "vacuum_steps": 1},
    "guide": {"block": 1024, "blocks_per_cu": 0, "refill_threshold": 48, "lds_tally_bytes": 32768,
              "bin_cache_slots": 0, "chunk": 1024, "waves_per_simd": 4,
              "grid_chunk": 0, "grid_walk_cells": 0, "vacuum_steps": 1},
    "vessel": {"block": 256, "blocks_per_cu": 0, "refill_threshold": 48, "lds_tally_bytes": 32768,
               "bin_cache_slots": 0, "chunk": 256, "waves_per_simd": 5,
               "grid_chunk": 0, "grid_walk_cells": 0, "vacuum_steps": 1},
    "imaging": {"block": 256, "blocks_per_cu": 0, "refill_threshold": 16, "lds_tally_bytes": 32768,
                "bin_cache_slots": 0, "chunk": 128, "waves_per_simd": 4,
                "grid_chunk": 0, "grid_walk_cells": 3, "vacuum_steps": 1},
    "paper_guide": {"block": 256, "blocks_per_cu": 0, "refill_threshold": 48, "lds_tally_bytes": 32768,
                    "bin_cache_slots": 0, "chunk": 1024, "waves_per_simd": 5,
                    "grid_chunk": 0, "grid_walk_cells": 0, "vacuum_steps": 1},
    "batch": {"block": 256, "blocks_per_cu": 0, "refill_threshold": 16, "lds_tally_bytes": 32768,
              "bin_cache_slots": 256, "chunk": 512, "waves_per_simd": 5,
              "grid_chunk": 128, "grid_walk_cells": 3, "vacuum_steps": 1},
    "paper_chopper": {"block": 256, "blocks_per_cu": 0, "refill_threshold": 24, "lds_tally_bytes": 32768,
                      "bin_cache_slots": 1024, "chunk": 1024, "waves_per_simd": 4, "grid_chunk": 0,
                      "grid_walk_cells": 0, "vacuum_steps": 1},
}

# Launch tunings of the PR_FP64_PERSISTENT policy (the same knobs; waves_per_simd
# does not apply to it), measured at each workload's full size by coordinate
# descent over refill threshold, chunk, blocks per CU, block size and bin-cache
# slots, starting from the FP32 entries.  Its lanes run longer steps, so more of
# them may wait before a refill (guide: 16 -> 48 idle lanes, -17 %).
TUNED_FP64_PERSISTENT = {
    "sample": dict(TUNED["sample"], block=256, chunk=256, refill_threshold=32),
    "guide": dict(TUNED["guide"], block=256, refill_threshold=48),
    "vessel": dict(TUNED["vessel"], chunk=1024),
    "imaging": dict(TUNED["imaging"], chunk=64, grid_walk_cells=0),
    "paper_guide": dict(TUNED["paper_guide"], refill_threshold=32),
    "paper_chopper": {"block": 256, "blocks_per_cu": 0, "refill_threshold": 48, "lds_tally_bytes": 32768,
                      "bin_cache_slots": 256, "chunk": 256, "waves_per_simd": 4,
                      "grid_chunk": 0, "grid_walk_cells": 0, "vacuum_steps": 1},
}
