"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle on the
same seeded inputs.

FP64 plain policy: element-wise, per history (event-sequence hash, termination,
scattering count, steps, draws, final weight, position, direction) and per
tally bin (equal up to summation order).  FP32 mixed policy: the tally
agreement test (merged-bin z-scores, chi^2 p > 1e-3, |z| > 4 count within the
binomial 99.9% quantile) plus a paired common-random-number comparison.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_06226_amd import binding as B
from paper_2304_06226_amd import workloads as W

from parity import ORACLE_FIRST, compare_records_fp64, compare_tallies_fp64, gpu_run, paired_fp32_fp64, tally_stat_test

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(device=0, seed=4096)
    yield c
    c.close()


def _fp64_case(ctx, prob, first, n, threads=8):
    print(f"[case] {prob.name} fp64 first={first} n={n}", flush=True)
    gres, grec, gst = gpu_run(ctx, prob, first=first, n=n, precision="fp64")
    ores = O.run(prob, first=first, n=n, threads=threads, records=True)
    same = compare_records_fp64(grec, ores.records)
    compare_tallies_fp64(gres, ores, grec, ores.records, same)
    for k in ("histories", "escaped", "absorbed", "killed", "detected", "capped", "outside"):
        assert abs(gst[k] - ores.stats[k]) <= int((~same).sum()), k
    return gres, grec, ores, same


def test_analog_sample_fp64_elementwise(ctx):
    _, grec, ores, same = _fp64_case(ctx, W.analog_sample(), 0, 100_000)
    assert same.mean() >= 0.999


def test_biased_sample_fp64_elementwise_first_1e6(ctx):
    _fp64_case(ctx, W.biased_sample(), 0, 1_000_000)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 257, 4097])
def test_ragged_sizes_fp64(ctx, n):
    _fp64_case(ctx, W.biased_sample(), 12345, n, threads=1)


def test_split_resume_fp64(ctx):
    import torch
    prob = W.biased_sample()
    sim = B.Simulation(ctx, prob)
    sim.run(first=0, n=30_000, precision="fp64")
    sim.run(first=30_000, n=70_001, precision="fp64")
    torch.cuda.synchronize()
    g = sim.results()
    o = O.run(prob, first=0, n=100_001, threads=8)
    for t, (sw, sw2, nh) in enumerate(g):
        assert nh == 100_001
        np.testing.assert_allclose(sw, o.sumw[t], rtol=1e-9, atol=1e-9)


def test_vessel_sample_fp64_elementwise(ctx):
    _fp64_case(ctx, W.vessel_sample(), 0, 100_000)


def test_m3_guide_fp64_elementwise(ctx):
    _fp64_case(ctx, W.m3_guide(nbins_xy=50, nbins_div=20), 0, 100_000)


def test_capped_and_outside(ctx):
    # closed all-mirror box with R = 1 everywhere: histories never end and are capped
    box = W.Volume("box", (0.0, 0.0, 0.0), (10.0, 10.0, 10.0), mirror_mask=0b111111,
                   mirror=W.Mirror(model="linear", R0=1.0, Qc=100.0, alpha=0.0, m=1.0))
    src = W.Source("pencil", origin=(0.0, 0.0, 0.0), direction=(0.3, 0.4, 0.866), spectrum="mono", lam0=2.0)
    prob = W.Problem([], [box], src, [W.Tally(trigger="escape")], n_histories=64, name="trap")
    gres, grec, ores, same = _fp64_case(ctx, prob, 0, 64, threads=1)
    assert np.all(grec["term"] == B.END_CAPPED) and np.all(grec["n_steps"] == 10000)
    # a source outside the world is terminated at birth and scores nothing
    prob2 = W.analog_sample(10)
    prob2.source = dataclasses.replace(prob2.source, origin=(0.0, 0.0, -2000.0))
    gres, grec, ores, same = _fp64_case(ctx, prob2, 0, 10, threads=1)
    assert np.all(grec["term"] == B.END_OUTSIDE)


def test_run_seed_fp64_elementwise(ctx):
    """pr_set_seed: with another run seed (one above 2^32, so both key words
    matter) the histories are those of the oracle under that seed, and they
    differ from the default seed's; setting the default seed back restores them."""
    prob = W.analog_sample(20_000)
    base = O.run(prob, seed=4096, first=0, n=20_000, threads=8, records=True).records
    try:
        for sd in (12345, (1 << 40) + 7):
            ctx.set_seed(sd)
            print(f"[case] analog sample fp64, seed {sd}", flush=True)
            gres, grec, gst = gpu_run(ctx, prob, first=0, n=20_000, precision="fp64")
            ores = O.run(prob, seed=sd, first=0, n=20_000, threads=8, records=True)
            same = compare_records_fp64(grec, ores.records)
            compare_tallies_fp64(gres, ores, grec, ores.records, same)
            assert (grec["hash"] != base["hash"]).mean() > 0.5
    finally:
        ctx.set_seed(4096)
    _, grec, _ = gpu_run(ctx, prob, first=0, n=20_000, precision="fp64")
    assert (grec["hash"] == base["hash"]).mean() >= 0.999


def test_reads_wait_for_runs_on_any_stream(ctx):
    """A run issued on a side stream and read back from the default stream gives
    the same tallies as a run on the default stream: reads wait for the device."""
    import torch
    prob = W.biased_sample(n=2_000_000)
    ref = B.Simulation(ctx, prob)
    ref.run(first=0, n=prob.n_histories, precision="fp32")
    expect = ref.results()
    side = torch.cuda.Stream()
    sim = B.Simulation(ctx, prob)
    with torch.cuda.stream(side):
        sim.run(first=0, n=prob.n_histories, precision="fp32")
    got = sim.results()          # read from the default stream, no explicit synchronisation
    for (sw, sw2, nh), (rw, rw2, rn) in zip(got, expect):
        assert nh == rn == prob.n_histories
        np.testing.assert_allclose(sw, rw, rtol=1e-9, atol=1e-12)


def test_detector_and_tally_filters(ctx):
    prob = W.analog_sample(50_000)
    prob.volumes.append(W.Volume("box", (0.0, 0.0, 300.0), (200.0, 200.0, 2.0), parent=0, detector=True))
    prob.tallies = [W.Tally(trigger="detect", trigger_volume=2, axes=[W.Axis("x", -100, 100, 40), W.Axis("y", -100, 100, 40)]),
                    W.Tally(trigger="escape", filter="nscat_eq", filter_arg=2, axes=[W.Axis("theta2", 0, 180, 90)]),
                    W.Tally(trigger="absorb", axes=[W.Axis("nscat", 0, 6, 6)]),
                    W.Tally(trigger="escape", axes=[W.Axis("z", -1000, 1000, 50), W.Axis("div_x", -90, 90, 30)])]
    _fp64_case(ctx, prob, 777, 50_000)


def _grazing_problem(n, grid):
    """A beam cutting the edge of a vacuum box (sides 20 mm at the origin) along the
    diagonal of the x-z plane: the rays pass through pieces of the box from about
    28 um long down to below one FP32 ulp of the position, or miss it.  With
    grid=True nine small boxes away from the beam give the world a daughter grid."""
    vols = [W.Volume("box", (0.0, 0.0, 0.0), (200.0, 200.0, 200.0)),
            W.Volume("box", (0.0, 0.0, 0.0), (20.0, 20.0, 20.0), parent=0)]
    if grid:
        vols += [W.Volume("box", (x, 50.0, 50.0), (5.0, 5.0, 5.0), parent=0) for x in range(-80, 81, 20)]
    c = float(np.sqrt(0.5))
    src = W.Source("rect", origin=(-30.0, 0.0, 10.0), direction=(c, 0.0, -c), size=(4e-5, 1.0),
                   spectrum="mono", lam0=2.0)
    return W.Problem([], vols, src, [W.Tally(trigger="escape")], n_histories=n, name="grazing")


@pytest.mark.parametrize("grid", [False, True])
def test_grazing_edge_fp32_makes_progress(ctx, grid):
    """A piece shorter than the position's rounding must not trap a history: every
    ray enters and leaves the box (or misses it) and escapes within four steps."""
    n = 100_000
    prob = _grazing_problem(n, grid)
    print(f"[case] grazing edge fp32 grid={grid} n={n}", flush=True)
    gres, grec, gst = gpu_run(ctx, prob, first=0, n=n, precision="fp32")
    assert gst["capped"] == 0
    assert np.all(grec["term"] == B.END_ESCAPE)
    assert grec["n_steps"].max() <= 4
    assert gres[0][2] == n and abs(gres[0][0][0] - n) < 1e-6


def test_imaging_history_that_grazed_an_edge_fp32(ctx):
    """History 21469436 of the 1000-box imaging problem (run seed 4096) grazes a box
    edge after its first scattering; without the FP32 piece tolerance it re-entered
    the same piece until the step cap."""
    prob = W.imaging_problem(n=64)
    print("[case] imaging fp32 histories 21469436..+64", flush=True)
    gres, grec, gst = gpu_run(ctx, prob, first=21_469_436, n=64, precision="fp32")
    assert gst["capped"] == 0 and grec["n_steps"].max() < 200


@pytest.mark.parametrize("grid", [False, True])
def test_grazing_edge_fp64_elementwise(ctx, grid):
    _, grec, _, same = _fp64_case(ctx, _grazing_problem(20_000, grid), 0, 20_000)
    assert grec["n_steps"].max() <= 4


# ---------------------------------------------------------------------------
# FP32 mixed policy
# ---------------------------------------------------------------------------

def _fp32_case(ctx, prob, n, n_oracle=None, threads=8):
    """FP32 GPU run over ids [0, n) against an independent oracle sample (ids from
    ORACLE_FIRST): the tally agreement test on every tally."""
    print(f"[case] {prob.name} fp32 n={n}", flush=True)
    gres, _, gst = gpu_run(ctx, prob, first=0, n=n, precision="fp32", records=False)
    ores = O.run(prob, first=ORACLE_FIRST, n=n_oracle or n, threads=threads)
    pvals = []
    for t, (sw, sw2, nh) in enumerate(gres):
        assert nh == n
        p, z = tally_stat_test(sw, sw2, nh, ores.sumw[t], ores.sumw2[t], ores.n)
        pvals.append(p)
    assert min(pvals) > 1e-3, pvals
    assert gst["histories"] == n and gst["capped"] == 0
    return gres, ores


def test_analog_sample_fp32_tally_agreement(ctx):
    _fp32_case(ctx, W.analog_sample(1_000_000), 1_000_000)


def test_biased_sample_fp32_tally_agreement(ctx):
    _fp32_case(ctx, W.biased_sample(), 1_000_000)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 4097])
def test_ragged_sizes_fp32(ctx, n):
    """Ragged run sizes: every history of the range runs exactly once (its record
    is written, with the draw count of a started history) and the FP32 records
    pair with the FP64 ones id by id."""
    prob = W.biased_sample()
    gres, grec, gst = gpu_run(ctx, prob, first=12345, n=n, precision="fp32")
    _, g64, _ = gpu_run(ctx, prob, first=12345, n=n, precision="fp64")
    assert gst["histories"] == n
    assert np.all(grec["term"] > 0) and np.all(grec["n_draws"] >= 1)
    # common random numbers: the source draws (the wavelength is fixed) agree
    assert (grec["hash"] == g64["hash"]).mean() >= (0.9 if n > 60 else 0.0)


def test_vessel_sample_fp32_tally_agreement(ctx):
    _fp32_case(ctx, W.vessel_sample(), 1_000_000)


def test_m3_guide_fp32_tally_agreement(ctx):
    _fp32_case(ctx, W.m3_guide(nbins_xy=50, nbins_div=20), 1_000_000)


def test_fp32_results_independent_of_launch_tuning(ctx):
    """Each history's outcome depends only on (seed, history id), not on which
    lane or block runs it: tallies agree across launch tunings up to the
    order of floating-point summation."""
    import torch
    prob = W.biased_sample(n=300_000)
    base = ctx.get_tuning()
    results = []
    tunings = [dict(waves_per_simd=4), dict(refill_threshold=1, chunk=64, block=64), dict(bin_cache_slots=0, lds_tally_bytes=0),
               dict(refill_threshold=64, chunk=4096, blocks_per_cu=1, bin_cache_slots=4096),
               dict(waves_per_simd=5), dict(waves_per_simd=5, refill_threshold=8, chunk=128, bin_cache_slots=0)]
    try:
        for t in tunings:
            ctx.set_tuning(**{**base, **t})
            sim = B.Simulation(ctx, prob)
            ctx.reset_stats()
            sim.run(first=0, n=prob.n_histories, precision="fp32")
            torch.cuda.synchronize()
            results.append((sim.results(), ctx.read_stats()))
    finally:
        ctx.set_tuning(**base)
    ref, ref_st = results[0]
    for res, st in results[1:]:
        assert st == ref_st
        for (sw, sw2, nh), (rw, rw2, rn) in zip(res, ref):
            assert nh == rn
            np.testing.assert_allclose(sw, rw, rtol=1e-9, atol=1e-12)
            np.testing.assert_allclose(sw2, rw2, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------------------
# Scatter-order-resolved momentum transfer and per-process biasing
# ---------------------------------------------------------------------------

def _q_orders_problem(mat, n):
    """The biased sample with momentum-transfer tallies resolved by scattering
    order (DeltaMomentum with a scattering-number filter) and a scattering-number
    histogram of escapes (MultiScat)."""
    p = W.analog_sample(n)
    p.materials = [mat]
    p.tallies = [W.Tally(trigger="escape", filter="nscat_eq", filter_arg=1, axes=[W.Axis("q", 0.0, 8.0, 400)]),
                 W.Tally(trigger="escape", filter="nscat_eq", filter_arg=2, axes=[W.Axis("q", 0.0, 8.0, 200)]),
                 W.Tally(trigger="escape", filter="scattered", axes=[W.Axis("q", 0.0, 8.0, 400)]),
                 W.Tally(trigger="escape", axes=[W.Axis("nscat", 0, 8, 8)]),
                 W.Tally(trigger="absorb")]
    p.name = "q-orders"
    return p


@pytest.mark.parametrize("gs,ga", [(4.0, 0.5), (1.0, 0.0), (0.0, 1.0), (0.0, 0.0)])
def test_q_orders_and_bias_factors_fp64_elementwise(ctx, gs, ga):
    mat = W.sample_material().biased(scatter_bias=gs, abs_bias=ga)
    _, grec, _, _ = _fp64_case(ctx, _q_orders_problem(mat, 50_000), 4242, 50_000)
    if gs == 0.0 and ga == 0.0:
        # every process removed: the sample is vacuum, every history passes with weight 1
        assert np.all(grec["n_scat"] == 0) and np.all(grec["w"] == 1.0) and np.all(grec["term"] == B.END_ESCAPE)


@pytest.mark.parametrize("gs,ga", [(4.0, 0.5), (1.0, 0.0)])
def test_q_orders_and_bias_factors_fp32(ctx, gs, ga):
    mat = W.sample_material().biased(scatter_bias=gs, abs_bias=ga)
    _fp32_case(ctx, _q_orders_problem(mat, 1_000_000), 1_000_000)


def test_biasing_validations_on_gpu(ctx):
    """The paper's two checks of the biasing scheme, on the GPU's FP32 policy with
    a synthetic powder: (1) the total-scattering Q distribution of the biased run
    (scatter bias 4, absorption bias 0.5) agrees with the unbiased run; (2) at equal
    history counts biasing lowers the single-scattering Q tally's variance on a
    thin sample (the quantity biasing targets)."""
    n = 2_000_000
    mat = dataclasses.replace(W.sample_material(), number_density=0.006)
    res = {}
    for key, m in (("analog", mat), ("biased", mat.biased(scatter_bias=4.0, abs_bias=0.5))):
        print(f"[case] biasing validation {key} fp32 n={n}", flush=True)
        gres, _, _ = gpu_run(ctx, _q_orders_problem(m, n), first=0, n=n, precision="fp32", records=False)
        res[key] = gres
    # (1) every tally agrees between the analog and the biased run
    for t in range(5):
        a, b = res["analog"][t], res["biased"][t]
        p, z = tally_stat_test(a[0], a[1], a[2], b[0], b[1], b[2])
        assert p > 1e-3, (t, p)
    # (2) single-scattering Q: summed variance of the bin means drops
    def var_sum(r):
        sw, sw2, nh = r
        m = sw / nh
        return float(np.sum((sw2 / nh - m * m) / (nh - 1)))
    assert var_sum(res["biased"][0]) < 0.5 * var_sum(res["analog"][0])


# ---------------------------------------------------------------------------
# Moderator-surface gun and the paper's m = 1 guide benchmark
# ---------------------------------------------------------------------------

def _gun_problem(n):
    vols = [W.Volume("box", (0.0, 0.0, 1000.0), (400.0, 400.0, 3000.0)),
            W.Volume("box", (0.0, 0.0, 1501.0), (300.0, 300.0, 2.0), parent=0, detector=True)]
    src = W.Source("moderator", origin=(10.0, -5.0, 0.0), size=(60.0, 40.0), spectrum="uniform", lam_lo=1.0,
                   lam_hi=4.0, slit_center=(3.0, 4.0, 500.0), slit_size=(20.0, 30.0))
    tallies = [W.Tally(trigger="detect", trigger_volume=1,
                       axes=[W.Axis("x", -150, 150, 60), W.Axis("y", -150, 150, 60), W.Axis("lambda", 1, 4, 6)])]
    return W.Problem([], vols, src, tallies, n_histories=n, name="moderator-gun")


def test_moderator_gun_fp64_elementwise(ctx):
    _fp64_case(ctx, _gun_problem(50_000), 99, 50_000)


def test_paper_guide_fp64_elementwise(ctx):
    _, grec, _, _ = _fp64_case(ctx, W.paper_guide(100_000), 0, 100_000)
    assert (grec["term"] == B.END_DETECT).mean() > 0.2


def test_paper_guide_fp32_tally_agreement(ctx):
    _fp32_case(ctx, W.paper_guide(1_000_000), 1_000_000)


# ---------------------------------------------------------------------------
# Time of flight and the disk chopper
# ---------------------------------------------------------------------------

def test_paper_chopper_fp64_elementwise(ctx):
    _, grec, _, _ = _fp64_case(ctx, W.paper_chopper(100_000), 0, 100_000)
    assert 0.15 < (grec["term"] == B.END_DETECT).mean() < 0.3


def test_paper_chopper_mono_fp64_elementwise(ctx):
    _fp64_case(ctx, W.paper_chopper(50_000, lam_mono=2.0, phase=37.0, tof_bins=3000), 5, 50_000)


def test_paper_chopper_fp32_tally_agreement(ctx):
    _fp32_case(ctx, W.paper_chopper(1_000_000), 1_000_000)
    _fp32_case(ctx, W.paper_chopper(1_000_000, chopper=False), 1_000_000)


# ---------------------------------------------------------------------------
# Tabulated cross sections
# ---------------------------------------------------------------------------

def _tabulated_problem(n):
    """The powder sample with absorption and incoherent cross sections given as
    tables (curved in lambda) and a uniform 1-5 A beam crossing many table rows;
    coherent scattering stays the Bragg sum."""
    p = W.analog_sample(n)
    base = W.sample_material().biased(scatter_bias=2.0)
    rows = np.linspace(0.8, 5.5, 24)
    mat = dataclasses.replace(base, table_lambda=rows, table_sigma_abs=1.5 + 0.4 * rows ** 1.5,
                              table_sigma_inc=3.0 + np.sin(rows))
    p.materials = [mat]
    p.source = dataclasses.replace(p.source, spectrum="uniform", lam_lo=1.0, lam_hi=5.0)
    p.tallies = [W.Tally(trigger="escape", filter="scattered", axes=[W.Axis("theta2", 0, 180, 180), W.Axis("lambda", 1, 5, 8)]),
                 W.Tally(trigger="escape", filter="unscattered", axes=[W.Axis("lambda", 1, 5, 40)]),
                 W.Tally(trigger="absorb", axes=[W.Axis("lambda", 1, 5, 40)])]
    p.name = "tabulated"
    return p


def test_tabulated_cross_sections_fp64_elementwise(ctx):
    _fp64_case(ctx, _tabulated_problem(100_000), 31, 100_000)


def test_tabulated_cross_sections_fp32(ctx):
    _fp32_case(ctx, _tabulated_problem(1_000_000), 1_000_000)


# ---------------------------------------------------------------------------
# Edge cases: empty runs, the top of the history-id range
# ---------------------------------------------------------------------------

def _largest_material_problem(n):
    """The largest material the library accepts: 1024 Bragg families (d from 6 A
    down to 0.5 A, so every 1.2-2.4 A wavelength sees hundreds of active edges)
    and 4096-row absorption/incoherent tables, in the sample cylinder under a
    uniform 1.2-2.4 A pencil beam, scattering biased by 2."""
    rng = np.random.default_rng(7)
    k = 1024
    d = np.sort(rng.uniform(0.5, 6.0, k))[::-1].copy()
    lam = np.linspace(0.4, 12.0, 4096)
    m = dataclasses.replace(W.sample_material(), d=d, mult=rng.integers(1, 49, k).astype(np.int32),
                            f2=rng.uniform(0.0, 0.3, k), table_lambda=lam,
                            table_sigma_abs=1.5 + 0.8 * lam, table_sigma_inc=4.0 + 0.1 * np.sin(lam))
    prob = W.analog_sample(n)
    prob.materials = [m.biased(scatter_bias=2.0)]
    prob.source = dataclasses.replace(prob.source, spectrum="uniform", lam_lo=1.2, lam_hi=2.4)
    prob.name = "largest-material"
    return prob


def test_largest_material_fp64_elementwise(ctx):
    _fp64_case(ctx, _largest_material_problem(20_000), 0, 20_000)


def test_largest_material_fp32(ctx):
    _fp32_case(ctx, _largest_material_problem(1_000_000), 1_000_000)


def test_empty_runs_change_nothing(ctx):
    import torch
    print("[case] empty runs", flush=True)
    prob = W.analog_sample(0)
    sim = B.Simulation(ctx, prob)
    ctx.reset_stats()
    for prec in ("fp64", "fp32"):
        sim.run(first=123, n=0, precision=prec)
    batch = W.Batch([W.analog_sample(0), W.analog_sample(0)])
    br = B.BatchRun(ctx, batch)
    br.run()
    pid = ctx.prepare_batch(br.descriptors(), stride=1)
    ctx.run_prepared(pid)
    torch.cuda.synchronize()
    ctx.release_batch(pid)
    assert ctx.read_stats()["histories"] == 0
    for s in [sim] + br.sims:
        for sw, sw2, nh in s.results():
            assert nh == 0 and not sw.any() and not sw2.any()
    # an empty simulation inside a batch leaves the others as run alone
    one = B.BatchRun(ctx, W.Batch([W.analog_sample(0), W.analog_sample(2000)]))
    alone = B.Simulation(ctx, W.analog_sample(2000))
    one.run()
    alone.run(first=one.offsets[1], n=2000, precision="fp32")
    torch.cuda.synchronize()
    for (a, a2, na), (b, b2, nb) in zip(one.sims[1].results(), alone.results()):
        assert na == nb == 2000
        assert np.allclose(a, b, rtol=1e-12, atol=0) and np.allclose(a2, b2, rtol=1e-12, atol=0)


def test_top_of_the_history_id_range_fp64(ctx):
    """History ids up to 2^62 (the largest accepted first id) drive the counter's
    high words: element-wise parity there too."""
    first = (1 << 62) - 1000
    _fp64_case(ctx, W.biased_sample(1000), first, 1000, threads=4)


def test_history_range_limits_are_enforced(ctx):
    sim = B.Simulation(ctx, W.analog_sample(10))
    with pytest.raises(B.PromptError) as e:
        sim.run(first=(1 << 62) + 1, n=10, precision="fp64")
    assert e.value.code == -1
    with pytest.raises(B.PromptError) as e:
        sim.run(first=0, n=(1 << 48) + 1, precision="fp32")
    assert e.value.code == -1
