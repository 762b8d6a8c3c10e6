"""GPU: the persistent FP64 policy (PR_FP64_PERSISTENT) against the plain FP64
kernel and the oracle, through the C-ABI.

Both policies run the same FP64 step on every history with the same random
numbers (draw k of history h from Philox block (k >> 1, h)), so each history's
record (event hash, termination, counts, final weight, position, direction,
wavelength, region) must be identical bit for bit, the run statistics equal,
and every tally bin equal up to the order in which the atomics summed it.
Parity with the oracle then follows from the plain kernel's own parity; one
case checks it directly as well.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_06226_amd import binding as B
from paper_2304_06226_amd import workloads as W

from parity import compare_records_fp64, compare_tallies_fp64, gpu_run
from test_gpu_parity import _grazing_problem, _gun_problem, _q_orders_problem, _tabulated_problem

pytestmark = pytest.mark.gpu

# a bin's sum of n non-negative weights in another order: |difference| stays
# within about sqrt(n) ulps, far inside this bound for n <= 1e6
SUM_RTOL = 1e-11


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(device=0, seed=4096)
    yield c
    c.close()


def _same_records(a, b):
    assert len(a) == len(b)
    for f in a.dtype.names:
        assert np.array_equal(a[f], b[f]), f"record field {f} differs in {np.sum(np.any((a[f] != b[f]).reshape(len(a), -1), axis=1))} histories"


def _same_tallies(ra, rb):
    assert len(ra) == len(rb)
    for (sa, s2a, na), (sb, s2b, nb) in zip(ra, rb):
        assert na == nb
        assert np.array_equal(sa == 0, sb == 0)
        np.testing.assert_allclose(sa, sb, rtol=SUM_RTOL, atol=0)
        np.testing.assert_allclose(s2a, s2b, rtol=SUM_RTOL, atol=0)


def _against_plain(ctx, prob, first, n):
    print(f"[case] {prob.name} fp64_persistent vs fp64 plain first={first} n={n}", flush=True)
    pres, prec, pst = gpu_run(ctx, prob, first=first, n=n, precision="fp64")
    qres, qrec, qst = gpu_run(ctx, prob, first=first, n=n, precision="fp64_persistent")
    _same_records(qrec, prec)
    _same_tallies(qres, pres)
    assert qst == pst
    return qres, qrec


CASES = [
    ("analog_sample", lambda: W.analog_sample(), 0, 100_000),
    ("biased_sample", lambda: W.biased_sample(), 0, 1_000_000),
    ("vessel_sample", lambda: W.vessel_sample(), 3_000_000, 200_000),
    ("m3_guide", lambda: W.m3_guide(nbins_xy=40, nbins_div=20), 0, 200_000),
    ("imaging", lambda: W.imaging_problem(), 0, 200_000),
    ("paper_guide", lambda: W.paper_guide(), 0, 200_000),
    ("paper_chopper", lambda: W.paper_chopper(), 0, 200_000),
    ("moderator_gun", lambda: _gun_problem(50_000), 0, 50_000),
    ("tabulated", lambda: _tabulated_problem(50_000), 0, 50_000),
    ("q_orders_biased", lambda: _q_orders_problem(W.sample_material().biased(scatter_bias=4.0, abs_bias=0.5),
                                                  50_000), 4242, 50_000),
    ("grazing", lambda: _grazing_problem(50_000, False), 0, 50_000),
    ("grazing_grid", lambda: _grazing_problem(50_000, True), 0, 50_000),
]


@pytest.mark.parametrize("name,make,first,n", CASES, ids=[c[0] for c in CASES])
def test_records_equal_plain(ctx, name, make, first, n):
    _against_plain(ctx, make(), first, n)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 257, 4097])
def test_ragged_sizes(ctx, n):
    _against_plain(ctx, W.biased_sample(), 12345, n)


def test_top_of_the_history_id_range(ctx):
    _against_plain(ctx, W.biased_sample(1000), (1 << 62) - 1000, 1000)


def test_against_oracle(ctx):
    prob = W.biased_sample()
    first, n = 777_000, 100_000
    print(f"[case] {prob.name} fp64_persistent vs oracle first={first} n={n}", flush=True)
    gres, grec, gst = gpu_run(ctx, prob, first=first, n=n, precision="fp64_persistent")
    ores = O.run(prob, first=first, n=n, threads=8, records=True)
    same = compare_records_fp64(grec, ores.records)
    compare_tallies_fp64(gres, ores, grec, ores.records, same)
    for k in ("histories", "escaped", "absorbed", "killed", "detected", "capped", "outside"):
        assert abs(gst[k] - ores.stats[k]) <= int((~same).sum()), k


TUNINGS = [
    dict(block=64, blocks_per_cu=0, refill_threshold=1, chunk=1, bin_cache_slots=0, lds_tally_bytes=32768),
    dict(block=256, blocks_per_cu=1, refill_threshold=64, chunk=4096, bin_cache_slots=2048, lds_tally_bytes=0),
    dict(block=128, blocks_per_cu=2, refill_threshold=17, chunk=100, bin_cache_slots=256, lds_tally_bytes=32768),
    dict(block=256, blocks_per_cu=0, refill_threshold=32, chunk=1024, bin_cache_slots=256, lds_tally_bytes=32768,
         grid_chunk=7),
]


@pytest.mark.parametrize("tuning", range(len(TUNINGS)))
@pytest.mark.parametrize("which", ["biased_sample", "imaging"])
def test_results_independent_of_launch_tuning(ctx, tuning, which):
    prob = W.biased_sample(200_000) if which == "biased_sample" else W.imaging_problem(100_000)
    saved = ctx.get_tuning()
    try:
        ctx.set_tuning(**TUNINGS[tuning])
        _against_plain(ctx, prob, 0, prob.n_histories)
    finally:
        ctx.set_tuning(**saved)


def test_empty_run_changes_nothing(ctx):
    import torch
    sim = B.Simulation(ctx, W.analog_sample(10))
    sim.run(first=0, n=0, precision="fp64_persistent")
    torch.cuda.synchronize()
    for sw, sw2, nh in sim.results():
        assert nh == 0 and not np.any(sw) and not np.any(sw2)
