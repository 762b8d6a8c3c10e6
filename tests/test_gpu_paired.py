"""FP32 mixed policy against the FP64 policy on the SAME history ids, for every
FP32 workload: per tally bin, the difference of the two tallies is scored
against the paired variance sum_h (x32_h - x64_h)^2 of the histories' own
contributions (each history's bin from its record), with a relative FP32
rounding allowance of 2e-5 per bin (parity.paired_check).  The FP64 policy is
itself checked history by history against the oracle elsewhere, so this is the
FP32 policy's error against the FP64 path, stated per tally (printed).  The
batch is paired through its simulations: a batched FP32 run against the same
simulations run one by one in FP64."""
import dataclasses

import numpy as np
import pytest

from paper_2304_06226_amd import binding as B
from paper_2304_06226_amd import workloads as W

from parity import gpu_run, paired_check, paired_fp32_fp64
from test_gpu_batch import _big_grid_problem, _deep_scene_problem, _mixed_grid_problem, _nested_grid_problem, _small_batch
from test_gpu_parity import _fp32_case, _largest_material_problem, _q_orders_problem, _tabulated_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(device=0, seed=4096)
    yield c
    c.close()


def far_chopper(n):
    """A 1 um thick disk chopper reached by neutrons born 4 m before it and 5 m from
    the origin (the chopper section's disk, Table tableDiskChopper: 4 windows of
    20 degrees, radii 130 and 250 mm, 100 Hz), a TOF detector 2 mm behind it."""
    vols = [W.Volume("box", (0.0, 0.0, 7000.0), (1200.0, 1200.0, 6000.0)),
            W.Volume("cylinder", (0.0, -190.0, 9000.0), (250.0, 0.001), axis=2, parent=0,
                     chopper=W.Chopper(n=4, r=130.0, rot_freq=100.0, theta0=20.0, phase=0.0)),
            W.Volume("box", (0.0, 0.0, 9002.0), (300.0, 300.0, 2.0), parent=0, detector=True)]
    src = W.Source("moderator", origin=(0.0, 0.0, 5000.0), size=(1.0, 1.0), spectrum="maxwell", kT=0.025249,
                   lam_lo=0.5, lam_hi=10.0, slit_center=(0.0, 0.0, 9000.0), slit_size=(45.0, 45.0))
    tallies = [W.Tally(trigger="detect", trigger_volume=2, axes=[W.Axis("tof", 0.0, 0.02, 400)]),
               W.Tally(trigger="detect", trigger_volume=2)]
    return W.Problem([], vols, src, tallies, n_histories=n, name="far_chopper")


CASES = {
    "analog_sample": (lambda: W.analog_sample(1_000_000), 1_000_000),
    "biased_sample": (lambda: W.biased_sample(), 1_000_000),
    "vessel": (lambda: W.vessel_sample(), 1_000_000),
    "m3_guide": (lambda: W.m3_guide(nbins_xy=50, nbins_div=20), 1_000_000),
    "imaging": (lambda: W.imaging_problem(n=1_000_000), 1_000_000),
    "paper_guide": (lambda: W.paper_guide(), 1_000_000),
    "paper_chopper": (lambda: W.paper_chopper(), 1_000_000),
    "paper_chopper_open": (lambda: W.paper_chopper(chopper=False), 1_000_000),
    "far_chopper": (lambda: far_chopper(1_000_000), 1_000_000),
    "tabulated": (lambda: _tabulated_problem(1_000_000), 1_000_000),
    "largest_material": (lambda: _largest_material_problem(1_000_000), 1_000_000),
    "q_orders_4_0.5": (lambda: _q_orders_problem(W.sample_material().biased(scatter_bias=4.0, abs_bias=0.5),
                                                 1_000_000), 1_000_000),
    "q_orders_1_0": (lambda: _q_orders_problem(W.sample_material().biased(scatter_bias=1.0, abs_bias=0.0), 1_000_000),
                     1_000_000),
    "mixed_kind_grid": (lambda: _mixed_grid_problem(1_000_000), 1_000_000),
    "nested_grid": (lambda: _nested_grid_problem(1_000_000), 1_000_000),
    "deep_scene": (lambda: _deep_scene_problem(1_000_000), 1_000_000),
    "big_grid": (lambda: _big_grid_problem(1_000_000), 1_000_000),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_paired_with_fp64(ctx, name):
    make, n = CASES[name]
    paired_fp32_fp64(ctx, make(), first=0, n=n, label=name)


def test_far_chopper_is_applied_in_fp32(ctx):
    """The thin disk reached from 5 m is entered in FP32 (its mask applies): the
    detected fraction is that of the FP64 policy, well below the open fraction."""
    n = 400_000
    prob = far_chopper(n)
    _, rec32, _ = gpu_run(ctx, prob, first=0, n=n, precision="fp32")
    _, rec64, _ = gpu_run(ctx, prob, first=0, n=n, precision="fp64")
    det32 = (rec32["term"] == B.END_DETECT).mean()
    det64 = (rec64["term"] == B.END_DETECT).mean()
    killed32 = (rec32["term"] == B.END_KILL).mean()
    assert killed32 > 0.5 and abs(det32 - det64) < 1e-3, (det32, det64, killed32)


def test_far_chopper_fp32_against_oracle(ctx):
    """The far chopper in FP32 against the oracle on disjoint history ids (the
    tally agreement test on the TOF histogram and the detected counter)."""
    _fp32_case(ctx, far_chopper(1_000_000), 1_000_000)


def test_batch_paired_with_fp64_one_by_one(ctx):
    """The batched FP32 run of a small batch (24 powder simulations and an imaging
    setup), paired simulation by simulation with FP64 runs of the same ids; the
    FP32 records come from one-by-one FP32 runs, whose tallies equal the batch's
    up to summation order."""
    import torch
    batch = _small_batch()
    br = B.BatchRun(ctx, batch, base=3_000_000)
    br.reset()
    br.run()
    torch.cuda.synchronize()
    for i in list(range(0, 24, 3)) + [24]:
        prob = batch.problems[i]
        n = prob.n_histories
        tb = br.sims[i].results()
        r32, rec32, _ = gpu_run(ctx, prob, first=br.offsets[i], n=n, precision="fp32")
        for (a, a2, na), (b, b2, nb) in zip(tb, r32):
            assert na == nb == n
            np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12)
        r64, rec64, _ = gpu_run(ctx, prob, first=br.offsets[i], n=n, precision="fp64_persistent")
        paired_check(prob, tb, rec32, r64, rec64, label=f"batch sim {i} ({prob.name})")
