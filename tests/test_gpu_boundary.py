"""The C-ABI's contracts on the GPU: runs overlapping on different streams,
caller workspaces and caller-owned tally storage, the step-cap status, the
first-collision trigger (against the oracle, history by history), and the
privatised tally slices of monochromatic sources."""
import ctypes as C
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_06226_amd import binding as B
from paper_2304_06226_amd import workloads as W

from parity import compare_records_fp64, compare_tallies_fp64, gpu_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(device=0, seed=4096)
    yield c
    c.close()


def _close(res, ref, rtol=1e-9):
    for (sw, sw2, nh), (rw, rw2, rn) in zip(res, ref):
        assert nh == rn
        np.testing.assert_allclose(sw, rw, rtol=rtol, atol=1e-12)
        np.testing.assert_allclose(sw2, rw2, rtol=rtol, atol=1e-12)


def test_overlapping_runs_on_two_streams(ctx):
    """Two FP32 runs of one context issued back to back on two non-blocking
    streams, with nothing in between that synchronises, each into its own tallies:
    each equals its twin run alone (the runs' history-claim counters are separate,
    so no history is lost or run twice)."""
    import torch
    p1, p2 = W.biased_sample(n=3_000_000), W.vessel_sample(n=2_000_000)
    s1, s2 = B.Simulation(ctx, p1), B.Simulation(ctx, p2)
    t1, t2 = B.Simulation(ctx, p1), B.Simulation(ctx, p2)
    torch.cuda.synchronize()
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    ctx.reset_stats()
    torch.cuda.synchronize()
    for rep in range(3):
        with torch.cuda.stream(a):
            s1.run(first=rep * p1.n_histories, n=p1.n_histories, precision="fp32")
        with torch.cuda.stream(b):
            s2.run(first=rep * p2.n_histories, n=p2.n_histories, precision="fp32")
    torch.cuda.synchronize()
    st = ctx.read_stats()
    assert st["histories"] == 3 * (p1.n_histories + p2.n_histories)
    for rep in range(3):
        t1.run(first=rep * p1.n_histories, n=p1.n_histories, precision="fp32")
        torch.cuda.synchronize()
        t2.run(first=rep * p2.n_histories, n=p2.n_histories, precision="fp32")
        torch.cuda.synchronize()
    _close(s1.results(), t1.results())
    _close(s2.results(), t2.results())


def test_caller_workspace_and_tally_storage(ctx):
    """A run with a caller workspace into tallies held in caller tensors equals
    the same run with library-owned storage; the caller's tensors hold the
    (sum w, sum w^2) pairs; too small a workspace or storage is PR_EWORKSPACE."""
    import torch
    prob = W.biased_sample(n=500_000)
    ref = B.Simulation(ctx, prob)
    ref.run(first=0, n=prob.n_histories, precision="fp32")
    torch.cuda.synchronize()
    ws_bytes = ctx.workspace_size("fp32")
    assert ws_bytes == 256
    ws = torch.zeros(ws_bytes, dtype=torch.uint8, device="cuda")
    storage = [torch.full((ctx.tally_storage_size(t) // 8,), 7.0, dtype=torch.float64, device="cuda")
               for t in prob.tallies]
    mats = [ctx.create_material(m) for m in prob.materials]
    geom = ctx.create_geometry(prob.volumes, mats)
    src = ctx.create_source(prob.source)
    tallies = [ctx.create_tally(t, storage=s) for t, s in zip(prob.tallies, storage)]
    for s in storage:
        assert not s.any().item()            # zeroed at creation
    for prec in ("fp32", "fp64_persistent", "fp64"):
        ctx.run(geom, src, tallies, 0, prob.n_histories, precision=prec, workspace=ws)
        torch.cuda.synchronize()
        got = [ctx.read_tally(t) for t in tallies]
        if prec == "fp32":
            _close(got, ref.results())
            for s, (sw, sw2, _) in zip(storage, got):
                host = s.cpu().numpy()
                assert np.array_equal(host[0::2], sw) and np.array_equal(host[1::2], sw2)
        for t in tallies:
            ctx.reset_tally(t)
    with pytest.raises(B.PromptError) as e:
        ctx.run(geom, src, tallies, 0, 10, precision="fp32", workspace=ws[:255])
    assert e.value.code == B.PR_EWORKSPACE
    small = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(B.PromptError) as e:
        ctx.create_tally(prob.tallies[0], storage=small)
    assert e.value.code == B.PR_EWORKSPACE
    torch.cuda.synchronize()


def test_capped_status_code(ctx):
    """pr_read_stats fills the statistics and returns PR_ECAPPED when histories hit
    the step cap; PR_OK again after a reset."""
    import torch
    box = W.Volume("box", (0.0, 0.0, 0.0), (10.0, 10.0, 10.0), mirror_mask=0b111111,
                   mirror=W.Mirror(model="linear", R0=1.0, Qc=100.0, alpha=0.0, m=1.0))
    src = W.Source("pencil", origin=(0.0, 0.0, 0.0), direction=(0.3, 0.4, 0.866), spectrum="mono", lam0=2.0)
    prob = W.Problem([], [box], src, [W.Tally(trigger="escape")], n_histories=16, name="trap")
    sim = B.Simulation(ctx, prob)
    ctx.reset_stats()
    sim.run(first=0, n=16, precision="fp32")
    torch.cuda.synchronize()
    st = B.pr_run_stats()
    rc = ctx.lib.pr_read_stats(ctx.h, C.byref(st), None)
    assert rc == B.PR_ECAPPED and st.capped == 16 and st.histories == 16
    ctx.reset_stats()
    rc = ctx.lib.pr_read_stats(ctx.h, C.byref(st), None)
    assert rc == 0 and st.capped == 0


def _first_collision_problem(n, gs=4.0, ga=0.5):
    p = W.analog_sample(n)
    p.materials = [W.sample_material().biased(scatter_bias=gs, abs_bias=ga)]
    p.tallies = [W.Tally(trigger="first_collision", axes=[W.Axis("theta2", 0.0, 180.0, 1800)]),
                 W.Tally(trigger="first_collision", filter="unscattered",
                         axes=[W.Axis("z", -6.0, 6.0, 24), W.Axis("x", -5.0, 7.0, 4)]),
                 W.Tally(trigger="first_collision", filter="nscat_eq", filter_arg=1,
                         axes=[W.Axis("div_x", -180, 180, 36), W.Axis("lambda", 1.0, 2.0, 2)]),
                 W.Tally(trigger="escape", filter="scattered", axes=[W.Axis("theta2", 0.0, 180.0, 180)])]
    p.name = "first-collision"
    return p


@pytest.mark.parametrize("prec", ["fp64", "fp64_persistent"])
def test_first_collision_tallies_fp64_elementwise(ctx, prec):
    prob = _first_collision_problem(100_000)
    print(f"[case] first-collision tallies {prec}", flush=True)
    gres, grec, gst = gpu_run(ctx, prob, first=321, n=100_000, precision=prec)
    ores = O.run(prob, first=321, n=100_000, threads=8, records=True)
    same = compare_records_fp64(grec, ores.records)
    compare_tallies_fp64(gres, ores, grec, ores.records, same)
    assert gres[0][0].sum() > 1000 and gres[1][0].sum() > 100


def test_first_collision_rejected_by_fp32_and_batches(ctx):
    prob = _first_collision_problem(10)
    sim = B.Simulation(ctx, prob)
    with pytest.raises(B.PromptError) as e:
        sim.run(first=0, n=10, precision="fp32")
    assert e.value.code == -1
    with pytest.raises(B.PromptError) as e:
        ctx.run_batch([(sim.geom, sim.src, sim.tallies, 0, 10)])
    assert e.value.code == -1


def _slice_problem(n, order):
    """The biased sample with 2theta x lambda tallies whose wavelength axis is
    last, first or in the middle (and one whose range excludes the source
    wavelength): the mixed policy privatises the slice at the source wavelength."""
    p = W.biased_sample(n=n)
    th = W.Axis("theta2", 0.0, 180.0, 900)
    la = W.Axis("lambda", 0.5, 5.0, 100)
    ns = W.Axis("nscat", 0, 4, 4)
    th4 = W.Axis("theta2", 0.0, 180.0, 400)
    axes = {"last": [th, la], "first": [la, th], "middle": [th4, la, ns], "outside": [th, W.Axis("lambda", 2.0, 5.0, 30)]}
    p.tallies = [W.Tally(trigger="escape", filter="scattered", axes=axes[order]),
                 W.Tally(trigger="escape", filter="unscattered"), W.Tally(trigger="absorb")]
    p.name = f"slice-{order}"
    return p


@pytest.mark.parametrize("order", ["last", "first", "middle", "outside"])
def test_tally_slices_equal_plain_fp64(ctx, order):
    """The persistent FP64 policy (slices privatised in LDS) gives the plain FP64
    policy's tallies (global atomics on the full tally) up to summation order, and
    the FP32 slices hold the same weight as FP32 runs without privatisation."""
    import torch
    prob = _slice_problem(300_000, order)
    r64, _, _ = gpu_run(ctx, prob, first=7, n=300_000, precision="fp64", records=False)
    rp, _, _ = gpu_run(ctx, prob, first=7, n=300_000, precision="fp64_persistent", records=False)
    _close(rp, r64, rtol=1e-11)
    if order != "outside":
        assert r64[0][0].sum() > 0
    base = ctx.get_tuning()
    try:
        r32, _, _ = gpu_run(ctx, prob, first=7, n=300_000, precision="fp32", records=False)
        ctx.set_tuning(**{**base, "lds_tally_bytes": 0, "bin_cache_slots": 0})
        g32, _, _ = gpu_run(ctx, prob, first=7, n=300_000, precision="fp32", records=False)
    finally:
        ctx.set_tuning(**base)
    _close(r32, g32)
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["guide", "vessel", "sample"])
def test_paired_global_scores_equal_cached_scores(ctx, name):
    """FP32 runs whose large tally scores straight into global memory (no bin
    cache: the wave scores together, paired-lane atomics) equal the same runs
    with an LDS bin cache (per-lane scoring) up to summation order."""
    import torch
    prob = {"guide": lambda: W.m3_guide(nbins_xy=50, nbins_div=20), "vessel": W.vessel_sample,
            "sample": W.biased_sample}[name]()
    n = 400_000
    base = ctx.get_tuning()
    try:
        # sample: a 4 KB LDS budget leaves its 2theta x lambda tally in global memory
        lds = 4096 if name == "sample" else base["lds_tally_bytes"]
        ctx.set_tuning(**{**base, "lds_tally_bytes": lds, "bin_cache_slots": 1024})
        cached, _, _ = gpu_run(ctx, prob, first=99, n=n, precision="fp32", records=False)
        ctx.set_tuning(**{**base, "lds_tally_bytes": lds, "bin_cache_slots": 0})
        paired, _, _ = gpu_run(ctx, prob, first=99, n=n, precision="fp32", records=False)
    finally:
        ctx.set_tuning(**base)
    _close(paired, cached)
    assert paired[0][0].sum() > 0
    torch.cuda.synchronize()
