"""The world crossing folded into the leaving step: when a convex volume (box,
cylinder, sphere) is the only daughter of a vacuum, mirrorless world of one of
those kinds, a history that leaves it can only fly on to the world's boundary,
and the kernels take that flight in the step that leaves the daughter; a
history born in such a world takes its first step (into the daughter or out of
the world) as soon as it is drawn.  Neither may change a history: every
world x daughter pairing runs both FP64 policies element-wise against the
oracle on the same ids (event hashes, steps, draws, end positions, times of
flight) and the FP32 policy paired with the FP64 one."""
import pytest

from oracle import oracle as O
from paper_2304_06226_amd import workloads as W

from parity import compare_records_fp64, compare_tallies_fp64, gpu_run, paired_fp32_fp64

pytestmark = pytest.mark.gpu

WORLDS = {"box": (2000.0, 1500.0, 2500.0), "cylinder": (900.0, 2200.0), "sphere": (1000.0,)}
DAUGHTERS = {"box": (10.0, 20.0, 8.0), "cylinder": (5.0, 20.0), "sphere": (6.0,)}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2304_06226_amd import binding as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(device=0, seed=4096)
    yield c
    c.close()


def _problem(world, daughter, n):
    """A biased powder sample of the given solid kind alone in a vacuum world of the
    given kind; a 14 x 14 mm Maxwellian beam, wider than the sample, so that some
    histories cross the world without meeting it; a time-of-flight tally keeps the
    clock running."""
    mats = [W.sample_material().biased(scatter_bias=2.0)]
    vols = [W.Volume(world, (0.0, 0.0, 0.0), WORLDS[world], axis=0),
            W.Volume(daughter, (0.5, -0.5, 0.0), DAUGHTERS[daughter], axis=1, parent=0, material=0)]
    src = W.Source("rect", origin=(0.0, 0.0, -100.0), size=(14.0, 14.0), spectrum="maxwell",
                   lam_lo=0.5, lam_hi=5.0, kT=0.025852)
    tallies = [W.Tally(trigger="escape", filter="scattered",
                       axes=[W.Axis("theta2", 0.0, 180.0, 180), W.Axis("lambda", 0.5, 5.0, 20)]),
               W.Tally(trigger="escape", filter="unscattered", axes=[W.Axis("tof", 0.0, 0.01, 50)]),
               W.Tally(trigger="absorb")]
    return W.Problem(mats, vols, src, tallies, n_histories=n, name=f"{daughter}-in-{world}")


@pytest.mark.parametrize("daughter", sorted(DAUGHTERS))
@pytest.mark.parametrize("world", sorted(WORLDS))
def test_world_crossing_fp64_elementwise(ctx, world, daughter):
    n = 20_000
    prob = _problem(world, daughter, n)
    ores = O.run(prob, first=0, n=n, threads=8, records=True)
    # the sample is met by some histories and missed by others
    assert 0 < (ores.records["n_steps"] == 1).sum() < n
    for precision in ("fp64", "fp64_persistent"):
        print(f"[case] {prob.name} {precision} n={n}", flush=True)
        gres, grec, gst = gpu_run(ctx, prob, first=0, n=n, precision=precision)
        same = compare_records_fp64(grec, ores.records)
        compare_tallies_fp64(gres, ores, grec, ores.records, same)
        assert gst["steps"] == int(ores.records["n_steps"].sum()) or not same.all()
        assert gst["escaped"] + gst["absorbed"] + gst["killed"] == n


@pytest.mark.parametrize("daughter", sorted(DAUGHTERS))
@pytest.mark.parametrize("world", sorted(WORLDS))
def test_world_crossing_fp32_pairs_with_fp64(ctx, world, daughter):
    prob = _problem(world, daughter, 200_000)
    paired_fp32_fp64(ctx, prob, first=0, n=200_000, label=prob.name)


def _void_problem(n):
    """The vessel's biased sample cylinder with a 4 x 8 x 4 mm void (vacuum) inside it,
    and a 30 x 30 x 2 mm aluminium plate 50 mm downstream, in a vacuum sphere under the
    vessel's Maxwellian 10 x 10 mm beam: histories enter the void from material and
    leave both solids for the world, so fold passes follow steps that end in a vacuum
    daughter as well as steps that leave for the world (two daughters: the
    lone-daughter crossing does not apply)."""
    prob = W.vessel_sample(n)
    prob.volumes = [prob.volumes[0], prob.volumes[2],
                    W.Volume("box", (1.0, 2.0, 0.5), (4.0, 8.0, 4.0), parent=1, material=-1),
                    W.Volume("box", (0.0, 0.0, 50.0), (30.0, 30.0, 2.0), parent=0, material=1)]
    prob.name = "void-in-sample"
    return prob


@pytest.mark.parametrize("workload,precision", [("sample", "fp32"), ("sample", "fp64_persistent"), ("sample", "fp64"),
                                                ("vessel", "fp32"), ("vessel", "fp64_persistent"),
                                                ("void", "fp32"), ("void", "fp64_persistent")])
def test_vacuum_steps_change_no_history(ctx, workload, precision):
    """The same ids with steps that draw nothing taken early (vacuum_steps = 1:
    the biased sample's world crossing folded into the leaving step and its
    newborn steps taken in the refill pass; fold passes in the vessel and in a
    sample with a void) and without (0): identical records and statistics,
    tallies equal up to summation order."""
    import numpy as np
    from paper_2304_06226_amd.tuning import TUNED
    n = 200_000
    prob = {"sample": W.biased_sample, "vessel": W.vessel_sample, "void": _void_problem}[workload](n)
    tun = TUNED["sample" if workload == "sample" else "vessel"]
    base = ctx.get_tuning()
    out = {}
    try:
        for v in (1, 0):
            print(f"[case] {workload} {precision} vacuum_steps={v}", flush=True)
            ctx.set_tuning(**{**tun, "vacuum_steps": v})
            out[v] = gpu_run(ctx, prob, first=0, n=n, precision=precision)
    finally:
        ctx.set_tuning(**base)
    (r1, rec1, st1), (r0, rec0, st0) = out[1], out[0]
    for k in rec0.dtype.names:
        diff = int((rec1[k] != rec0[k]).reshape(n, -1).any(axis=1).sum())
        assert diff == 0, (k, diff)
    assert st1 == st0
    for (a, a2, an), (b, b2, bn) in zip(r1, r0):
        assert an == bn == n
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(a2, b2, rtol=1e-12, atol=1e-300)


def _pencil_problem(offset, n):
    """The biased sample cylinder alone in a vacuum sphere, hit (offset 0) or missed
    (offset 40 mm) by a 1.8 A pencil beam; a time-of-flight tally of the unscattered
    escapes checks the clock of the copied first step."""
    prob = W.biased_sample(n)
    prob.source = W.Source("pencil", origin=(offset, 0.0, -100.0), direction=(0.0, 0.0, 1.0), spectrum="mono",
                           lam0=1.8)
    prob.tallies = [prob.tallies[0],
                    W.Tally(trigger="escape", filter="unscattered", axes=[W.Axis("tof", 0.0, 0.005, 100)]),
                    prob.tallies[2]]
    prob.name = f"pencil-{offset:g}"
    return prob


@pytest.mark.parametrize("precision", ["fp32", "fp64_persistent"])
@pytest.mark.parametrize("offset", [0.0, 40.0])
def test_pencil_newborns_without_records(ctx, offset, precision):
    """Runs without records start the newborns of a one-wavelength pencil beam in
    vacuum from the state of the wave's first newborn after its first step (all
    of them draw nothing until then); runs with records take every step.  The
    same ids with vacuum_steps 1 and 0, and with and without records: equal
    statistics, tallies equal up to summation order."""
    import numpy as np
    from paper_2304_06226_amd.tuning import TUNED
    n = 500_000
    prob = _pencil_problem(offset, n)
    base = ctx.get_tuning()
    runs = []
    try:
        for v, rec in ((1, False), (0, False), (1, True)):
            print(f"[case] {prob.name} {precision} vacuum_steps={v} records={rec}", flush=True)
            ctx.set_tuning(**{**TUNED["sample"], "vacuum_steps": v})
            res, _, st = gpu_run(ctx, prob, first=0, n=n, precision=precision, records=rec)
            runs.append((res, st))
    finally:
        ctx.set_tuning(**base)
    (r1, st1) = runs[0]
    assert st1["histories"] == n
    assert (st1["escaped"] == n) == (offset != 0.0)
    for r, st in runs[1:]:
        assert st == st1
        for (a, a2, an), (b, b2, bn) in zip(r1, r):
            assert an == bn == n
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-300)
            np.testing.assert_allclose(a2, b2, rtol=1e-12, atol=1e-300)


def test_void_scene_fp64_persistent_elementwise(ctx):
    """The sample-with-void scene (fold passes in the persistent FP64 kernel) history
    by history against the oracle on the same ids."""
    n = 50_000
    prob = _void_problem(n)
    print(f"[case] {prob.name} fp64_persistent n={n}", flush=True)
    gres, grec, gst = gpu_run(ctx, prob, first=0, n=n, precision="fp64_persistent")
    ores = O.run(prob, first=0, n=n, threads=8, records=True)
    same = compare_records_fp64(grec, ores.records)
    compare_tallies_fp64(gres, ores, grec, ores.records, same)
    assert gst["histories"] == n
