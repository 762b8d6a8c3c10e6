"""The C-ABI library loads on a machine without a GPU, exports every function
declared in include/*.h, and validates descriptors (device-less context:
hip_device = -1) with the documented error codes."""
import ctypes as C
import subprocess
import dataclasses
import glob
import os
import re

import numpy as np
import pytest

from paper_2304_06226_amd import binding as B
from paper_2304_06226_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prompt_mi355x.h")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:int|void|const char\*)\s+\**(pr_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    lib = B.load()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def test_struct_sizes_match_header(tmp_path):
    """The binding's ctypes structs have the sizes and field offsets that a C
    compiler gives the header's structs."""
    structs = {"pr_material_desc": B.pr_material_desc, "pr_mirror_desc": B.pr_mirror_desc,
               "pr_chopper_desc": B.pr_chopper_desc, "pr_volume_desc": B.pr_volume_desc,
               "pr_source_desc": B.pr_source_desc, "pr_tally_axis": B.pr_tally_axis,
               "pr_tally_desc": B.pr_tally_desc, "pr_history_record": None, "pr_run_stats": B.pr_run_stats,
               "pr_sim": B.pr_sim, "pr_tuning": B.pr_tuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        if cls is not None:
            for f in cls._fields_:
                lines.append(f'  printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines.append('  return 0; }')
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for name, cls in structs.items():
        if cls is None:
            assert int(out[name]) == B.RECORD_DTYPE.itemsize == 96
            continue
        assert int(out[name]) == C.sizeof(cls), name
        for f in cls._fields_:
            assert int(out[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, (name, f[0])


@pytest.fixture
def ctx():
    c = B.Context(device=-1)
    yield c
    c.close()


def code_of(fn):
    with pytest.raises(B.PromptError) as e:
        fn()
    return e.value.code


def test_material_validation(ctx):
    m = W.sample_material()
    assert ctx.create_material(m) == 0
    assert code_of(lambda: ctx.create_material(dataclasses.replace(m, number_density=-1.0))) == -1
    assert code_of(lambda: ctx.create_material(dataclasses.replace(m, scatter_bias=-2.0))) == -1
    assert code_of(lambda: ctx.create_material(dataclasses.replace(m, d=m.d[::-1].copy()))) == -1
    assert code_of(lambda: ctx.create_material(dataclasses.replace(m, cell_volume=0.0))) == -1
    # a bias factor of 0 is allowed: it removes the process
    assert ctx.create_material(m.biased(abs_bias=0.0)) == 1


def test_geometry_validation(ctx):
    p = W.vessel_sample()
    ids = [ctx.create_material(m) for m in p.materials]
    assert ctx.create_geometry(p.volumes, ids) == 0
    # sample touching the vessel's bore
    bad = list(p.volumes)
    bad[2] = dataclasses.replace(bad[2], size=(10.0, 20.0))
    assert code_of(lambda: ctx.create_geometry(bad, ids)) == -3
    # daughter leaving the world
    bad = list(p.volumes)
    bad[2] = dataclasses.replace(bad[2], center=(0.0, 0.0, 995.0))
    assert code_of(lambda: ctx.create_geometry(bad, ids)) == -3
    # shell with r_in >= r_out, negative size, parent after child, unknown material
    assert code_of(lambda: ctx.create_geometry([p.volumes[0], dataclasses.replace(p.volumes[1], size=(11.0, 10.0, 40.0))], ids)) == -1
    assert code_of(lambda: ctx.create_geometry([p.volumes[0], dataclasses.replace(p.volumes[2], size=(-1.0, 20.0))], ids)) == -1
    assert code_of(lambda: ctx.create_geometry([p.volumes[0], dataclasses.replace(p.volumes[2], parent=1)], ids)) == -1
    assert code_of(lambda: ctx.create_geometry([p.volumes[0], dataclasses.replace(p.volumes[2], material=7)], [0, 1, 2, 3, 4, 5, 6, 99])) == -2
    # world must have parent -1
    assert code_of(lambda: ctx.create_geometry([dataclasses.replace(p.volumes[0], parent=0)], ids)) == -1
    # overlapping boxes
    world = W.Volume("box", (0, 0, 0), (100, 100, 100))
    a = W.Volume("box", (0, 0, 0), (10, 10, 10), parent=0)
    b = W.Volume("box", (9, 0, 0), (10, 10, 10), parent=0)
    c = W.Volume("box", (20, 0, 0), (10, 10, 10), parent=0)
    assert code_of(lambda: ctx.create_geometry([world, a, b], [])) == -3
    assert ctx.create_geometry([world, a, c], []) >= 0


def test_source_and_tally_validation(ctx):
    s = W.m3_guide().source
    assert ctx.create_source(s) == 0
    assert code_of(lambda: ctx.create_source(dataclasses.replace(s, direction=(0.0, 1.0, 1.0)))) == -1
    assert code_of(lambda: ctx.create_source(dataclasses.replace(s, lam_lo=5.0, lam_hi=1.0))) == -1
    assert code_of(lambda: ctx.create_source(dataclasses.replace(s, direction=(0.0, 0.0, 0.0)))) == -1
    t = W.Tally(axes=[W.Axis("theta2", 0, 180, 1800)])
    assert ctx.create_tally(t) == 0
    assert ctx.tally_nbins(0) == 1800
    assert code_of(lambda: ctx.create_tally(W.Tally(axes=[W.Axis("theta2", 10, 10, 5)]))) == -1
    assert code_of(lambda: ctx.create_tally(W.Tally(axes=[W.Axis("theta2", 0, 1, 0)]))) == -1
    assert code_of(lambda: ctx.tally_nbins(5)) == -2


def test_size_limits_are_enforced(ctx):
    """Each documented size limit is checked just beyond it (and accepted at it)."""
    # tally bins: at most 2^36 over all axes
    big = [W.Axis("x", 0, 1, 1024)] * 3
    assert code_of(lambda: ctx.create_tally(W.Tally(axes=big + [W.Axis("y", 0, 1, 65)]))) == -1
    # Bragg families: at most 1024
    m = W.sample_material()
    def families(k):
        d = np.linspace(3.0, 0.5, k)
        return dataclasses.replace(m, d=d, mult=np.full(k, 6, dtype=np.int32), f2=np.full(k, 2.0))
    assert ctx.create_material(families(1024)) >= 0
    assert code_of(lambda: ctx.create_material(families(1025))) == -1
    # tables: 2..4096 rows
    def table(k):
        lam = np.linspace(0.5, 10.0, k)
        return dataclasses.replace(m, table_lambda=lam, table_sigma_abs=np.ones(k), table_sigma_inc=np.ones(k))
    assert ctx.create_material(table(4096)) >= 0
    assert code_of(lambda: ctx.create_material(table(4097))) == -1
    assert code_of(lambda: ctx.create_material(table(1))) == -1
    # geometry: at least one volume
    assert code_of(lambda: ctx.create_geometry([], [])) == -1
    # batches: at least one simulation
    assert code_of(lambda: ctx.run_batch([], stream=0)) == -1


def test_run_needs_a_device(ctx):
    """Every precision policy passes argument checks and then needs the device;
    an unknown policy is rejected first."""
    p = W.analog_sample()
    sim = B.Simulation(ctx, p)
    for prec in ("fp64", "fp32", "fp64_persistent"):
        with pytest.raises(B.PromptError) as e:
            ctx.run(sim.geom, sim.src, sim.tallies, 0, 10, prec, None, 0)
        assert e.value.code == -5
    assert code_of(lambda: ctx.run(sim.geom, sim.src, sim.tallies, 0, 10, 3, None, 0)) == -1


def test_tuning_validation(ctx):
    t = ctx.get_tuning()
    assert t["block"] == 256 and t["chunk"] >= 1
    assert code_of(lambda: ctx.set_tuning(block=1088)) == -1
    assert code_of(lambda: ctx.set_tuning(block=100)) == -1
    assert code_of(lambda: ctx.set_tuning(bin_cache_slots=1000)) == -1
    assert code_of(lambda: ctx.set_tuning(refill_threshold=0)) == -1
    assert code_of(lambda: ctx.set_tuning(waves_per_simd=3)) == -1
    assert code_of(lambda: ctx.set_tuning(vacuum_steps=2)) == -1
    assert t["vacuum_steps"] == 1
    ctx.set_tuning(vacuum_steps=0)
    assert ctx.get_tuning()["vacuum_steps"] == 0
    ctx.set_tuning(vacuum_steps=1)
    assert code_of(lambda: ctx.set_tuning(grid_chunk=-1)) == -1
    assert code_of(lambda: ctx.set_tuning(grid_chunk=(1 << 20) + 1)) == -1
    ctx.set_tuning(grid_chunk=128)
    assert ctx.get_tuning()["grid_chunk"] == 128
    ctx.set_tuning(grid_chunk=0)
    ctx.set_tuning(refill_threshold=8, waves_per_simd=5)
    assert ctx.get_tuning()["refill_threshold"] == 8 and ctx.get_tuning()["waves_per_simd"] == 5
    ctx.set_tuning(waves_per_simd=0)
    assert ctx.get_tuning()["waves_per_simd"] == 4


def test_stored_tunings_are_valid(ctx):
    """Every stored launch tuning (both persistent policies) is accepted as is."""
    from paper_2304_06226_amd.tuning import TUNED, TUNED_FP64_PERSISTENT
    for table in (TUNED, TUNED_FP64_PERSISTENT):
        for name, t in table.items():
            ctx.set_tuning(**t)
            assert ctx.get_tuning() == t, name


def test_prepared_batch_validation(ctx):
    p = W.analog_sample()
    sim = B.Simulation(ctx, p)
    desc = [(sim.geom, sim.src, sim.tallies, 0, 1000)]
    # a validation-only context has no device to hold a prepared batch
    assert code_of(lambda: ctx.prepare_batch(desc, stride=1000)) == -5
    assert code_of(lambda: ctx.prepare_batch(desc, stride=1000, precision="fp64")) == -1
    assert code_of(lambda: ctx.prepare_batch([], stride=1000)) == -1
    assert code_of(lambda: ctx.run_prepared(0, stream=0)) == -2
    assert code_of(lambda: ctx.release_batch(3)) == -2


def test_boundary_sizes_and_rejections(ctx):
    """pr_workspace_size and pr_tally_storage_size answer without a device; the
    Kahan accumulator is rejected; first-collision tallies are refused by the FP32
    policy before any device work; caller tally storage is size-checked."""
    for prec in ("fp64", "fp32", "fp64_persistent"):
        assert ctx.workspace_size(prec) == 256
    assert code_of(lambda: ctx.workspace_size(7)) == -1
    t = W.Tally(axes=[W.Axis("theta2", 0, 180, 1800), W.Axis("lambda", 0.5, 5, 100)])
    assert ctx.tally_storage_size(t) == 2 * 1800 * 100 * 8
    assert code_of(lambda: ctx.create_tally(dataclasses.replace(t, accumulator="kahan_fp32"))) == -1
    assert code_of(lambda: ctx.tally_storage_size(dataclasses.replace(t, accumulator="kahan_fp32"))) == -1
    p = W.analog_sample()
    p.tallies = [W.Tally(trigger="first_collision")]
    sim = B.Simulation(ctx, p)
    assert code_of(lambda: ctx.run(sim.geom, sim.src, sim.tallies, 0, 10, "fp32", None, 0)) == -1
    for prec in ("fp64", "fp64_persistent"):
        assert code_of(lambda: ctx.run(sim.geom, sim.src, sim.tallies, 0, 10, prec, None, 0)) == -5
    d = B.tally_desc(t)
    i = C.c_int32()
    assert ctx.lib.pr_create_tally_in(ctx.h, C.byref(d), C.c_void_p(4096), 1000, C.byref(i)) == B.PR_EWORKSPACE
    assert ctx.lib.pr_create_tally_in(ctx.h, C.byref(d), C.c_void_p(4096), 1 << 22, C.byref(i)) == -5
    assert ctx.lib.pr_create_tally_in(ctx.h, C.byref(d), None, 1 << 22, C.byref(i)) == -1
