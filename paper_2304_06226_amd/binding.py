"""Thin ctypes binding of libprompt_mi355x.so (argument marshalling only).

Every step of the history loop runs in the library's HIP kernels; this module
only converts the neutral workload description into the C-ABI structures of
include/prompt_mi355x.h and passes device pointers and the current HIP stream.
It fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprompt_mi355x.so")

PR_OK = 0
PR_EWORKSPACE = -4
PR_ECAPPED = -7
PR_FP64_PLAIN, PR_FP32_MIXED, PR_FP64_PERSISTENT = 0, 1, 2
PRECISION = {"fp64": PR_FP64_PLAIN, "fp64_plain": PR_FP64_PLAIN, "fp32": PR_FP32_MIXED, "fp32_mixed": PR_FP32_MIXED,
             "fp64_persistent": PR_FP64_PERSISTENT}

SOLID = {"box": 0, "cylinder": 1, "cyl_shell": 2, "sphere": 3, "sph_shell": 4}
SOURCE = {"pencil": 0, "rect": 1, "rect_divergent": 2, "moderator": 3}
SPECTRUM = {"mono": 0, "uniform": 1, "maxwell": 2}
TRIGGER = {"escape": 0, "absorb": 1, "detect": 2, "first_collision": 3}
FILTER = {"all": 0, "unscattered": 1, "scattered": 2, "nscat_eq": 3}
QUANTITY = {"theta2": 0, "lambda": 1, "x": 2, "y": 3, "z": 4, "div_x": 5, "div_y": 6, "nscat": 7, "q": 8, "tof": 9}
MIRROR = {"linear": 0, "tanh": 1}
ACCUMULATOR = {"fp64": 0, "kahan_fp32": 1}

END_ESCAPE, END_ABSORB, END_KILL, END_DETECT, END_CAPPED, END_OUTSIDE = 1, 2, 3, 4, 5, 6

# pr_history_record (96 bytes)
RECORD_DTYPE = np.dtype([("hash", "<u8"), ("w", "<f8"), ("pos", "<f8", 3), ("dir", "<f8", 3),
                         ("lambda", "<f8"), ("term", "<i4"), ("n_scat", "<i4"), ("n_steps", "<i4"),
                         ("n_draws", "<i4"), ("region", "<i4"), ("tof", "<f4")])
RECORD_BYTES = 96

EXPORTS = ["pr_init", "pr_destroy", "pr_last_error", "pr_set_seed", "pr_create_material", "pr_create_geometry",
           "pr_create_source", "pr_create_tally", "pr_tally_storage_size", "pr_create_tally_in", "pr_tally_nbins",
           "pr_workspace_size", "pr_run_histories", "pr_read_tally", "pr_read_tally_range", "pr_reset_tally",
           "pr_read_stats", "pr_reset_stats", "pr_set_tuning", "pr_get_tuning", "pr_run_batch", "pr_autotune",
           "pr_prepare_batch", "pr_run_prepared", "pr_release_batch", "pr_run_batch_static"]


class pr_material_desc(C.Structure):
    _fields_ = [("number_density", C.c_double), ("sigma_inc", C.c_double), ("sigma_abs_ref", C.c_double),
                ("scatter_bias", C.c_double), ("abs_bias", C.c_double), ("cell_volume", C.c_double),
                ("atoms_per_cell", C.c_int32), ("n_families", C.c_int32), ("d", C.POINTER(C.c_double)),
                ("mult", C.POINTER(C.c_int32)), ("f2", C.POINTER(C.c_double)), ("n_table", C.c_int32),
                ("table_pad", C.c_int32), ("table_lambda", C.POINTER(C.c_double)),
                ("table_sigma_abs", C.POINTER(C.c_double)), ("table_sigma_inc", C.POINTER(C.c_double))]


class pr_mirror_desc(C.Structure):
    _fields_ = [("model", C.c_int32), ("pad", C.c_int32), ("R0", C.c_double), ("Qc", C.c_double),
                ("alpha", C.c_double), ("m", C.c_double), ("W", C.c_double)]


class pr_chopper_desc(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad", C.c_int32), ("r", C.c_double), ("rot_freq", C.c_double),
                ("theta0", C.c_double), ("phase", C.c_double)]


class pr_volume_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("axis", C.c_int32), ("parent", C.c_int32), ("material", C.c_int32),
                ("is_detector", C.c_int32), ("mirror_mask", C.c_int32), ("center", C.c_double * 3),
                ("size", C.c_double * 3), ("mirror", pr_mirror_desc), ("chopper", pr_chopper_desc)]


class pr_source_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("spectrum", C.c_int32), ("origin", C.c_double * 3), ("dir", C.c_double * 3),
                ("size", C.c_double * 2), ("div_deg", C.c_double * 2), ("lam0", C.c_double), ("lam_lo", C.c_double),
                ("lam_hi", C.c_double), ("kT", C.c_double), ("slit_center", C.c_double * 3),
                ("slit_size", C.c_double * 2)]


class pr_tally_axis(C.Structure):
    _fields_ = [("quantity", C.c_int32), ("nbins", C.c_int32), ("lo", C.c_double), ("hi", C.c_double)]


class pr_tally_desc(C.Structure):
    _fields_ = [("trigger", C.c_int32), ("trigger_volume", C.c_int32), ("filter", C.c_int32),
                ("filter_arg", C.c_int32), ("naxes", C.c_int32), ("accumulator", C.c_int32),
                ("axes", pr_tally_axis * 4), ("beam", C.c_double * 3)]


class pr_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32), ("refill_threshold", C.c_int32),
                ("lds_tally_bytes", C.c_int32), ("bin_cache_slots", C.c_int32), ("chunk", C.c_int32),
                ("waves_per_simd", C.c_int32), ("grid_chunk", C.c_int32), ("grid_walk_cells", C.c_int32),
                ("vacuum_steps", C.c_int32)]


class pr_sim(C.Structure):
    _fields_ = [("geom", C.c_int32), ("src", C.c_int32), ("n_tallies", C.c_int32), ("tallies", C.c_int32 * 8),
                ("pad", C.c_int32), ("first_history", C.c_uint64), ("n", C.c_uint64)]


class pr_run_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("histories", "escaped", "absorbed", "killed", "detected", "capped",
                                          "outside", "steps", "draws", "scatters")]


_lib = None


def load():
    """Load the built library; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run paper_2304_06226_amd.build.build_library() "
                           "(the history loop only runs in the HIP library)")
    L = C.CDLL(LIB_PATH)
    vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
    L.pr_init.argtypes = [C.POINTER(vp), C.c_int, u64]
    L.pr_destroy.argtypes = [vp]
    L.pr_destroy.restype = None
    L.pr_last_error.argtypes = [vp]
    L.pr_last_error.restype = C.c_char_p
    L.pr_set_seed.argtypes = [vp, u64]
    L.pr_create_material.argtypes = [vp, C.POINTER(pr_material_desc), C.POINTER(i32)]
    L.pr_create_geometry.argtypes = [vp, C.POINTER(pr_volume_desc), i32, C.POINTER(i32)]
    L.pr_create_source.argtypes = [vp, C.POINTER(pr_source_desc), C.POINTER(i32)]
    L.pr_create_tally.argtypes = [vp, C.POINTER(pr_tally_desc), C.POINTER(i32)]
    L.pr_tally_storage_size.argtypes = [vp, C.POINTER(pr_tally_desc), C.POINTER(C.c_size_t)]
    L.pr_create_tally_in.argtypes = [vp, C.POINTER(pr_tally_desc), vp, C.c_size_t, C.POINTER(i32)]
    L.pr_tally_nbins.argtypes = [vp, i32, C.POINTER(u64)]
    L.pr_workspace_size.argtypes = [vp, i32, C.POINTER(C.c_size_t)]
    L.pr_run_histories.argtypes = [vp, i32, i32, C.POINTER(i32), i32, u64, u64, i32, vp, vp, C.c_size_t, vp]
    L.pr_read_tally.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(u64), C.c_size_t, vp]
    L.pr_read_tally_range.argtypes = [vp, i32, u64, u64, C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
    L.pr_reset_tally.argtypes = [vp, i32, vp]
    L.pr_read_stats.argtypes = [vp, C.POINTER(pr_run_stats), vp]
    L.pr_reset_stats.argtypes = [vp, vp]
    L.pr_set_tuning.argtypes = [vp, C.POINTER(pr_tuning)]
    L.pr_run_batch.argtypes = [vp, C.POINTER(pr_sim), i32, i32, vp]
    L.pr_run_batch_static.argtypes = [vp, C.POINTER(pr_sim), i32, i32, vp]
    L.pr_autotune.argtypes = [vp, C.POINTER(pr_sim), i32, C.c_double, C.POINTER(pr_tuning), vp]
    L.pr_get_tuning.argtypes = [vp, C.POINTER(pr_tuning)]
    L.pr_prepare_batch.argtypes = [vp, C.POINTER(pr_sim), i32, i32, u64, C.POINTER(i32)]
    L.pr_run_prepared.argtypes = [vp, i32, vp]
    L.pr_release_batch.argtypes = [vp, i32]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("pr_destroy", "pr_last_error"):
            f.restype = C.c_int
    _lib = L
    return L


class PromptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"prompt_mi355x error {code}: {msg}")
        self.code = code


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def material_desc(m: W.Material, keep: list) -> pr_material_desc:
    d = np.ascontiguousarray(m.d, dtype=np.float64)
    mu = np.ascontiguousarray(m.mult, dtype=np.int32)
    f2 = np.ascontiguousarray(m.f2, dtype=np.float64)
    keep += [d, mu, f2]
    s = pr_material_desc()
    s.number_density, s.sigma_inc, s.sigma_abs_ref = m.number_density, m.sigma_inc, m.sigma_abs_ref
    s.scatter_bias, s.abs_bias, s.cell_volume = m.scatter_bias, m.abs_bias, m.cell_volume
    s.atoms_per_cell, s.n_families = m.atoms_per_cell, len(d)
    s.d = d.ctypes.data_as(C.POINTER(C.c_double))
    s.mult = mu.ctypes.data_as(C.POINTER(C.c_int32))
    s.f2 = f2.ctypes.data_as(C.POINTER(C.c_double))
    if m.table_lambda is not None:
        tl, ta, ti = (np.ascontiguousarray(a, dtype=np.float64)
                      for a in (m.table_lambda, m.table_sigma_abs, m.table_sigma_inc))
        keep += [tl, ta, ti]
        s.n_table = len(tl)
        s.table_lambda = tl.ctypes.data_as(C.POINTER(C.c_double))
        s.table_sigma_abs = ta.ctypes.data_as(C.POINTER(C.c_double))
        s.table_sigma_inc = ti.ctypes.data_as(C.POINTER(C.c_double))
    return s


def volume_desc(v: W.Volume, mat_ids: Sequence[int]) -> pr_volume_desc:
    s = pr_volume_desc()
    s.kind, s.axis, s.parent = SOLID[v.kind], v.axis, v.parent
    s.material = mat_ids[v.material] if v.material >= 0 else -1
    s.is_detector, s.mirror_mask = int(bool(v.detector)), v.mirror_mask
    for k in range(3):
        s.center[k] = v.center[k]
    for k, x in enumerate(v.size):
        s.size[k] = x
    if v.mirror is not None:
        mi = v.mirror
        s.mirror.model = MIRROR[mi.model]
        s.mirror.R0, s.mirror.Qc, s.mirror.alpha, s.mirror.m, s.mirror.W = mi.R0, mi.Qc, mi.alpha, mi.m, mi.W
    if v.chopper is not None:
        ch = v.chopper
        s.chopper.n, s.chopper.r, s.chopper.rot_freq = ch.n, ch.r, ch.rot_freq
        s.chopper.theta0, s.chopper.phase = ch.theta0, ch.phase
    return s


def source_desc(src: W.Source) -> pr_source_desc:
    s = pr_source_desc()
    s.kind, s.spectrum = SOURCE[src.kind], SPECTRUM[src.spectrum]
    for k in range(3):
        s.origin[k] = src.origin[k]
        s.dir[k] = src.direction[k]
    s.size[0], s.size[1] = src.size
    s.div_deg[0], s.div_deg[1] = src.divergence
    s.lam0, s.lam_lo, s.lam_hi, s.kT = src.lam0, src.lam_lo, src.lam_hi, src.kT
    for k in range(3):
        s.slit_center[k] = src.slit_center[k]
    s.slit_size[0], s.slit_size[1] = src.slit_size
    return s


def tally_desc(t: W.Tally) -> pr_tally_desc:
    s = pr_tally_desc()
    s.trigger, s.trigger_volume = TRIGGER[t.trigger], t.trigger_volume
    s.filter, s.filter_arg = FILTER[t.filter], t.filter_arg
    s.naxes, s.accumulator = len(t.axes), ACCUMULATOR[t.accumulator]
    for i, a in enumerate(t.axes):
        s.axes[i].quantity, s.axes[i].nbins, s.axes[i].lo, s.axes[i].hi = QUANTITY[a.quantity], a.nbins, a.lo, a.hi
    for k in range(3):
        s.beam[k] = t.beam[k]
    return s


class Context:
    """A library context on one HIP device (device=-1: validation only, no GPU)."""

    def __init__(self, device: int = 0, seed: int = 4096):
        self.lib = load()
        self.h = C.c_void_p()
        rc = self.lib.pr_init(C.byref(self.h), device, seed)
        if rc != PR_OK:
            raise PromptError(rc, f"pr_init(device={device}) failed")
        self.device = device

    def close(self):
        if self.h:
            self.lib.pr_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != PR_OK:
            raise PromptError(rc, self.lib.pr_last_error(self.h).decode())
        return rc

    def set_seed(self, seed: int):
        self._check(self.lib.pr_set_seed(self.h, seed))

    def create_material(self, m: W.Material) -> int:
        keep: list = []
        d = material_desc(m, keep)
        i = C.c_int32()
        self._check(self.lib.pr_create_material(self.h, C.byref(d), C.byref(i)))
        return i.value

    def create_geometry(self, vols: List[W.Volume], mat_ids: Sequence[int]) -> int:
        arr = (pr_volume_desc * len(vols))(*[volume_desc(v, mat_ids) for v in vols])
        i = C.c_int32()
        self._check(self.lib.pr_create_geometry(self.h, arr, len(vols), C.byref(i)))
        return i.value

    def create_source(self, s: W.Source) -> int:
        d = source_desc(s)
        i = C.c_int32()
        self._check(self.lib.pr_create_source(self.h, C.byref(d), C.byref(i)))
        return i.value

    def create_tally(self, t: W.Tally, storage=None) -> int:
        """storage: None (the library allocates), or a caller-owned CUDA tensor of at
        least tally_storage_size(t) bytes that holds the tally's (sum w, sum w^2) pairs."""
        d = tally_desc(t)
        i = C.c_int32()
        if storage is None:
            self._check(self.lib.pr_create_tally(self.h, C.byref(d), C.byref(i)))
        else:
            nbytes = storage.numel() * storage.element_size()
            self._check(self.lib.pr_create_tally_in(self.h, C.byref(d), C.c_void_p(storage.data_ptr()), nbytes,
                                                    C.byref(i)))
        return i.value

    def tally_storage_size(self, t: W.Tally) -> int:
        d = tally_desc(t)
        n = C.c_size_t()
        self._check(self.lib.pr_tally_storage_size(self.h, C.byref(d), C.byref(n)))
        return n.value

    def workspace_size(self, precision="fp32") -> int:
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        n = C.c_size_t()
        self._check(self.lib.pr_workspace_size(self.h, prec, C.byref(n)))
        return n.value

    def tally_nbins(self, t: int) -> int:
        n = C.c_uint64()
        self._check(self.lib.pr_tally_nbins(self.h, t, C.byref(n)))
        return n.value

    def run(self, geom: int, src: int, tallies: Sequence[int], first: int, n: int, precision="fp64",
            records_ptr: Optional[int] = None, stream=None, workspace=None):
        """workspace: None (a slot of the context's counter ring) or a caller-owned
        CUDA tensor of at least workspace_size() bytes."""
        ts = (C.c_int32 * max(1, len(tallies)))(*tallies)
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        st = _current_stream() if stream is None else C.c_void_p(stream)
        ws, wsb = None, 0
        if workspace is not None:
            ws, wsb = C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
        self._check(self.lib.pr_run_histories(self.h, geom, src, ts, len(tallies), first, n, prec,
                                              C.c_void_p(records_ptr) if records_ptr else None, ws, wsb, st))

    def read_tally(self, t: int, stream=None):
        nb = self.tally_nbins(t)
        sw = np.zeros(nb, dtype=np.float64)
        sw2 = np.zeros(nb, dtype=np.float64)
        nh = C.c_uint64()
        st = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(self.lib.pr_read_tally(self.h, t, sw.ctypes.data_as(C.POINTER(C.c_double)),
                                           sw2.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nh), nb, st))
        return sw, sw2, nh.value

    def read_tally_range(self, t: int, offset: int, count: int, stream=None):
        sw = np.zeros(count, dtype=np.float64)
        sw2 = np.zeros(count, dtype=np.float64)
        st = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(self.lib.pr_read_tally_range(self.h, t, offset, count, sw.ctypes.data_as(C.POINTER(C.c_double)),
                                                 sw2.ctypes.data_as(C.POINTER(C.c_double)), st))
        return sw, sw2

    def reset_tally(self, t: int, stream=None):
        st = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(self.lib.pr_reset_tally(self.h, t, st))

    def read_stats(self, stream=None) -> dict:
        """Run statistics since the last reset (PR_ECAPPED, returned when some history
        reached the step cap, is not an error here: out["capped"] says so)."""
        s = pr_run_stats()
        st = _current_stream() if stream is None else C.c_void_p(stream)
        rc = self.lib.pr_read_stats(self.h, C.byref(s), st)
        if rc != PR_ECAPPED:
            self._check(rc)
        return {name: getattr(s, name) for name, _ in pr_run_stats._fields_}

    @staticmethod
    def _sims(sims):
        arr = (pr_sim * len(sims))()
        for i, (g, sr, ts, first, n) in enumerate(sims):
            arr[i].geom, arr[i].src, arr[i].n_tallies = g, sr, len(ts)
            for j, t in enumerate(ts):
                arr[i].tallies[j] = t
            arr[i].first_history, arr[i].n = first, n
        return arr

    def autotune(self, sims, sample_fraction=0.1, stream=None) -> dict:
        """Measure and set the launch tuning for a workload (list of (geom, src, tallies, first, n))."""
        arr = self._sims(sims)
        t = pr_tuning()
        st = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(self.lib.pr_autotune(self.h, arr, len(sims), sample_fraction, C.byref(t), st))
        return {name: getattr(t, name) for name, _ in pr_tuning._fields_}

    def run_batch(self, sims, precision="fp32", stream=None):
        """sims: list of (geom, src, tallies, first, n)."""
        arr = self._sims(sims)
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        st = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(self.lib.pr_run_batch(self.h, arr, len(sims), prec, st))

    def run_batch_static(self, sims, precision="fp32", stream=None):
        """As run_batch, with descriptors and counters in the library's fixed device
        scratch (no device allocation; overlapping calls on one GPU race)."""
        arr = self._sims(sims)
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        st = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(self.lib.pr_run_batch_static(self.h, arr, len(sims), prec, st))

    def prepare_batch(self, sims, stride, precision="fp32") -> int:
        """Upload a batch once (sims as for run_batch); each run_prepared advances its ids by stride."""
        arr = self._sims(sims)
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        out = C.c_int32()
        self._check(self.lib.pr_prepare_batch(self.h, arr, len(sims), prec, stride, C.byref(out)))
        return out.value

    def run_prepared(self, batch: int, stream=None):
        st = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(self.lib.pr_run_prepared(self.h, batch, st))

    def release_batch(self, batch: int):
        self._check(self.lib.pr_release_batch(self.h, batch))

    def get_tuning(self) -> dict:
        t = pr_tuning()
        self._check(self.lib.pr_get_tuning(self.h, C.byref(t)))
        return {name: getattr(t, name) for name, _ in pr_tuning._fields_}

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = pr_tuning(**cur)
        self._check(self.lib.pr_set_tuning(self.h, C.byref(t)))

    def reset_stats(self, stream=None):
        st = _current_stream() if stream is None else C.c_void_p(stream)
        self._check(self.lib.pr_reset_stats(self.h, st))


class Simulation:
    """A workload instantiated in a context: materials, geometry, source, tallies."""

    def __init__(self, ctx: Context, prob: W.Problem):
        self.ctx = ctx
        self.prob = prob
        self.mat_ids = [ctx.create_material(m) for m in prob.materials]
        self.geom = ctx.create_geometry(prob.volumes, self.mat_ids)
        self.src = ctx.create_source(prob.source)
        self.tallies = [ctx.create_tally(t) for t in prob.tallies]

    def run(self, first: int = 0, n: Optional[int] = None, precision="fp64", records=None, stream=None,
            workspace=None):
        """records: None or a torch uint8 CUDA tensor of n * 96 bytes; workspace: None or
        a caller-owned CUDA tensor of Context.workspace_size() bytes."""
        if n is None:
            n = self.prob.n_histories
        ptr = None
        if records is not None:
            if records.numel() < n * RECORD_BYTES or not records.is_cuda:
                raise ValueError("records must be a CUDA uint8 tensor of n * 96 bytes")
            ptr = records.data_ptr()
        self.ctx.run(self.geom, self.src, self.tallies, first, n, precision, ptr, stream, workspace)

    def reset(self):
        for t in self.tallies:
            self.ctx.reset_tally(t)

    def results(self):
        out = []
        for t in self.tallies:
            out.append(self.ctx.read_tally(t))
        return out


def records_to_numpy(records, n: int) -> np.ndarray:
    """Copy a device record buffer (torch uint8 tensor) to a structured numpy array."""
    host = records[: n * RECORD_BYTES].cpu().numpy()
    return host.view(RECORD_DTYPE)


class BatchRun:
    """A batch of workloads instantiated in one context; simulation i covers the
    history ids [offset_i, offset_i + n_i) with consecutive offsets, so the
    random-number streams of different simulations are disjoint."""

    def __init__(self, ctx: Context, batch: "W.Batch", base: int = 0):
        self.ctx = ctx
        self.batch = batch
        self.sims = [Simulation(ctx, p) for p in batch.problems]
        self.offsets = []
        off = base
        for p in batch.problems:
            self.offsets.append(off)
            off += p.n_histories
        self.span = off - base

    def descriptors(self, shift: int = 0):
        return [(s.geom, s.src, s.tallies, o + shift, s.prob.n_histories) for s, o in zip(self.sims, self.offsets)]

    def run(self, shift: int = 0, stream=None):
        self.ctx.run_batch(self.descriptors(shift), "fp32", stream)

    def reset(self):
        for s in self.sims:
            s.reset()
