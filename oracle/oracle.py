"""ctypes wrapper of the plain FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg.  It translates the neutral workload description
(paper_2304_06226_amd.workloads) into the oracle's own C structures; it imports
nothing from the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

SOLID = {"box": 0, "cylinder": 1, "cyl_shell": 2, "sphere": 3, "sph_shell": 4}
SOURCE = {"pencil": 0, "rect": 1, "rect_divergent": 2, "moderator": 3}
SPECTRUM = {"mono": 0, "uniform": 1, "maxwell": 2}
TRIGGER = {"escape": 0, "absorb": 1, "detect": 2, "first_collision": 3}
FILTER = {"all": 0, "unscattered": 1, "scattered": 2, "nscat_eq": 3}
QUANTITY = {"theta2": 0, "lambda": 1, "x": 2, "y": 3, "z": 4, "div_x": 5, "div_y": 6, "nscat": 7, "q": 8, "tof": 9}
MIRROR = {"linear": 0, "tanh": 1}

END_ESCAPE, END_ABSORB, END_KILL, END_DETECT, END_CAPPED, END_OUTSIDE = 1, 2, 3, 4, 5, 6

# per-history record as laid out by orc_record (96 bytes)
RECORD_DTYPE = np.dtype([("hash", "<u8"), ("w", "<f8"), ("pos", "<f8", 3), ("dir", "<f8", 3),
                         ("lambda", "<f8"), ("term", "<i4"), ("n_scat", "<i4"), ("n_steps", "<i4"),
                         ("n_draws", "<i4"), ("region", "<i4"), ("tof", "<f4")])
assert RECORD_DTYPE.itemsize == 96


class orc_material(C.Structure):
    _fields_ = [("number_density", C.c_double), ("sigma_inc", C.c_double), ("sigma_abs_ref", C.c_double),
                ("scatter_bias", C.c_double), ("abs_bias", C.c_double), ("cell_volume", C.c_double),
                ("atoms_per_cell", C.c_int32), ("n_families", C.c_int32),
                ("d", C.POINTER(C.c_double)), ("mult", C.POINTER(C.c_int32)), ("f2", C.POINTER(C.c_double)),
                ("n_table", C.c_int32), ("table_pad", C.c_int32), ("table_lambda", C.POINTER(C.c_double)),
                ("table_sigma_abs", C.POINTER(C.c_double)), ("table_sigma_inc", C.POINTER(C.c_double))]


class orc_volume(C.Structure):
    _fields_ = [("kind", C.c_int32), ("axis", C.c_int32), ("parent", C.c_int32), ("material", C.c_int32),
                ("is_detector", C.c_int32), ("mirror_mask", C.c_int32),
                ("center", C.c_double * 3), ("size", C.c_double * 3),
                ("mirror_model", C.c_int32), ("pad", C.c_int32),
                ("R0", C.c_double), ("Qc", C.c_double), ("alpha", C.c_double), ("m", C.c_double), ("W", C.c_double),
                ("chop_n", C.c_int32), ("chop_pad", C.c_int32), ("chop_r", C.c_double), ("chop_freq", C.c_double),
                ("chop_theta0", C.c_double), ("chop_phase", C.c_double)]


class orc_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("spectrum", C.c_int32), ("origin", C.c_double * 3), ("dir", C.c_double * 3),
                ("size", C.c_double * 2), ("div_deg", C.c_double * 2), ("lam0", C.c_double),
                ("lam_lo", C.c_double), ("lam_hi", C.c_double), ("kT", C.c_double),
                ("slit_center", C.c_double * 3), ("slit_size", C.c_double * 2)]


class orc_tally(C.Structure):
    _fields_ = [("trigger", C.c_int32), ("trigger_volume", C.c_int32), ("filter", C.c_int32),
                ("filter_arg", C.c_int32), ("naxes", C.c_int32), ("quantity", C.c_int32 * 4),
                ("nbins", C.c_int32 * 4), ("pad", C.c_int32), ("lo", C.c_double * 4), ("hi", C.c_double * 4),
                ("beam", C.c_double * 3)]


class orc_problem(C.Structure):
    _fields_ = [("n_materials", C.c_int32), ("n_volumes", C.c_int32), ("n_tallies", C.c_int32), ("pad", C.c_int32),
                ("materials", C.POINTER(orc_material)), ("volumes", C.POINTER(orc_volume)),
                ("source", C.POINTER(orc_source)), ("tallies", C.POINTER(orc_tally))]


class orc_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("histories", "escaped", "absorbed", "killed", "detected", "capped",
                                          "outside", "steps", "draws")]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, no GPU)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", LIB_PATH, SRC_PATH, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        L.orc_run.argtypes = [C.POINTER(orc_problem), C.c_uint64, C.c_uint64, C.c_uint64, C.c_int,
                              C.POINTER(C.POINTER(C.c_double)), C.POINTER(C.POINTER(C.c_double)),
                              C.c_void_p, C.POINTER(orc_stats)]
        L.orc_run.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_philox4x32_10.restype = None
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_intervals.argtypes = [C.POINTER(orc_volume), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_intervals.restype = C.c_int
        L.orc_contains.argtypes = [C.POINTER(orc_volume), C.POINTER(C.c_double)]
        L.orc_contains.restype = C.c_int
        L.orc_macro_xs.argtypes = [C.POINTER(orc_material), C.c_double, C.POINTER(C.c_double)]
        L.orc_macro_xs.restype = None
        L.orc_mirror_reflectivity.argtypes = [C.POINTER(orc_volume), C.c_double]
        L.orc_mirror_reflectivity.restype = C.c_double
        L.orc_ev_from_angstrom.argtypes = [C.c_double]
        L.orc_ev_from_angstrom.restype = C.c_double
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# translation of the neutral workload description
# --------------------------------------------------------------------------

class _Keep:
    """Holds the numpy arrays the C structures point into."""

    def __init__(self):
        self.arrays = []

    def dptr(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.arrays.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    def iptr(self, a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        self.arrays.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_int32))


def make_material(m, keep: _Keep) -> orc_material:
    s = orc_material()
    s.number_density = m.number_density
    s.sigma_inc = m.sigma_inc
    s.sigma_abs_ref = m.sigma_abs_ref
    s.scatter_bias = m.scatter_bias
    s.abs_bias = m.abs_bias
    s.cell_volume = m.cell_volume
    s.atoms_per_cell = m.atoms_per_cell
    s.n_families = len(m.d)
    s.d = keep.dptr(m.d)
    s.mult = keep.iptr(m.mult)
    s.f2 = keep.dptr(m.f2)
    if m.table_lambda is not None:
        s.n_table = len(m.table_lambda)
        s.table_lambda = keep.dptr(m.table_lambda)
        s.table_sigma_abs = keep.dptr(m.table_sigma_abs)
        s.table_sigma_inc = keep.dptr(m.table_sigma_inc)
    return s


def make_volume(v) -> orc_volume:
    s = orc_volume()
    s.kind = SOLID[v.kind]
    s.axis = v.axis
    s.parent = v.parent
    s.material = v.material
    s.is_detector = 1 if v.detector else 0
    s.mirror_mask = v.mirror_mask
    for k in range(3):
        s.center[k] = v.center[k]
    for k, x in enumerate(v.size):
        s.size[k] = x
    mir = v.mirror
    if mir is not None:
        s.mirror_model = MIRROR[mir.model]
        s.R0, s.Qc, s.alpha, s.m, s.W = mir.R0, mir.Qc, mir.alpha, mir.m, mir.W
    ch = getattr(v, "chopper", None)
    if ch is not None:
        s.chop_n, s.chop_r, s.chop_freq, s.chop_theta0, s.chop_phase = ch.n, ch.r, ch.rot_freq, ch.theta0, ch.phase
    return s


def make_source(src) -> orc_source:
    s = orc_source()
    s.kind = SOURCE[src.kind]
    s.spectrum = SPECTRUM[src.spectrum]
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


def make_tally(t) -> orc_tally:
    s = orc_tally()
    s.trigger = TRIGGER[t.trigger]
    s.trigger_volume = t.trigger_volume
    s.filter = FILTER[t.filter]
    s.filter_arg = t.filter_arg
    s.naxes = len(t.axes)
    for i, a in enumerate(t.axes):
        s.quantity[i] = QUANTITY[a.quantity]
        s.lo[i] = a.lo
        s.hi[i] = a.hi
        s.nbins[i] = a.nbins
    for k in range(3):
        s.beam[k] = t.beam[k]
    return s


class CProblem:
    def __init__(self, prob):
        self.keep = _Keep()
        mats = [make_material(m, self.keep) for m in prob.materials]
        self.mats = (orc_material * max(1, len(mats)))(*mats)
        vols = [make_volume(v) for v in prob.volumes]
        self.vols = (orc_volume * len(vols))(*vols)
        self.src = make_source(prob.source)
        tals = [make_tally(t) for t in prob.tallies]
        self.tals = (orc_tally * max(1, len(tals)))(*tals)
        self.p = orc_problem(len(mats), len(vols), len(tals), 0,
                             C.cast(self.mats, C.POINTER(orc_material)), C.cast(self.vols, C.POINTER(orc_volume)),
                             C.pointer(self.src), C.cast(self.tals, C.POINTER(orc_tally)))


@dataclass
class Result:
    sumw: List[np.ndarray]
    sumw2: List[np.ndarray]
    n: int
    stats: dict
    records: Optional[np.ndarray]

    def mean(self, t):
        return self.sumw[t] / self.n

    def var_of_mean(self, t):
        """Variance of the per-history mean: (E[w^2] - mean^2) / (N - 1)."""
        m = self.sumw[t] / self.n
        return np.maximum(self.sumw2[t] / self.n - m * m, 0.0) / max(self.n - 1, 1)


def run(prob, seed: int = 4096, first: int = 0, n: Optional[int] = None, threads: int = 1,
        records: bool = False) -> Result:
    """Run histories [first, first+n) of the problem through the oracle."""
    if n is None:
        n = prob.n_histories
    cp = CProblem(prob)
    sumw = [np.zeros(t.nbins, dtype=np.float64) for t in prob.tallies]
    sumw2 = [np.zeros(t.nbins, dtype=np.float64) for t in prob.tallies]
    nt = max(1, len(sumw))
    pw = (C.POINTER(C.c_double) * nt)(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in sumw])
    pw2 = (C.POINTER(C.c_double) * nt)(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in sumw2])
    rec = np.zeros(n, dtype=RECORD_DTYPE) if records else None
    st = orc_stats()
    rc = lib().orc_run(C.byref(cp.p), seed, first, n, threads, pw, pw2,
                       rec.ctypes.data if rec is not None else None, C.byref(st))
    if rc != 0:
        raise RuntimeError(f"orc_run failed: {rc}")
    stats = {name: getattr(st, name) for name, _ in orc_stats._fields_}
    return Result(sumw, sumw2, n, stats, rec)


# pieces for the pin tests

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def uniform(seed, history, draw):
    return lib().orc_uniform(seed, history, draw)


def intervals(vol, p, u):
    v = make_volume(vol)
    pp = (C.c_double * 3)(*p)
    uu = (C.c_double * 3)(*u)
    ti = (C.c_double * 2)()
    to = (C.c_double * 2)()
    fi = (C.c_int32 * 2)()
    fo = (C.c_int32 * 2)()
    n = lib().orc_intervals(C.byref(v), pp, uu, ti, to, fi, fo)
    return [(ti[i], to[i], fi[i], fo[i]) for i in range(n)]


def contains(vol, p):
    v = make_volume(vol)
    return bool(lib().orc_contains(C.byref(v), (C.c_double * 3)(*p)))


def macro_xs(mat, lam):
    keep = _Keep()
    m = make_material(mat, keep)
    out = (C.c_double * 4)()
    lib().orc_macro_xs(C.byref(m), lam, out)
    return list(out)


def mirror_reflectivity(vol, Q):
    v = make_volume(vol)
    return lib().orc_mirror_reflectivity(C.byref(v), Q)


def ev_from_angstrom(lam):
    return lib().orc_ev_from_angstrom(lam)
