"""Seeded synthetic workloads: the neutral problem description fed to both the
GPU library and the CPU oracle.

This module holds no transport arithmetic.  It only *describes* problems
(materials, volumes, a source, tallies) with plain numbers and arrays, and
generates the synthetic crystal data that stands in for NCrystal material files
(reflection families of an fcc lattice with seeded |F|^2 values).  Both the HIP
binding and the oracle's wrapper translate these descriptions into their own
C structures; neither shares code with the other.

Units everywhere: lengths in mm, wavelengths in Angstrom, cross sections in
barn, number densities in atoms per Angstrom^3, angles in degrees, kT in eV.

Workloads (synthetic stand-ins for the paper's benchmark setups, section 4):
  analog_sample  plain FP64 powder sample, pencil beam, 1e5 histories
  biased_sample  same sample, scattering bias 4, 1e7 histories, 2theta x lambda
  vessel_sample  sample inside a cylindrical vessel shell, Maxwellian white beam
  m3_guide  straight 10 m mirror guide (m=3, piecewise-linear reflectivity)
  sample_batch  batch of small simulations plus an imaging setup of boxes
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

RUN_SEED = 4096  # the launcher's default seed (program section, launcher options table)

# Kinds are plain strings so that each binding maps them to its own integers.
SOLIDS = ("box", "cylinder", "cyl_shell", "sphere", "sph_shell")
SOURCES = ("pencil", "rect", "rect_divergent", "moderator")
SPECTRA = ("mono", "uniform", "maxwell")
TRIGGERS = ("escape", "absorb", "detect", "first_collision")
FILTERS = ("all", "unscattered", "scattered", "nscat_eq")
QUANTITIES = ("theta2", "lambda", "x", "y", "z", "div_x", "div_y", "nscat", "q", "tof")
MIRROR_MODELS = ("linear", "tanh")


@dataclass
class Material:
    number_density: float          # atoms / A^3
    sigma_inc: float               # b, constant (bound incoherent elastic)
    sigma_abs_ref: float           # b at 1.798 A (1/v law)
    scatter_bias: float = 1.0      # g for incoherent + coherent scattering
    abs_bias: float = 1.0          # g for absorption
    cell_volume: float = 0.0       # A^3, 0 means no Bragg scattering
    atoms_per_cell: int = 0
    d: np.ndarray = field(default_factory=lambda: np.zeros(0))       # A, descending
    mult: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int32))
    f2: np.ndarray = field(default_factory=lambda: np.zeros(0))      # b per cell
    # optional tables (lambda [A] increasing, sigma_abs [b], sigma_inc [b]) replacing the
    # 1/v absorption and the constant incoherent cross section by linear interpolation
    table_lambda: Optional[np.ndarray] = None
    table_sigma_abs: Optional[np.ndarray] = None
    table_sigma_inc: Optional[np.ndarray] = None

    def biased(self, scatter_bias=None, abs_bias=None) -> "Material":
        m = dataclasses.replace(self)
        if scatter_bias is not None:
            m.scatter_bias = float(scatter_bias)
        if abs_bias is not None:
            m.abs_bias = float(abs_bias)
        return m


@dataclass
class Mirror:
    model: str = "linear"   # "linear": R0 - alpha (Q - Qc) up to m Qc, "tanh": paper form
    R0: float = 0.99
    Qc: float = 0.0219      # 1/A
    alpha: float = 6.07     # A
    m: float = 1.0
    W: float = 0.003        # 1/A


@dataclass
class Chopper:
    n: int = 4                  # windows
    r: float = 130.0            # mm, inner black radius
    rot_freq: float = 100.0     # Hz
    theta0: float = 20.0        # degrees, window opening
    phase: float = 0.0          # degrees


@dataclass
class Volume:
    kind: str
    center: Tuple[float, float, float]
    size: Tuple[float, ...]          # box: sides; cylinder: r, h; cyl_shell: r_in, r_out, h;
                                     # sphere: r; sph_shell: r_in, r_out
    axis: int = 2                    # cylinder axis (0 x, 1 y, 2 z)
    parent: int = -1                 # -1 only for the world (index 0)
    material: int = -1               # -1 = vacuum
    detector: bool = False           # entering it scores 'detect' tallies and ends the history
    mirror_mask: int = 0             # faces carrying a mirror (bit per face id)
    mirror: Optional[Mirror] = None
    chopper: Optional["Chopper"] = None   # disk chopper carried by a cylinder


@dataclass
class Source:
    kind: str = "pencil"
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    direction: Tuple[float, float, float] = (0.0, 0.0, 1.0)
    size: Tuple[float, float] = (0.0, 0.0)         # rect width (x), height (y)
    divergence: Tuple[float, float] = (0.0, 0.0)   # rect_divergent half range, degrees
    spectrum: str = "mono"
    lam0: float = 1.8
    lam_lo: float = 0.5
    lam_hi: float = 5.0
    kT: float = 0.025852
    slit_center: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # moderator: slit centre, mm
    slit_size: Tuple[float, float] = (0.0, 0.0)                 # moderator: slit width (x), height (y)


@dataclass
class Axis:
    quantity: str
    lo: float
    hi: float
    nbins: int


@dataclass
class Tally:
    trigger: str = "escape"
    filter: str = "all"
    filter_arg: int = 0
    axes: List[Axis] = field(default_factory=list)
    beam: Tuple[float, float, float] = (0.0, 0.0, 1.0)
    trigger_volume: int = -1
    accumulator: str = "fp64"        # "fp64" or "kahan_fp32" (GPU side)

    @property
    def nbins(self) -> int:
        n = 1
        for a in self.axes:
            n *= int(a.nbins)
        return n

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(int(a.nbins) for a in self.axes) or (1,)


@dataclass
class Problem:
    materials: List[Material]
    volumes: List[Volume]
    source: Source
    tallies: List[Tally]
    n_histories: int = 0
    name: str = ""


# --------------------------------------------------------------------------
# synthetic crystal data (stands in for NCrystal's reflection lists)
# --------------------------------------------------------------------------

def fcc_families(a: float, dmin: float) -> Tuple[np.ndarray, np.ndarray, List[Tuple[int, int, int]]]:
    """Reflection families of a face-centred cubic lattice with d >= dmin.

    A family is the set of signed permutations of (h,k,l) (the m-3m point
    group acting on Miller indices); fcc allows only unmixed parity.  Returns
    (d, multiplicity, representative) in canonical order: d descending, then
    the representative (h>=k>=l>=0) descending lexicographically.  Families of
    equal d (e.g. 511 and 333) stay separate.
    """
    smax = int(np.floor((a / dmin) ** 2 + 1e-9))
    hmax = int(np.floor(np.sqrt(smax))) + 1
    fams = {}
    for h in range(-hmax, hmax + 1):
        for k in range(-hmax, hmax + 1):
            for l in range(-hmax, hmax + 1):
                if h == 0 and k == 0 and l == 0:
                    continue
                s = h * h + k * k + l * l
                if s > smax:
                    continue
                par = {h & 1, k & 1, l & 1}
                if len(par) != 1:
                    continue
                d = a / np.sqrt(s)
                if d < dmin:
                    continue
                rep = tuple(sorted((abs(h), abs(k), abs(l)), reverse=True))
                fams[rep] = fams.get(rep, 0) + 1
    reps = sorted(fams.keys(), key=lambda r: (-a / np.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2), tuple(-x for x in r)))
    d = np.array([a / np.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2) for r in reps], dtype=np.float64)
    m = np.array([fams[r] for r in reps], dtype=np.int32)
    return d, m, reps


def setup_rng(config: int) -> np.random.Generator:
    """Setup stream of a workload: numpy's Philox keyed on 4096 + config."""
    return np.random.Generator(np.random.Philox(key=RUN_SEED + config))


def fcc_material(a: float, number_density: float, sigma_inc: float, sigma_abs_ref: float,
                 rng: np.random.Generator, dmin: float = 0.5) -> Material:
    d, m, _ = fcc_families(a, dmin)
    f2 = rng.uniform(1.0, 10.0, size=len(d))
    return Material(number_density=number_density, sigma_inc=sigma_inc, sigma_abs_ref=sigma_abs_ref,
                    cell_volume=a ** 3, atoms_per_cell=4, d=d, mult=m, f2=f2)


def sample_material() -> Material:
    """The powder sample of the single-sample workloads: n=0.06/A^3, sigma_inc=5 b,
    sigma_abs=2 b at 1.798 A, fcc a=4.0 A, reflections d>=0.5 A, |F|^2 ~ U[1,10] b."""
    return fcc_material(4.0, 0.06, 5.0, 2.0, setup_rng(0))


def vessel_material() -> Material:
    """Aluminium-like vessel: fcc a=4.05 A, n=4/a^3, sigma_inc=0.01 b, sigma_abs=0.23 b."""
    a = 4.05
    return fcc_material(a, 4.0 / a ** 3, 0.01, 0.23, setup_rng(2))


def _angle_tally_2theta(nbins=1800) -> Tally:
    return Tally(trigger="escape", filter="scattered", axes=[Axis("theta2", 0.0, 180.0, nbins)])


def analog_sample(n: int = 100_000) -> Problem:
    """Plain FP64, no biasing: pencil beam lambda=1.8 A onto a solid cylinder (r=5, h=20 mm, axis y)."""
    mats = [sample_material()]
    vols = [Volume("sphere", (0.0, 0.0, 0.0), (1000.0,)),
            Volume("cylinder", (0.0, 0.0, 0.0), (5.0, 20.0), axis=1, parent=0, material=0)]
    src = Source("pencil", origin=(0.0, 0.0, -100.0), direction=(0.0, 0.0, 1.0), spectrum="mono", lam0=1.8)
    tallies = [_angle_tally_2theta(),
               Tally(trigger="escape", filter="unscattered"),   # transmitted
               Tally(trigger="absorb", filter="all")]           # absorbed
    return Problem(mats, vols, src, tallies, n_histories=n, name="analog_sample")


def biased_sample(n: int = 10_000_000, scatter_bias: float = 4.0) -> Problem:
    """Same sample with scattering biased by 4; 2theta(1800) x lambda(100 on [0.5,5] A)."""
    p = analog_sample(n)
    p.materials = [p.materials[0].biased(scatter_bias=scatter_bias)]
    p.tallies = [Tally(trigger="escape", filter="scattered",
                       axes=[Axis("theta2", 0.0, 180.0, 1800), Axis("lambda", 0.5, 5.0, 100)]),
                 Tally(trigger="escape", filter="unscattered"),
                 Tally(trigger="absorb", filter="all")]
    p.name = "biased_sample"
    return p


def vessel_sample(n: int = 100_000_000) -> Problem:
    """Powder diffractometer: sample (bias 2) inside an Al-like vessel shell, 300 K Maxwellian
    clipped to 0.5-5 A over a 10x10 mm square; 2theta(3600) x lambda(1000)."""
    mats = [sample_material().biased(scatter_bias=2.0), vessel_material()]
    vols = [Volume("sphere", (0.0, 0.0, 0.0), (1000.0,)),
            Volume("cyl_shell", (0.0, 0.0, 0.0), (10.0, 11.0, 40.0), axis=1, parent=0, material=1),
            Volume("cylinder", (0.0, 0.0, 0.0), (5.0, 20.0), axis=1, parent=0, material=0)]
    src = Source("rect", origin=(0.0, 0.0, -100.0), size=(10.0, 10.0), spectrum="maxwell",
                 lam_lo=0.5, lam_hi=5.0, kT=0.025852)
    tallies = [Tally(trigger="escape", filter="scattered",
                     axes=[Axis("theta2", 0.0, 180.0, 3600), Axis("lambda", 0.5, 5.0, 1000)]),
               Tally(trigger="escape", filter="unscattered"),
               Tally(trigger="absorb", filter="all")]
    return Problem(mats, vols, src, tallies, n_histories=n, name="vessel_sample")


def guide_mirror() -> Mirror:
    """m=3 supermirror, R=0.99 up to Qc=0.0219/A, then falling by 0.01 per 0.001/A, 0 beyond 3Qc."""
    return Mirror(model="linear", R0=0.99, Qc=0.0219, alpha=10.0, m=3.0, W=0.003)


def m3_guide(n: int = 100_000_000, nbins_xy: int = 200, nbins_div: int = 100) -> Problem:
    """Straight rectangular guide 50x50 mm, 10 m long, mirrors on the four side walls."""
    vols = [Volume("box", (0.0, 0.0, 5000.0), (50.0, 50.0, 10000.0), mirror_mask=0b001111,
                   mirror=guide_mirror())]
    src = Source("rect_divergent", origin=(0.0, 0.0, 0.0), size=(50.0, 50.0), divergence=(1.0, 1.0),
                 spectrum="uniform", lam_lo=1.0, lam_hi=10.0)
    tallies = [Tally(trigger="escape", filter="all",
                     axes=[Axis("x", -25.0, 25.0, nbins_xy), Axis("y", -25.0, 25.0, nbins_xy),
                           Axis("div_x", -1.0, 1.0, nbins_div), Axis("div_y", -1.0, 1.0, nbins_div)])]
    return Problem([], vols, src, tallies, n_histories=n, name="m3_guide")


def paper_guide(n: int = 100_000_000, det_side: float = 100.0, det_bins: int = 100) -> Problem:
    """The straight-guide benchmark of the paper's neutron guide section (a
    reproduction of McStas' Test_Guides): a 50x50 mm moderator surface at z = 0
    emitting 3.39 A neutrons aimed at a 50x50 mm window 1 m downstream (the front
    detector plane); an m = 1 straight guide formed by four wall boxes around a
    50x50x1000 mm opening whose entrance is at z = 1100 mm, with the paper's mirror
    model and default parameters (R0 0.99, Qc 0.0219 1/A, alpha 6.07 A, W 0.003
    1/A) on the opening's side faces and strongly absorbing walls (neutrons that
    miss the entrance stop in them); and a rear position-sensitive detector whose
    front face is 3.2 m from the source (det_side x det_side mm, det_bins^2
    pixels).  The walls stand 0.01 mm off the opening (volumes must not touch)."""
    mirror = Mirror(model="tanh", R0=0.99, Qc=0.0219, alpha=6.07, m=1.0, W=0.003)
    wall = Material(number_density=0.05, sigma_inc=0.0, sigma_abs_ref=5000.0)
    z0, length, t, gap = 1600.0, 1000.0, 10.0, 0.01
    half = 25.0 + gap
    vols = [Volume("box", (0.0, 0.0, 1650.0), (1000.0, 1000.0, 3500.0)),
            Volume("box", (0.0, 0.0, z0), (50.0, 50.0, length), parent=0, mirror_mask=0b001111, mirror=mirror),
            Volume("box", (+(half + t / 2), 0.0, z0), (t, 2 * (half + t), length), parent=0, material=0),
            Volume("box", (-(half + t / 2), 0.0, z0), (t, 2 * (half + t), length), parent=0, material=0),
            Volume("box", (0.0, +(half + t / 2), z0), (2 * half - 2 * gap, t, length), parent=0, material=0),
            Volume("box", (0.0, -(half + t / 2), z0), (2 * half - 2 * gap, t, length), parent=0, material=0),
            Volume("box", (0.0, 0.0, 3201.0), (det_side, det_side, 2.0), parent=0, detector=True)]
    det = len(vols) - 1
    src = Source("moderator", origin=(0.0, 0.0, 0.0), size=(50.0, 50.0), spectrum="mono", lam0=3.39,
                 slit_center=(0.0, 0.0, 1000.0), slit_size=(50.0, 50.0))
    h = det_side / 2
    tallies = [Tally(trigger="detect", trigger_volume=det, axes=[Axis("x", -h, h, det_bins), Axis("y", -h, h, det_bins)]),
               Tally(trigger="detect", trigger_volume=det)]
    return Problem([wall], vols, src, tallies, n_histories=n, name="paper_guide")


def paper_chopper(n: int = 10_000_000, chopper: bool = True, lam_mono: Optional[float] = None,
                  slit: float = 45.0, phase: float = 0.0, tof_bins: int = 600) -> Problem:
    """The disk-chopper benchmark of the paper's chopper section: a 293 K
    Maxwellian moderator gun (1x1 mm opening at z = 0 aimed at a 45x45 mm opening
    10 m away), a disk chopper in that plane (4 windows of 20 degrees, radii 130 and
    250 mm, 100 Hz; its axis is offset so that the beam crosses the middle of the
    window annulus, 190 mm from the axis), and a time-of-flight detector just behind
    it (TOF 0-30 ms).  chopper=False leaves the disk out; lam_mono replaces the
    Maxwellian by one wavelength."""
    vols = [Volume("box", (0.0, 0.0, 10000.0), (1200.0, 1200.0, 20400.0))]
    if chopper:
        vols.append(Volume("cylinder", (0.0, -190.0, 10000.0), (250.0, 0.002), axis=2, parent=0,
                           chopper=Chopper(n=4, r=130.0, rot_freq=100.0, theta0=20.0, phase=phase)))
    vols.append(Volume("box", (0.0, 0.0, 10002.0), (300.0, 300.0, 2.0), parent=0, detector=True))
    det = len(vols) - 1
    if lam_mono is None:
        src = Source("moderator", origin=(0.0, 0.0, 0.0), size=(1.0, 1.0), spectrum="maxwell", kT=0.025249,
                     lam_lo=0.1, lam_hi=20.0, slit_center=(0.0, 0.0, 10000.0), slit_size=(slit, slit))
    else:
        src = Source("moderator", origin=(0.0, 0.0, 0.0), size=(1.0, 1.0), spectrum="mono", lam0=lam_mono,
                     slit_center=(0.0, 0.0, 10000.0), slit_size=(slit, slit))
    tallies = [Tally(trigger="detect", trigger_volume=det, axes=[Axis("tof", 0.0, 0.03, tof_bins)]),
               Tally(trigger="detect", trigger_volume=det)]
    return Problem([], vols, src, tallies, n_histories=n, name="paper_chopper")


def with_histories(p: Problem, n: int) -> Problem:
    q = dataclasses.replace(p)
    q.n_histories = int(n)
    return q


# --------------------------------------------------------------------------
# batched workload: many small powder simulations plus an imaging setup
# --------------------------------------------------------------------------

@dataclass
class Batch:
    problems: List[Problem]          # one per simulation; n_histories each
    name: str = "batch"

    @property
    def total_histories(self) -> int:
        return int(sum(p.n_histories for p in self.problems))


def batch_sample_sims(n_sims: int = 256, scale: float = 1.0, rng: Optional[np.random.Generator] = None) -> List[Problem]:
    """Independent powder simulations: cylinder r ~ U[1,20] mm (h 20 mm, axis y),
    odd ones inside an Al-like vessel wall (r_in = r + 5, r_out = r_in + 1, h 40 mm);
    fcc a ~ U[3.5,6] A with n = 4/a^3, sigma_inc 5 b, sigma_abs 2 b; mono pencil
    lambda ~ U[1,5] A; scattering bias g in {1,2,4,8}; N ~ 10^U[4,6] (times scale);
    2theta(1800) of scattered escapes and a transmitted counter."""
    rng = setup_rng(4) if rng is None else rng
    vessel = vessel_material()
    sims = []
    for i in range(n_sims):
        r = rng.uniform(1.0, 20.0)
        lam = rng.uniform(1.0, 5.0)
        a = rng.uniform(3.5, 6.0)
        g = float(rng.choice([1.0, 2.0, 4.0, 8.0]))
        n = int(round(10 ** rng.uniform(4.0, 6.0) * scale))
        mat = fcc_material(a, 4.0 / a ** 3, 5.0, 2.0, rng).biased(scatter_bias=g)
        vols = [Volume("sphere", (0.0, 0.0, 0.0), (1000.0,)),
                Volume("cylinder", (0.0, 0.0, 0.0), (r, 20.0), axis=1, parent=0, material=0)]
        mats = [mat]
        if i % 2 == 1:
            mats.append(vessel)
            vols.append(Volume("cyl_shell", (0.0, 0.0, 0.0), (r + 5.0, r + 6.0, 40.0), axis=1, parent=0, material=1))
        src = Source("pencil", origin=(0.0, 0.0, -100.0), direction=(0.0, 0.0, 1.0), spectrum="mono", lam0=lam)
        tallies = [_angle_tally_2theta(), Tally(trigger="escape", filter="unscattered")]
        sims.append(Problem(mats, vols, src, tallies, n_histories=max(n, 1), name=f"sim{i}"))
    return sims


def imaging_problem(n: int = 10_000_000, n_boxes: int = 1000, rng: Optional[np.random.Generator] = None) -> Problem:
    """Imaging: n_boxes non-overlapping axis-aligned boxes (sides U[5,50] mm, placed
    by rejection with a 0.5 mm gap in 500x500x300 mm) of the powder-sample and vessel
    materials alternately, a parallel 2 A beam over 500x500 mm along +z and a 512x512
    pixel detector (500x500 mm) behind them."""
    rng = setup_rng(5) if rng is None else rng
    lo = np.array([-250.0, -250.0, -150.0])
    hi = np.array([250.0, 250.0, 150.0])
    centers, halves = [], []
    gap = 0.5
    attempts = 0
    while len(centers) < n_boxes:
        attempts += 1
        if attempts > 2_000_000:
            raise RuntimeError("could not place the imaging boxes")
        h = rng.uniform(5.0, 50.0, 3) / 2
        c = rng.uniform(lo + h, hi - h)
        if centers:
            C = np.asarray(centers)
            H = np.asarray(halves)
            sep = np.abs(C - c) - (H + h)
            if np.any(np.all(sep < gap, axis=1)):
                continue
        centers.append(c)
        halves.append(h)
    mats = [sample_material(), vessel_material()]
    vols = [Volume("box", (0.0, 0.0, 0.0), (700.0, 700.0, 600.0))]
    for i, (c, h) in enumerate(zip(centers, halves)):
        vols.append(Volume("box", tuple(c), tuple(2 * h), parent=0, material=i % 2))
    vols.append(Volume("box", (0.0, 0.0, 200.0), (520.0, 520.0, 2.0), parent=0, detector=True))
    det = len(vols) - 1
    src = Source("rect", origin=(0.0, 0.0, -250.0), direction=(0.0, 0.0, 1.0), size=(500.0, 500.0),
                 spectrum="mono", lam0=2.0)
    tallies = [Tally(trigger="detect", trigger_volume=det,
                     axes=[Axis("x", -250.0, 250.0, 512), Axis("y", -250.0, 250.0, 512)]),
               Tally(trigger="detect", trigger_volume=det, filter="unscattered",
                     axes=[Axis("x", -250.0, 250.0, 512), Axis("y", -250.0, 250.0, 512)])]
    return Problem(mats, vols, src, tallies, n_histories=n, name="imaging")


def sample_batch(scale: float = 1.0, imaging_histories: int = 10_000_000, n_sims: int = 256) -> Batch:
    """Batched: 256 uneven powder simulations plus the 1000-box imaging setup."""
    sims = batch_sample_sims(n_sims, scale)
    sims.append(imaging_problem(int(imaging_histories)))
    return Batch(sims, name="sample_batch")


