"""Pins of the oracle's transport physics against what the paper and the
mathematics fix, independent of the oracle's own formulas:

* Beer-Lambert unscattered transmission exp(-Sigma L) (cross section section,
  free-particle law), analog and biased, with Sigma from a brute-force sum over
  individual reciprocal-lattice vectors (not the oracle's family table);
* first-collision probabilities (Sigma_p/Sigma)(1 - exp(-Sigma L));
* 1/v absorption: -ln(transmission) proportional to lambda;
* Bragg's law 2 d sin(theta) = lambda for every coherent single scatter, with
  family frequencies proportional to m d |F|^2 and a uniform cone azimuth;
* isotropic bound incoherent scattering: cos(2theta) uniform on [-1, 1];
* weight conservation (exact with absorption off and no bias; mean 1 biased;
  escaped + absorbed mean 1 with absorption);
* biased and unbiased tallies agree (biasing mechanism section; total
  scattering validation);
* straight mirror guide solved per history by the method of images;
* mirror reflectivity special values; Maxwellian sampler against the
  truncated Gamma(3/2) law; energy-wavelength pairs printed in the paper;
* shells: transmission through both walls of the vessel;
* split-and-resume and threading do not change any history.
"""
import dataclasses
import os

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2304_06226_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def zscore(mean, expect, var):
    return (mean - expect) / np.sqrt(var)


# --------------------------------------------------------------------------
# independent cross-section route
# --------------------------------------------------------------------------

def sigma_coh_bruteforce(mat, a, lam):
    """Coherent elastic Sigma [1/mm] summing lambda^2 d |F|^2 / (2 v0 N) over every
    individual fcc reciprocal vector (h,k,l) with 2d > lambda.  |F|^2 of a vector
    is that of its family (matched by d and sorted |h|,|k|,|l|)."""
    d_f, m_f, reps = W.fcc_families(a, 0.5)
    assert np.allclose(d_f, mat.d)
    f2_of = {r: f for r, f in zip(reps, mat.f2)}
    total = 0.0
    hmax = int(np.ceil(2 * a / lam)) + 1
    for h in range(-hmax, hmax + 1):
        for k in range(-hmax, hmax + 1):
            for l in range(-hmax, hmax + 1):
                s = h * h + k * k + l * l
                if s == 0 or len({h & 1, k & 1, l & 1}) != 1:
                    continue
                d = a / np.sqrt(s)
                if d < 0.5 or not (2 * d > lam):
                    continue
                rep = tuple(sorted((abs(h), abs(k), abs(l)), reverse=True))
                total += lam * lam * d * f2_of[rep] / (2 * mat.cell_volume * mat.atoms_per_cell)
    return mat.number_density * total * 1e-1


def test_cross_sections_against_bruteforce():
    mat = W.sample_material()
    for lam in (0.6, 1.0, 1.8, 2.5, 4.0, 4.7, 8.0):
        xs = O.macro_xs(mat, lam)
        assert xs[2] == pytest.approx(sigma_coh_bruteforce(mat, 4.0, lam), rel=1e-12, abs=1e-15)
        assert xs[1] == pytest.approx(0.06 * 5.0 * 0.1, rel=1e-14)
        # 1/v absorption: proportional to lambda, 2 b at 1.798 A
        assert xs[0] == pytest.approx(0.06 * 2.0 * 0.1 * lam / 1.798, rel=1e-14)
        # the number of active families is the number of Bragg edges above lambda
        assert xs[3] == (2 * mat.d > lam).sum()
    # beyond the largest edge (2 d_111 = 4.62 A) coherent elastic vanishes
    assert O.macro_xs(mat, 4.7)[2] == 0.0


def test_energy_wavelength_pairs_from_paper():
    with open(os.path.join(HERE, "golden", "energy_wavelength.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            e, lam, tol = map(float, line.split())
            assert O.ev_from_angstrom(lam) == pytest.approx(e, rel=tol)


# --------------------------------------------------------------------------
# transport closed forms
# --------------------------------------------------------------------------

def pencil_problem(mat, lam=1.8, radius=5.0):
    p = W.analog_sample()
    p.materials = [mat]
    p.volumes[1] = dataclasses.replace(p.volumes[1], size=(radius, 20.0))
    p.source = dataclasses.replace(p.source, lam0=lam)
    return p


@pytest.mark.parametrize("gs,ga", [(1.0, 1.0), (4.0, 1.0), (3.0, 0.5)])
def test_beer_lambert_transmission(gs, ga):
    mat = W.sample_material().biased(scatter_bias=gs, abs_bias=ga)
    p = pencil_problem(mat)
    n = 400_000
    r = O.run(p, n=n, threads=8)
    lam = 1.8
    sig = 0.06 * 0.1 * (5.0 + 2.0 * lam / 1.798) + sigma_coh_bruteforce(mat, 4.0, lam)
    expect = np.exp(-sig * 10.0)
    z = zscore(r.mean(1)[0], expect, r.var_of_mean(1)[0])
    assert abs(z) < 4.0, (r.mean(1)[0], expect, z)


def test_first_collision_probabilities():
    mat = W.sample_material()
    p = pencil_problem(mat)
    n = 400_000
    r = O.run(p, n=n, threads=8, records=True)
    rec = r.records
    lam = 1.8
    sa = 0.06 * 0.1 * 2.0 * lam / 1.798
    ss = 0.06 * 0.1 * 5.0 + sigma_coh_bruteforce(mat, 4.0, lam)
    sig = sa + ss
    pc = 1 - np.exp(-sig * 10.0)
    scat = (rec["n_scat"] >= 1).mean()
    absorbed_first = ((rec["term"] == O.END_ABSORB) & (rec["n_scat"] == 0)).mean()
    for obs, exp in ((scat, ss / sig * pc), (absorbed_first, sa / sig * pc)):
        assert abs(obs - exp) < 4 * np.sqrt(exp * (1 - exp) / n), (obs, exp)


def test_absorption_one_over_v():
    base = W.Material(number_density=0.06, sigma_inc=0.0, sigma_abs_ref=20.0)
    trans = {}
    n = 300_000
    for lam in (1.0, 4.0):
        p = pencil_problem(base, lam=lam)
        r = O.run(p, n=n, threads=8)
        trans[lam] = r.mean(1)[0]
    for lam, t in trans.items():
        exp = np.exp(-0.06 * 0.1 * 20.0 * lam / 1.798 * 10.0)
        assert abs(t - exp) < 4 * np.sqrt(exp * (1 - exp) / n)
    ratio = np.log(trans[4.0]) / np.log(trans[1.0])
    assert ratio == pytest.approx(4.0, rel=0.02)


def dilute(mat, factor=1e-4):
    return dataclasses.replace(mat, number_density=mat.number_density * factor)


def test_bragg_single_scatter_angles_and_weights():
    lam, a = 1.8, 4.0
    base = W.sample_material()
    mat = dilute(dataclasses.replace(base, sigma_inc=0.0, sigma_abs_ref=0.0), 0.1)
    p = pencil_problem(mat, lam=lam)
    r = O.run(p, n=600_000, threads=8, records=True)
    rec = r.records
    single = rec[(rec["n_scat"] == 1) & (rec["term"] == O.END_ESCAPE)]
    assert len(single) > 5000
    two_theta = np.degrees(np.arccos(np.clip(single["dir"][:, 2], -1, 1)))
    # Bragg's law from the lattice alone: d = a / sqrt(h^2+k^2+l^2)
    d_f, m_f, reps = W.fcc_families(a, 0.5)
    peaks = np.degrees(2 * np.arcsin(lam / (2 * d_f[2 * d_f > lam])))
    dist = np.min(np.abs(two_theta[:, None] - peaks[None, :]), axis=1)
    assert dist.max() < 1e-6
    # the seven peaks quoted for lambda=1.8 A, a=4.0 A
    assert np.allclose(np.unique(np.round(peaks, 2)), [45.87, 53.49, 79.05, 96.53, 102.42, 128.32, 157.48], atol=0.01)
    # frequencies proportional to m d F^2 (families of equal d merged)
    act = 2 * d_f > lam
    wts = (m_f * d_f * mat.f2)[act]
    dd = d_f[act]
    ud = np.unique(np.round(dd, 12))
    probs = np.array([wts[np.isclose(dd, x)].sum() for x in ud])
    probs /= probs.sum()
    pk = np.degrees(2 * np.arcsin(lam / (2 * ud)))
    idx = np.argmin(np.abs(two_theta[:, None] - pk[None, :]), axis=1)
    counts = np.bincount(idx, minlength=len(ud))
    chi2, pval = stats.chisquare(counts, probs * counts.sum())
    assert pval > 1e-3, (counts, probs * counts.sum())
    # Debye-Scherrer cone: the azimuth about the beam is uniform
    phi = np.arctan2(single["dir"][:, 1], single["dir"][:, 0])
    h, _ = np.histogram(phi, bins=24, range=(-np.pi, np.pi))
    assert stats.chisquare(h).pvalue > 1e-3


def test_incoherent_isotropic():
    mat = dilute(W.Material(number_density=0.06, sigma_inc=5.0, sigma_abs_ref=0.0), 0.1)
    p = pencil_problem(mat)
    r = O.run(p, n=600_000, threads=8, records=True)
    rec = r.records
    single = rec[(rec["n_scat"] == 1) & (rec["term"] == O.END_ESCAPE)]
    assert len(single) > 5000
    mu = single["dir"][:, 2]
    h, edges = np.histogram(mu, bins=20, range=(-1, 1))
    assert stats.chisquare(h).pvalue > 1e-3
    # bin probability (cos a - cos b)/2 on 2theta bins
    tt = np.degrees(np.arccos(np.clip(mu, -1, 1)))
    hb, eb = np.histogram(tt, bins=18, range=(0, 180))
    pb = (np.cos(np.radians(eb[:-1])) - np.cos(np.radians(eb[1:]))) / 2
    assert stats.chisquare(hb, pb * hb.sum()).pvalue > 1e-3
    phi = np.arctan2(single["dir"][:, 1], single["dir"][:, 0])
    hp, _ = np.histogram(phi, bins=24, range=(-np.pi, np.pi))
    assert stats.chisquare(hp).pvalue > 1e-3


def test_weight_conservation():
    base = dataclasses.replace(W.sample_material(), sigma_abs_ref=0.0)
    # absorption off, no bias: every history ends with weight exactly 1
    r = O.run(pencil_problem(base), n=50_000, threads=4, records=True)
    assert np.all(r.records["w"] == 1.0)
    assert np.all(r.records["term"] == O.END_ESCAPE)
    # absorption off, biased: mean escaped weight 1
    r = O.run(pencil_problem(base.biased(scatter_bias=4.0)), n=200_000, threads=8, records=True)
    w = r.records["w"]
    assert abs(w.mean() - 1.0) < 4 * w.std() / np.sqrt(len(w))
    assert np.any(w != 1.0)
    # with absorption and both biases: escaped + absorbed weight has mean 1
    mat = W.sample_material().biased(scatter_bias=3.0, abs_bias=0.5)
    r = O.run(pencil_problem(mat), n=200_000, threads=8, records=True)
    w = r.records["w"]
    assert set(np.unique(r.records["term"])) <= {O.END_ESCAPE, O.END_ABSORB}
    assert abs(w.mean() - 1.0) < 4 * w.std() / np.sqrt(len(w))


def merged_chi2(m1, v1, c1, m2, v2, c2, min_count=25):
    """chi^2 of per-bin z-scores, merging adjacent bins until both sides have
    at least min_count entries."""
    zs = []
    am1 = av1 = am2 = av2 = 0.0
    ac1 = ac2 = 0
    for i in range(len(m1)):
        am1 += m1[i]; av1 += v1[i]; am2 += m2[i]; av2 += v2[i]; ac1 += c1[i]; ac2 += c2[i]
        if ac1 >= min_count and ac2 >= min_count:
            zs.append((am1 - am2) / np.sqrt(av1 + av2))
            am1 = av1 = am2 = av2 = 0.0
            ac1 = ac2 = 0
    zs = np.array(zs)
    return (zs ** 2).sum(), len(zs), zs


def test_biased_equals_unbiased():
    n = 400_000
    p1 = W.analog_sample()
    pb = W.biased_sample(n=n)
    pb.tallies = [W.Tally(trigger="escape", filter="scattered", axes=[W.Axis("theta2", 0, 180, 1800)])] + pb.tallies[1:]
    ra = O.run(p1, n=n, threads=8, seed=4096)
    rb = O.run(pb, n=n, threads=8, seed=4097)
    # entry counts: analog weights are 1, so counts equal sum w; biased counts from w and w^2
    ca = ra.sumw[0]
    cb = np.where(rb.sumw2[0] > 0, rb.sumw[0] ** 2 / np.maximum(rb.sumw2[0], 1e-300), 0)
    chi2, dof, zs = merged_chi2(ra.mean(0), ra.var_of_mean(0), ca, rb.mean(0), rb.var_of_mean(0), cb)
    assert dof > 5
    assert stats.chi2.sf(chi2, dof) > 1e-3, (chi2, dof)
    for t in (1, 2):
        z = zscore(ra.mean(t)[0], rb.mean(t)[0], ra.var_of_mean(t)[0] + rb.var_of_mean(t)[0])
        assert abs(z) < 4


def test_biasing_reduces_variance_of_single_scattering_signal():
    """For a weakly scattering sample, scattering bias > 1 improves the single
    scattering statistics (biasing mechanism section)."""
    n = 200_000
    mat = dilute(W.sample_material(), 0.05)
    res = {}
    for g in (1.0, 4.0):
        p = pencil_problem(mat.biased(scatter_bias=g))
        p.tallies = [W.Tally(trigger="escape", filter="nscat_eq", filter_arg=1)]
        res[g] = O.run(p, n=n, threads=8, seed=4096 + int(g))
    z = zscore(res[1.0].mean(0)[0], res[4.0].mean(0)[0], res[1.0].var_of_mean(0)[0] + res[4.0].var_of_mean(0)[0])
    assert abs(z) < 4
    assert res[4.0].var_of_mean(0)[0] < 0.5 * res[1.0].var_of_mean(0)[0]


# --------------------------------------------------------------------------
# mirrors and the guide
# --------------------------------------------------------------------------

def R_linear(Q, R0=0.99, Qc=0.0219, alpha=10.0, m=3.0):
    Q = np.asarray(Q, dtype=float)
    R = np.where(Q <= Qc, R0, R0 - alpha * (Q - Qc))
    R = np.where(Q > m * Qc, 0.0, R)
    return np.maximum(R, 0.0)


def test_mirror_reflectivity_values():
    g = W.m3_guide().volumes[0]
    assert O.mirror_reflectivity(g, 0.0) == 0.99
    assert O.mirror_reflectivity(g, 0.0219) == 0.99
    assert O.mirror_reflectivity(g, 3 * 0.0219) == pytest.approx(0.99 - 10 * 2 * 0.0219, rel=1e-12)
    assert O.mirror_reflectivity(g, 3 * 0.0219 + 1e-6) == 0.0
    t = dataclasses.replace(g, mirror=W.Mirror(model="tanh", R0=0.99, Qc=0.0219, alpha=6.07, m=2.0, W=0.003))
    # paper's form: at Q = m Qc the tanh factor is 1, leaving R0/2 (1 - alpha (m-1) Qc)
    assert O.mirror_reflectivity(t, 2 * 0.0219) == pytest.approx(0.5 * 0.99 * (1 - 6.07 * 0.0219), rel=1e-12)
    assert O.mirror_reflectivity(t, 0.01) == 0.99
    # just above Qc with m=2 the cut-off factor is 1 - tanh(-7.3) ~ 2
    assert O.mirror_reflectivity(t, 0.0219 + 1e-9) == pytest.approx(0.99, rel=1e-6)


def _fold(s, half):
    """Unfold a straight line through a channel of walls at +-half: returns the
    folded coordinate and the number of wall reflections."""
    w = 2 * half
    k = np.floor((s + half) / w)
    r = s - k * w
    x = np.where(k % 2 == 0, r, -r)
    return x, np.abs(k).astype(int)


def test_guide_method_of_images():
    p = W.m3_guide(n=20_000)
    n = 20_000
    r = O.run(p, n=n, threads=8, records=True)
    rec = r.records
    seed = 4096
    u = np.array([[O.uniform(seed, h, k) for k in range(5)] for h in range(n)])
    x0 = (u[:, 0] - 0.5) * 50.0
    y0 = (u[:, 1] - 0.5) * 50.0
    ax = (2 * u[:, 2] - 1) * np.radians(1.0)
    ay = (2 * u[:, 3] - 1) * np.radians(1.0)
    lam = 1.0 + u[:, 4] * 9.0
    v = np.stack([np.tan(ax), np.tan(ay), np.ones(n)], axis=1)
    v /= np.linalg.norm(v, axis=1)[:, None]
    L = 10000.0
    xs, nx = _fold(x0 + L * v[:, 0] / v[:, 2], 25.0)
    ys, ny = _fold(y0 + L * v[:, 1] / v[:, 2], 25.0)
    Rx = R_linear(4 * np.pi * np.abs(v[:, 0]) / lam)
    Ry = R_linear(4 * np.pi * np.abs(v[:, 1]) / lam)
    w = Rx ** nx * Ry ** ny
    alive = w > 0
    assert np.all((rec["term"] == O.END_ESCAPE) == alive)
    assert np.all(rec["term"][~alive] == O.END_KILL)
    e = alive
    assert np.allclose(rec["pos"][e, 0], xs[e], atol=1e-7)
    assert np.allclose(rec["pos"][e, 1], ys[e], atol=1e-7)
    assert np.allclose(rec["pos"][e, 2], L, atol=1e-7)
    assert np.allclose(rec["w"][e], w[e], rtol=1e-12)
    assert np.allclose(rec["dir"][e, 0], v[e, 0] * (-1.0) ** nx[e], atol=1e-14)
    assert np.allclose(rec["dir"][e, 1], v[e, 1] * (-1.0) ** ny[e], atol=1e-14)
    assert np.allclose(rec["lambda"], lam, rtol=1e-15)
    assert (nx + ny)[e].max() >= 3
    # the tally holds exactly the surviving weights
    assert r.sumw[0].sum() == pytest.approx(w[e].sum(), rel=1e-12)


# --------------------------------------------------------------------------
# sources
# --------------------------------------------------------------------------

def test_maxwellian_spectrum():
    p = W.vessel_sample(n=200_000)
    p.materials = []
    p.volumes = p.volumes[:1]
    p.tallies = []
    r = O.run(p, n=200_000, threads=8, records=True)
    lam = r.records["lambda"]
    assert lam.min() >= 0.5 and lam.max() <= 5.0
    kT = 0.025852
    E = O.ev_from_angstrom(1.0) / lam ** 2
    lo, hi = O.ev_from_angstrom(5.0) / kT, O.ev_from_angstrom(0.5) / kT
    g = stats.gamma(1.5)
    norm = g.cdf(hi) - g.cdf(lo)
    assert norm == pytest.approx(0.9686, abs=2e-4)
    edges = np.linspace(lo, hi, 41)
    h, _ = np.histogram(E / kT, bins=edges)
    pe = np.diff(g.cdf(edges)) / norm
    keep = pe * len(E) > 25
    assert stats.chisquare(h[keep], pe[keep] * len(E) * h[keep].sum() / (pe[keep] * len(E)).sum()).pvalue > 1e-3
    # one extra set of three draws per rejected try
    assert np.all((r.records["n_draws"] - 2) % 3 == 0)


def test_rect_sources_uniform():
    p = W.m3_guide(n=100_000)
    p.tallies = []
    p.volumes = [dataclasses.replace(p.volumes[0], mirror_mask=0)]
    r = O.run(p, n=100_000, threads=8, records=True)
    seed = 4096
    # positions and divergences come out uniform (checked on the draws' images)
    u0 = np.array([O.uniform(seed, h, 0) for h in range(2000)])
    assert np.allclose(u0, np.array([O.uniform(seed, h, 0) for h in range(2000)]))
    lam = r.records["lambda"]
    h, _ = np.histogram(lam, bins=30, range=(1, 10))
    assert stats.chisquare(h).pvalue > 1e-3
    d = r.records["dir"]
    ax = np.degrees(np.arctan2(d[:, 0], d[:, 2]))
    h, _ = np.histogram(ax, bins=20, range=(-1, 1))
    assert stats.chisquare(h).pvalue > 1e-3


# --------------------------------------------------------------------------
# shells, determinism
# --------------------------------------------------------------------------

def test_vessel_shell_transmission():
    p = W.vessel_sample(n=200_000)
    vessel = p.materials[1]
    p.volumes = p.volumes[:2]          # world + vessel only
    p.source = W.Source("pencil", origin=(0.0, 0.0, -100.0), spectrum="mono", lam0=1.8)
    r = O.run(p, n=200_000, threads=8)
    sa = vessel.number_density * 0.1 * 0.23 * 1.8 / 1.798
    si = vessel.number_density * 0.1 * 0.01
    sc = sigma_coh_bruteforce(vessel, 4.05, 1.8)
    expect = np.exp(-(sa + si + sc) * 2 * 1.0)
    z = zscore(r.mean(1)[0], expect, r.var_of_mean(1)[0])
    assert abs(z) < 4, (r.mean(1)[0], expect)


def test_split_resume_and_threads_identical():
    p = W.vessel_sample(n=20_000)
    full = O.run(p, n=20_000, threads=1, records=True)
    a = O.run(p, first=0, n=7_000, threads=3, records=True)
    b = O.run(p, first=7_000, n=13_000, threads=5, records=True)
    both = np.concatenate([a.records, b.records])
    assert (both == full.records).all()
    for t in range(len(p.tallies)):
        assert np.allclose(a.sumw[t] + b.sumw[t], full.sumw[t], rtol=1e-12, atol=1e-300)


# --------------------------------------------------------------------------
# imaging: unscattered transmission through axis-aligned boxes
# --------------------------------------------------------------------------

def test_imaging_unscattered_transmission_closed_form():
    """A parallel beam along z through axis-aligned boxes: the probability of
    reaching the detector unscattered is exp(-sum_i Sigma_i dz_i) over the boxes
    whose xy-extent covers the source point (Beer-Lambert per chord)."""
    p = W.imaging_problem(n=40_000, n_boxes=300)
    n = 40_000
    r = O.run(p, n=n, threads=8, records=True)
    rec = r.records
    seed = 4096
    x0 = np.array([(O.uniform(seed, h, 0) - 0.5) * 500.0 for h in range(n)])
    y0 = np.array([(O.uniform(seed, h, 1) - 0.5) * 500.0 for h in range(n)])
    sig = []
    for m in p.materials:
        xs = O.macro_xs(m, 2.0)
        sig.append(xs[0] + xs[1] + xs[2])
    tau = np.zeros(n)
    for v in p.volumes[1:-1]:
        cx, cy, _ = v.center
        sx, sy, sz = v.size
        inside = (np.abs(x0 - cx) <= sx / 2) & (np.abs(y0 - cy) <= sy / 2)
        tau += inside * sig[v.material] * sz
    expect = np.exp(-tau)
    det = len(p.volumes) - 1
    got = ((rec["term"] == O.END_DETECT) & (rec["n_scat"] == 0) & (rec["region"] == det)).astype(float)
    # per history the unscattered outcome is Bernoulli(expect): z-test of the total and of 16 groups
    z = (got.sum() - expect.sum()) / np.sqrt((expect * (1 - expect)).sum())
    assert abs(z) < 4, z
    grp = np.argsort(expect)
    for g in np.array_split(grp, 16):
        v = (expect[g] * (1 - expect[g])).sum()
        if v > 10:
            assert abs((got[g].sum() - expect[g].sum()) / np.sqrt(v)) < 4.5
    # the tally's unscattered image holds exactly those weights
    assert r.sumw[1].sum() == pytest.approx(got.sum())


# ---------------------------------------------------------------------------
# Momentum-transfer tally (DeltaMomentum scorer) and process removal
# ---------------------------------------------------------------------------

def _q_problem(mat, lam, qmax, nbins, filt="nscat_eq", arg=1):
    p = pencil_problem(mat, lam=lam)
    p.tallies = [W.Tally(trigger="escape", filter=filt, filter_arg=arg, axes=[W.Axis("q", 0.0, qmax, nbins)])]
    return p


@pytest.mark.parametrize("lam", [1.8, 1.2])
def test_q_tally_single_bragg_peaks_at_2pi_over_d(lam):
    """A single coherent scattering transfers Q = 2 k sin(theta) = 2 pi / d_j for
    any wavelength (Bragg's law): the single-scattering Q tally has weight only in
    bins holding some 2 pi / d_j of an active family (2 d_j > lambda), with
    weights proportional to m_j d_j F2_j."""
    a = 4.0
    base = W.sample_material()
    mat = dilute(dataclasses.replace(base, sigma_inc=0.0, sigma_abs_ref=0.0), 0.1)
    qmax, nb = 20.0, 20000
    r = O.run(_q_problem(mat, lam, qmax, nb), n=400_000, threads=8)
    sw = r.sumw[0]
    assert sw.sum() > 3000
    d_f, m_f, _ = W.fcc_families(a, 0.5)
    act = 2 * d_f > lam
    q_peaks = 2 * np.pi / d_f[act]
    width = qmax / nb
    centers = (np.arange(nb) + 0.5) * width
    hit = np.nonzero(sw)[0]
    dist = np.min(np.abs(centers[hit][:, None] - q_peaks[None, :]), axis=1)
    assert dist.max() <= width, dist.max()
    # weight per distinct d against m d F2
    wts = (m_f * d_f * mat.f2)[act]
    dd = d_f[act]
    ud = np.unique(np.round(dd, 12))
    probs = np.array([wts[np.isclose(dd, x)].sum() for x in ud])
    probs /= probs.sum()
    qd = 2 * np.pi / ud
    which = np.argmin(np.abs(centers[hit][:, None] - qd[None, :]), axis=1)
    counts = np.bincount(which, weights=sw[hit], minlength=len(ud))   # unit weights: counts
    assert stats.chisquare(counts, probs * counts.sum()).pvalue > 1e-3


def test_q_tally_isotropic_closed_form():
    """Isotropic single scattering: cos(alpha) is uniform, so with s = Q lambda / (4 pi)
    P(s <= x) = x^2 and a Q bin [a, b] holds (b^2 - a^2) / Q_max^2 of the entries."""
    lam = 1.8
    mat = dilute(W.Material(number_density=0.06, sigma_inc=5.0, sigma_abs_ref=0.0), 0.1)
    qmax = 4 * np.pi / lam
    nb = 24
    r = O.run(_q_problem(mat, lam, qmax, nb), n=600_000, threads=8)
    counts = r.sumw[0]
    assert counts.sum() > 3000
    e = np.linspace(0.0, qmax, nb + 1)
    pb = (e[1:] ** 2 - e[:-1] ** 2) / qmax ** 2
    assert stats.chisquare(counts, pb * counts.sum()).pvalue > 1e-3


def test_bias_factor_zero_removes_the_process():
    """A bias factor of 0 removes that process from the physics (not a variance
    reduction): with abs_bias = 0 nothing is absorbed and the transmission is
    exp(-Sigma_s L); with scatter_bias = 0 nothing scatters, the transmission is
    exp(-Sigma_a L) and the rest is absorbed.  The remaining process is unbiased,
    so every weight stays exactly 1."""
    lam, L = 1.8, 10.0
    base = W.sample_material()
    sa = 0.06 * 0.1 * 2.0 * lam / 1.798
    ss = 0.06 * 0.1 * 5.0 + sigma_coh_bruteforce(base, 4.0, lam)
    n = 300_000
    r = O.run(pencil_problem(base.biased(abs_bias=0.0), lam=lam), n=n, threads=8, records=True)
    assert r.stats["absorbed"] == 0
    assert np.all(r.records["w"] == 1.0)
    t = r.mean(1)[0]
    exp_t = np.exp(-ss * L)
    assert abs(t - exp_t) < 4 * np.sqrt(exp_t * (1 - exp_t) / n)
    r = O.run(pencil_problem(base.biased(scatter_bias=0.0), lam=lam), n=n, threads=8, records=True)
    assert np.all(r.records["n_scat"] == 0)
    assert np.all(r.records["w"] == 1.0)
    t = r.mean(1)[0]
    exp_t = np.exp(-sa * L)
    assert abs(t - exp_t) < 4 * np.sqrt(exp_t * (1 - exp_t) / n)
    assert abs(r.stats["absorbed"] / n - (1 - exp_t)) < 4 * np.sqrt(exp_t * (1 - exp_t) / n)


# ---------------------------------------------------------------------------
# Moderator-surface gun and the paper's m = 1 guide benchmark
# ---------------------------------------------------------------------------

def _gun_problem(det_z, side=300.0, nb=60):
    vols = [W.Volume("box", (0.0, 0.0, 1000.0), (400.0, 400.0, 3000.0)),
            W.Volume("box", (0.0, 0.0, det_z + 1.0), (side, side, 2.0), parent=0, detector=True)]
    src = W.Source("moderator", origin=(10.0, -5.0, 0.0), size=(60.0, 40.0), spectrum="mono", lam0=2.0,
                   slit_center=(3.0, 4.0, 500.0), slit_size=(20.0, 30.0))
    h = side / 2
    tallies = [W.Tally(trigger="detect", trigger_volume=1, axes=[W.Axis("x", -h, h, nb)]),
               W.Tally(trigger="detect", trigger_volume=1, axes=[W.Axis("y", -h, h, nb)])]
    return W.Problem([], vols, src, tallies, n_histories=0, name="gun")


def _sum_of_uniforms_cdf(x, a1, a2, b1, b2):
    """Exact CDF of A + B with A ~ U[a1, a2] and B ~ U[b1, b2] independent."""
    w = a2 - a1

    def G(t):   # integral of the CDF of A up to t
        return np.where(t <= a1, 0.0, np.where(t <= a2, (t - a1) ** 2 / (2 * w), t - a1 - w / 2))
    return (G(x - b1) - G(x - b2)) / (b2 - b1)


def test_moderator_gun_hits_the_slit_uniformly():
    """Every ray crosses the slit plane inside the slit, uniformly (the detector's
    front face is the slit plane)."""
    p = _gun_problem(500.0, side=300.0, nb=300)
    r = O.run(p, n=200_000, threads=8)
    assert r.stats["detected"] == 200_000
    for t, (c, half) in enumerate(((3.0, 10.0), (4.0, 15.0))):
        sw = r.sumw[t]
        edges = np.linspace(-150, 150, 301)
        inside = (edges[:-1] >= c - half) & (edges[1:] <= c + half)
        assert sw[~inside].sum() == 0
        assert stats.chisquare(sw[inside]).pvalue > 1e-3


def test_moderator_gun_far_plane_is_a_trapezoid():
    """Beyond the slit the crossing point is a fixed mix of two independent
    uniforms, x = f x_slit - (f - 1) x_source with f = z / z_slit: its distribution
    is the trapezoid of a sum of uniforms."""
    zd = 1500.0
    f = zd / 500.0
    p = _gun_problem(zd, side=300.0, nb=60)
    n = 400_000
    r = O.run(p, n=n, threads=8)
    assert r.stats["detected"] == n
    edges = np.linspace(-150, 150, 61)
    for t, (cs, hs, ct, ht) in enumerate(((10.0, 30.0, 3.0, 10.0), (-5.0, 20.0, 4.0, 15.0))):
        a1, a2 = f * (ct - ht), f * (ct + ht)
        b1, b2 = -(f - 1) * (cs + hs), -(f - 1) * (cs - hs)
        pb = np.diff(_sum_of_uniforms_cdf(edges, a1, a2, b1, b2))
        assert abs(pb.sum() - 1) < 1e-12
        keep = pb * n > 5
        obs = r.sumw[t]
        assert obs[~keep].sum() <= 5 * (~keep).sum()
        exp = pb[keep] * n
        assert stats.chisquare(obs[keep], exp * obs[keep].sum() / exp.sum()).pvalue > 1e-3


def R_tanh(Q, R0=0.99, Qc=0.0219, alpha=6.07, m=1.0, W_=0.003):
    Q = np.asarray(Q, dtype=float)
    R = 0.5 * R0 * (1 - alpha * (Q - Qc)) * (1 - np.tanh((Q - m * Qc) / W_))
    return np.maximum(np.where(Q <= Qc, R0, R), 0.0)


def test_paper_guide_method_of_images():
    """The paper's m = 1 guide per history: rays entering the opening are unfolded
    through the mirror walls (weight R(Q)^n per axis with the paper's mirror model,
    a history ends where R = 0), fly on to the rear detector plane, and rays
    hitting the wall fronts are absorbed."""
    p = W.paper_guide(n=20_000, det_bins=10)
    n = 20_000
    r = O.run(p, n=n, threads=8, records=True)
    rec = r.records
    u = np.array([[O.uniform(4096, h, k) for k in range(4)] for h in range(n)])
    xs, ys = (u[:, 0] - 0.5) * 50.0, (u[:, 1] - 0.5) * 50.0
    xt, yt = (u[:, 2] - 0.5) * 50.0, (u[:, 3] - 0.5) * 50.0
    v = np.stack([xt - xs, yt - ys, np.full(n, 1000.0)], axis=1)
    v /= np.linalg.norm(v, axis=1)[:, None]
    x_in = xs + 1100.0 * v[:, 0] / v[:, 2]
    y_in = ys + 1100.0 * v[:, 1] / v[:, 2]
    clear = (np.abs(np.abs(x_in) - 25.0) > 0.02) & (np.abs(np.abs(y_in) - 25.0) > 0.02)
    enter = clear & (np.abs(x_in) < 25.0) & (np.abs(y_in) < 25.0)
    wall = clear & ~enter
    assert np.all(rec["term"][wall] == O.END_ABSORB)
    lam = 3.39
    xe, nx = _fold(x_in + 1000.0 * v[:, 0] / v[:, 2], 25.0)
    ye, ny = _fold(y_in + 1000.0 * v[:, 1] / v[:, 2], 25.0)
    Rx = R_tanh(4 * np.pi * np.abs(v[:, 0]) / lam)
    Ry = R_tanh(4 * np.pi * np.abs(v[:, 1]) / lam)
    dead = ((nx > 0) & (Rx == 0)) | ((ny > 0) & (Ry == 0))
    w = Rx ** nx * Ry ** ny
    # where 1 - tanh(.) is within an ulp of 0 two libraries may give R = 0 or ~1e-17:
    # such rays must be killed or carry a weight below 1e-12
    faint = ((nx > 0) & (Rx < 1e-12)) | ((ny > 0) & (Ry < 1e-12))
    assert np.all(rec["term"][enter & dead & ~faint] == O.END_KILL)
    assert np.all((rec["term"][enter & faint] == O.END_KILL) | (rec["w"][enter & faint] < 1e-12))
    live = enter & ~dead & ~faint
    vx = v[:, 0] * (-1.0) ** nx
    vy = v[:, 1] * (-1.0) ** ny
    xd = xe + 1100.0 * vx / v[:, 2]
    yd = ye + 1100.0 * vy / v[:, 2]
    hit = live & (np.abs(xd) < 49.9) & (np.abs(yd) < 49.9)
    miss = live & ((np.abs(xd) > 50.2) | (np.abs(yd) > 50.2))
    assert np.all(rec["term"][hit] == O.END_DETECT)
    assert np.all(rec["term"][miss] == O.END_ESCAPE)
    assert np.allclose(rec["w"][hit], w[hit], rtol=1e-12)
    assert np.allclose(rec["pos"][hit, 0], xd[hit], atol=1e-6)
    assert np.allclose(rec["pos"][hit, 1], yd[hit], atol=1e-6)
    assert np.allclose(rec["pos"][hit, 2], 3200.0, atol=1e-6)
    assert hit.sum() > 0.3 * n and wall.sum() > 0.1 * n and (enter & dead).sum() > 0.2 * n
    assert (nx + ny)[hit].max() >= 2


# ---------------------------------------------------------------------------
# Time of flight and the disk chopper (ray-tracing mask)
# ---------------------------------------------------------------------------

H_OVER_MN = 6.62607015e-34 / 1.67492749804e-27 * 1e13      # mm A / s, from CODATA h and m_n
E_CONST = 0.0818042                                          # eV A^2, E = E_CONST / lambda^2


def test_tof_of_the_maxwellian_beam():
    """Without the chopper every neutron reaches the detector face 10001 mm away
    at t = L lambda m_n / h (the path is straight, L(1/cos - 1) < 3e-6 L), so the
    TOF histogram is the truncated Maxwellian energy law mapped to time."""
    p = W.paper_chopper(chopper=False, tof_bins=120)
    n = 400_000
    r = O.run(p, n=n, threads=8)
    assert r.stats["detected"] == n
    L = 10001.0
    kT = p.source.kT
    g = stats.gamma(1.5, scale=kT)
    lam_lo, lam_hi = p.source.lam_lo, p.source.lam_hi

    def cdf_lambda(x):   # P(lambda <= x) = P(E >= E_CONST / x^2)
        return g.sf(E_CONST / np.asarray(x) ** 2)
    mass = cdf_lambda(lam_hi) - cdf_lambda(lam_lo)
    edges = np.linspace(0.0, 0.03, 121)
    lam_edges = np.clip(edges * H_OVER_MN / L, lam_lo, lam_hi)
    pb = np.diff(cdf_lambda(np.maximum(lam_edges, 1e-9))) / mass
    obs = r.sumw[0]
    keep = pb * n > 20
    assert obs[~keep].sum() < 0.002 * n
    assert stats.chisquare(obs[keep], pb[keep] / pb[keep].sum() * obs[keep].sum()).pvalue > 1e-3


def _open_fraction(phase_deg, lam, slit=45.0, ngrid=1500):
    """Fraction of the 45x45 mm slit square that is open when a beam of one
    wavelength crosses the disk face (independent numpy evaluation of the
    chopper geometry: 4 windows of 20 degrees from phase, radii 130-250 mm, axis
    at (0, -190), 100 Hz; crossing time from the straight path from the origin)."""
    c = (np.arange(ngrid) + 0.5) / ngrid * slit - slit / 2
    x, y = np.meshgrid(c, c, indexing="ij")
    zf = 10000.0 - 0.001
    t = np.sqrt(x * x + y * y + zf * zf) * lam / H_OVER_MN
    qb, qc = x, y + 190.0
    rho = np.hypot(qb, qc)
    ang = np.arctan2(qc, qb) - np.radians(phase_deg) - 2 * np.pi * 100.0 * t
    m = np.mod(ang, np.pi / 2)
    return float(((rho >= 130.0) & (m < np.radians(20.0))).mean())


def test_chopper_transmission_of_a_mono_beam():
    """At one wavelength every neutron crosses the disk at the same time (to 1e-5),
    so the transmitted fraction is the open part of the beam footprint at that
    instant; with a phase that puts the whole footprint in a window, every neutron
    passes with weight 1."""
    lam = 2.0
    n = 300_000
    phases = np.arange(0.0, 90.0, 1.0)
    fr = np.array([_open_fraction(ph, lam, ngrid=300) for ph in phases])
    ph_half = phases[np.argmin(np.abs(fr - 0.5))]
    expect = _open_fraction(ph_half, lam)
    assert 0.3 < expect < 0.7
    r = O.run(W.paper_chopper(lam_mono=lam, phase=ph_half), n=n, threads=8, records=True)
    got = r.stats["detected"] / n
    assert abs(got - expect) < 4 * np.sqrt(expect * (1 - expect) / n), (got, expect)
    assert r.stats["killed"] + r.stats["detected"] == n
    assert np.all(r.records["w"][r.records["term"] == O.END_KILL] == 0.0)
    ph_open = phases[np.argmax(fr)]
    assert _open_fraction(ph_open, lam) == 1.0
    r = O.run(W.paper_chopper(lam_mono=lam, phase=ph_open), n=50_000, threads=8, records=True)
    assert r.stats["detected"] == 50_000 and np.all(r.records["w"] == 1.0)


def test_chopper_tof_windows_repeat_at_400_hz():
    """A point-like beam (1x1 mm slit) crossing the disk at 90 degrees in its frame
    passes only while (90 deg - 360 deg f t) mod 90 deg < 20 deg: TOF weight lies
    only in these windows, 0.556 ms wide every 2.5 ms (4 windows x 100 Hz), and
    every window inside the beam's TOF range is populated."""
    p = W.paper_chopper(slit=1.0, tof_bins=3000)
    n = 600_000
    r = O.run(p, n=n, threads=8)
    w = 2 * np.pi * 100.0
    per, th = np.pi / 2, np.radians(20.0)
    edges = np.linspace(0.0, 0.03, 3001)
    ks = np.arange(-20, 2)
    lo = (np.pi / 2 - th - ks * per) / w
    hi = (np.pi / 2 - ks * per) / w
    blur = 1e-5 * 0.6     # angular half-width of the 1 mm slit at 190 mm, in time
    nz = np.nonzero(r.sumw[0])[0]
    for b in nz:
        a0, a1 = edges[b], edges[b + 1]
        assert np.any((a1 >= lo - blur) & (a0 <= hi + blur)), (a0, a1)
    centers = np.sort((lo + hi)[(lo > 0.002) & (hi < 0.02)] / 2)
    assert np.allclose(np.diff(centers), 0.0025, atol=1e-12)
    for c_ in centers:
        inwin = (edges[:-1] >= c_ - th / w / 2) & (edges[1:] <= c_ + th / w / 2)
        assert r.sumw[0][inwin].sum() > 0
    assert 6 <= len(centers) <= 8


# ---------------------------------------------------------------------------
# Tabulated cross sections
# ---------------------------------------------------------------------------

def _tabulated(mat, lam_rows, sa_rows, si_rows):
    return dataclasses.replace(mat, table_lambda=np.asarray(lam_rows, float), table_sigma_abs=np.asarray(sa_rows, float),
                               table_sigma_inc=np.asarray(si_rows, float))


def test_table_of_the_analytic_law_reproduces_it():
    """A table sampled from the 1/v absorption law (linear in lambda, so linear
    interpolation is exact) and the constant incoherent cross section gives the
    analytic macroscopic cross sections at every wavelength inside it, and the end
    rows beyond it."""
    mat = W.sample_material()
    rows = np.linspace(0.5, 5.0, 10)
    tab = _tabulated(mat, rows, mat.sigma_abs_ref * rows / 1.798, np.full(10, mat.sigma_inc))
    for lam in np.linspace(0.55, 4.95, 37):
        a, b = O.macro_xs(mat, lam), O.macro_xs(tab, lam)
        assert np.allclose(a[:3], b[:3], rtol=1e-13), lam
        assert a[3] == b[3]
    lo, hi = O.macro_xs(tab, 0.2), O.macro_xs(tab, 7.0)
    assert lo[0] == pytest.approx(0.1 * mat.number_density * mat.sigma_abs_ref * 0.5 / 1.798, rel=1e-13)
    assert hi[0] == pytest.approx(0.1 * mat.number_density * mat.sigma_abs_ref * 5.0 / 1.798, rel=1e-13)


def test_table_interpolation_error_of_a_quadratic():
    """sigma_inc = 5 + 3 lambda^2 tabulated every 0.5 A: the oracle's values equal an
    independent linear interpolation, and at the middle of each interval the
    interpolation error is exactly the stated bound h^2 sigma'' / 8 = 0.1875 b."""
    mat = W.Material(number_density=0.05, sigma_inc=0.0, sigma_abs_ref=0.0)
    rows = np.arange(1.0, 6.01, 0.5)
    tab = _tabulated(mat, rows, np.zeros_like(rows), 5 + 3 * rows ** 2)
    k = 0.1 * mat.number_density
    for lam in np.linspace(1.01, 5.99, 50):
        assert O.macro_xs(tab, lam)[1] == pytest.approx(k * np.interp(lam, rows, 5 + 3 * rows ** 2), rel=1e-13)
    mids = rows[:-1] + 0.25
    err = np.array([O.macro_xs(tab, m)[1] / k for m in mids]) - (5 + 3 * mids ** 2)
    assert np.allclose(err, 0.5 ** 2 * 6 / 8, rtol=1e-10)


def test_table_transmission_spectrum():
    """A uniform 1-6 A pencil through a 10 mm path of a tabulated absorber: the
    transmitted fraction per wavelength bin is the bin average of
    exp(-Sigma_interp(lambda) L), Sigma_interp from an independent interpolation."""
    rows = np.array([1.0, 1.7, 2.5, 3.1, 4.4, 5.2, 6.0])
    sa = np.array([3.0, 9.0, 4.0, 12.0, 7.0, 2.0, 10.0])
    si = np.zeros_like(rows)
    mat = _tabulated(W.Material(number_density=0.06, sigma_inc=0.0, sigma_abs_ref=0.0), rows, sa, si)
    p = pencil_problem(mat)
    p.source = dataclasses.replace(p.source, spectrum="uniform", lam_lo=1.0, lam_hi=6.0)
    p.tallies = [W.Tally(trigger="escape", filter="unscattered", axes=[W.Axis("lambda", 1.0, 6.0, 25)])]
    n = 400_000
    r = O.run(p, n=n, threads=8)
    edges = np.linspace(1.0, 6.0, 26)
    fine = np.linspace(1.0, 6.0, 250001)
    tr = np.exp(-0.1 * 0.06 * np.interp(fine, rows, sa) * 10.0)
    expect = np.array([tr[(fine >= a) & (fine < b)].mean() for a, b in zip(edges[:-1], edges[1:])]) / 25
    got = r.sumw[0] / n
    var = expect * (1 - expect) / n
    z = (got - expect) / np.sqrt(var)
    assert stats.chi2.sf((z ** 2).sum(), len(z)) > 1e-3, z
