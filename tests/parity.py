"""Shared helpers of the GPU parity tests: run a workload through the C-ABI and
through the oracle on the same seeded inputs and compare.

Which comparison assumes what:
* compare_records_fp64 / compare_tallies_fp64: the FP64 policies against the
  oracle on the SAME history ids (the same random numbers), history by history.
* tally_stat_test: the FP32 policy against an oracle sample on history ids
  DISJOINT from the GPU's (ORACLE_FIRST onwards): it scores z = (m1 - m2) /
  sqrt(v1 + v2), which assumes the two samples are independent.  With shared ids
  most histories coincide and that statistic would be far too forgiving.
* paired_fp32_fp64: the FP32 and FP64 GPU policies on the SAME ids; per bin the
  difference of the two tallies is scored against the paired variance
  sum_h (x32_h - x64_h)^2 of the histories' own contributions (from their
  records), plus a stated FP32 rounding allowance.
"""
import numpy as np
from scipy import stats

from oracle import oracle as O
from paper_2304_06226_amd import binding as B

# first history id of the oracle samples that statistical comparisons run
# against: far from every id range a GPU test uses, so the samples are independent
ORACLE_FIRST = 1 << 40


def gpu_run(ctx, prob, first=0, n=None, precision="fp64", records=True):
    import torch
    n = prob.n_histories if n is None else n
    sim = B.Simulation(ctx, prob)
    rec = None
    if records:
        rec = torch.zeros(max(1, n) * B.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    ctx.reset_stats()
    sim.run(first=first, n=n, precision=precision, records=rec)
    torch.cuda.synchronize()
    res = sim.results()
    st = ctx.read_stats()
    recs = B.records_to_numpy(rec, n) if records else None
    return res, recs, st


def compare_records_fp64(g, o, min_identity=0.999):
    """Element-wise comparison of per-history records (FP64 policy vs oracle).
    Returns the boolean mask of histories with identical event sequences."""
    assert len(g) == len(o)
    same = g["hash"] == o["hash"]
    frac = same.mean() if len(g) else 1.0
    assert frac >= min_identity, f"event identity {frac:.5f} < {min_identity}"
    s = same
    assert np.array_equal(g["term"][s], o["term"][s])
    assert np.array_equal(g["n_scat"][s], o["n_scat"][s])
    assert np.array_equal(g["n_steps"][s], o["n_steps"][s])
    assert np.array_equal(g["n_draws"][s], o["n_draws"][s])
    assert np.array_equal(g["region"][s], o["region"][s])
    np.testing.assert_allclose(g["w"][s], o["w"][s], rtol=1e-11, atol=0)
    np.testing.assert_allclose(g["lambda"][s], o["lambda"][s], rtol=1e-13, atol=0)
    np.testing.assert_allclose(g["dir"][s], o["dir"][s], rtol=0, atol=1e-10)
    scale = np.maximum(1.0, np.abs(o["pos"][s]))
    assert np.all(np.abs(g["pos"][s] - o["pos"][s]) <= 1e-9 * scale)
    if g["tof"].any():   # the run tracked the time of flight (a chopper or a TOF tally)
        np.testing.assert_allclose(g["tof"][s], o["tof"][s], rtol=1e-6, atol=0)
    return same


def compare_tallies_fp64(gres, ores, grec, orec, same, weights_tol=1e-10):
    """Per-bin comparison: equal up to summation order, except for the weight of
    histories whose event sequence differs (bounded by their own weights)."""
    slack_w = np.abs(grec["w"][~same]).sum() + np.abs(orec["w"][~same]).sum() if same is not None else 0.0
    slack_w2 = (grec["w"][~same] ** 2).sum() + (orec["w"][~same] ** 2).sum() if same is not None else 0.0
    for t, (gsw, gsw2, gn) in enumerate(gres):
        osw, osw2 = ores.sumw[t], ores.sumw2[t]
        assert gn == ores.n
        tol = weights_tol * max(1.0, np.abs(osw).max()) + slack_w
        assert np.all(np.abs(gsw - osw) <= tol), (t, np.abs(gsw - osw).max(), tol)
        tol2 = weights_tol * max(1.0, np.abs(osw2).max()) + slack_w2
        assert np.all(np.abs(gsw2 - osw2) <= tol2), (t, np.abs(gsw2 - osw2).max(), tol2)


def merged_z(m1, v1, c1, m2, v2, c2, min_count=25):
    """Per-bin z-scores, merging adjacent bins until both sides hold min_count entries."""
    zs = []
    a = np.zeros(6)
    for i in range(len(m1)):
        a += (m1[i], v1[i], c1[i], m2[i], v2[i], c2[i])
        if a[2] >= min_count and a[5] >= min_count:
            var = a[1] + a[4]
            zs.append((a[0] - a[3]) / np.sqrt(var) if var > 0 else 0.0)
            a[:] = 0
    return np.array(zs)


def tally_stat_test(gsw, gsw2, gn, osw, osw2, on, min_count=25):
    """The tally agreement test between two INDEPENDENT samples (see the module
    docstring): chi^2 of merged-bin z-scores with p > 1e-3 and the count of
    |z| > 4 within the 99.9% binomial quantile."""
    gm, om = gsw / gn, osw / on
    gv = np.maximum(gsw2 / gn - gm * gm, 0) / max(gn - 1, 1)
    ov = np.maximum(osw2 / on - om * om, 0) / max(on - 1, 1)
    # effective entry counts (sum w)^2 / sum w^2
    gc = np.where(gsw2 > 0, gsw ** 2 / np.where(gsw2 > 0, gsw2, 1), 0)
    oc = np.where(osw2 > 0, osw ** 2 / np.where(osw2 > 0, osw2, 1), 0)
    z = merged_z(gm, gv, gc, om, ov, oc, min_count)
    if len(z) == 0:
        return 1.0, z
    chi2 = float((z ** 2).sum())
    p = float(stats.chi2.sf(chi2, len(z)))
    n_big = int((np.abs(z) > 4).sum())
    limit = int(stats.binom.ppf(0.999, len(z), 6.3e-5))
    assert n_big <= limit, (n_big, limit)
    return p, z


_TERM = {"escape": B.END_ESCAPE, "absorb": B.END_ABSORB, "detect": B.END_DETECT}


def record_bins(tally, rec, edge_rel=0.0):
    """Flat bin of every history's score in `tally` (a workloads.Tally), computed
    here in numpy from the history's record (-1: not scored), and the flat
    indices of the neighbouring bins (columns per axis and side, -1: none) that
    another precision may round the history to: those across an edge lying
    within edge_rel (relative to the value, plus 1e-12 of the axis range)."""
    n = len(rec)
    ok = rec["term"] == _TERM[tally.trigger]
    if tally.trigger == "detect" and tally.trigger_volume >= 0:
        ok &= rec["region"] == tally.trigger_volume
    ns = rec["n_scat"]
    if tally.filter == "unscattered":
        ok &= ns == 0
    elif tally.filter == "scattered":
        ok &= ns >= 1
    elif tally.filter == "nscat_eq":
        ok &= ns == tally.filter_arg
    beam = np.asarray(tally.beam, dtype=np.float64)
    beam = beam / np.linalg.norm(beam)
    d = rec["dir"]
    c = np.clip(d @ beam, -1.0, 1.0)
    flat = np.zeros(n, dtype=np.int64)
    strides = []
    for a in tally.axes:
        strides = [st * a.nbins for st in strides] + [1]
    alts = []
    near_out = np.zeros(n, dtype=bool)
    for a, stride in zip(tally.axes, strides):
        q = a.quantity
        if q == "theta2":
            x = np.degrees(np.arccos(c))
        elif q == "lambda":
            x = rec["lambda"]
        elif q in ("x", "y", "z"):
            x = rec["pos"][:, "xyz".index(q)]
        elif q == "div_x":
            x = np.degrees(np.arctan2(d[:, 0], d[:, 2]))
        elif q == "div_y":
            x = np.degrees(np.arctan2(d[:, 1], d[:, 2]))
        elif q == "nscat":
            x = ns.astype(np.float64)
        elif q == "q":
            x = 4 * np.pi / rec["lambda"] * np.sqrt((1 - c) / 2)
        else:
            x = rec["tof"].astype(np.float64)
        pos = (x - a.lo) / (a.hi - a.lo) * a.nbins
        inside = (x >= a.lo) & (x <= a.hi)
        b = np.clip(np.floor(pos).astype(np.int64), 0, a.nbins - 1)
        b = np.where(x == a.hi, a.nbins - 1, b)
        tol = (edge_rel * np.abs(x) + 1e-12 * (a.hi - a.lo)) / (a.hi - a.lo) * a.nbins
        frac = pos - np.floor(pos)
        lo_edge = inside & (frac <= tol) & (b > 0)
        hi_edge = inside & (1 - frac <= tol) & (b < a.nbins - 1)
        alts.append((lo_edge, -stride))
        alts.append((hi_edge, +stride))
        # values within rounding outside the range may be scored by another precision
        near_out |= ~inside & ((np.abs(x - a.lo) <= tol * (a.hi - a.lo) / a.nbins) |
                               (np.abs(x - a.hi) <= tol * (a.hi - a.lo) / a.nbins))
        ok &= inside
        flat = flat * a.nbins + b
    flat = np.where(ok, flat, -1)
    alt = np.full((n, len(alts)), -1, dtype=np.int64)
    for j, (m, off) in enumerate(alts):
        alt[:, j] = np.where(ok & m, flat + off, -1)
    return flat, alt, near_out


def paired_variance(tally, rec32, rec64, edge_rel32=2e-6, edge_rel64=2e-7):
    """Per-bin paired variance sum_h (x32_h - x64_h)^2 of the two policies'
    per-history contributions.  A history whose value lies within edge_rel of a
    bin edge counts its weight in the neighbouring bin too: its bin is uncertain
    at that distance (FP32 arithmetic on the FP32 side; on the FP64 side the
    record's time of flight, rounded to FP32)."""
    nb = tally.nbins
    b32, alt32, out32 = record_bins(tally, rec32, edge_rel32)
    b64, alt64, out64 = record_bins(tally, rec64, edge_rel64)
    w32, w64 = rec32["w"], rec64["w"]
    V = np.zeros(nb)
    uncertain = (alt32 >= 0).any(axis=1) | out32 | (alt64 >= 0).any(axis=1) | out64
    same = (b32 == b64) & (b32 >= 0) & ~uncertain
    np.add.at(V, b32[same], (w32[same] - w64[same]) ** 2)
    m = (b32 >= 0) & ~same
    np.add.at(V, b32[m], w32[m] ** 2)
    m = (b64 >= 0) & ~same
    np.add.at(V, b64[m], w64[m] ** 2)
    for alt, w in ((alt32, w32), (alt64, w64)):
        for j in range(alt.shape[1]):
            m = alt[:, j] >= 0
            np.add.at(V, alt[m, j], w[m] ** 2)
    return V


def paired_check(prob, r32, rec32, r64, rec64, rel_round=2e-5, label=""):
    """FP32 tallies r32 against FP64 tallies r64 of the same history ids (records
    rec32, rec64 of those histories): every bin's difference within 4 paired
    standard deviations (plus a relative FP32 rounding allowance rel_round of the
    bin), with the count of larger deviations within the 99.9% binomial quantile
    of (bins, 6.3e-5), and each tally's total within 4 paired standard deviations
    plus rel_round.  The rounding allowance is systematic, not statistical: the
    FP32 policy evaluates cross sections and flight exponents in FP32, so one
    rounding of (g - 1) Sigma is shared by every step of every history of a
    material; at large bias factors and path lengths it shifts the weights by up
    to ~1e-5 relative.  Returns per tally (total relative difference, moved
    fraction sum|D| / sum|w64|) for reporting."""
    out = []
    n = len(rec32)
    for t, tally in enumerate(prob.tallies):
        (w32, _, n32), (w64, _, n64) = r32[t], r64[t]
        assert n32 == n64 == n, (label, t, n32, n64, n)
        V = paired_variance(tally, rec32, rec64)
        D = w32 - w64
        den = np.sqrt(V + (rel_round * np.abs(w64)) ** 2)
        bad = np.abs(D) > 4 * den + 1e-300
        used = (V > 0) | (w64 != 0) | (w32 != 0)
        limit = int(stats.binom.ppf(0.999, max(1, int(used.sum())), 6.3e-5))
        assert int(bad.sum()) <= limit, (label, t, int(bad.sum()), limit, np.nonzero(bad)[0][:10], D[bad][:10],
                                         den[bad][:10])
        tot = np.abs(w64).sum()
        if tot > 0:
            assert abs(D.sum()) <= 4 * np.sqrt(V.sum()) + rel_round * tot, (label, t, D.sum(), np.sqrt(V.sum()), tot)
            out.append((float(D.sum() / tot), float(np.abs(D).sum() / tot)))
        else:
            assert np.all(w32 == 0), (label, t)
            out.append((0.0, 0.0))
    print(f"[paired] {label or prob.name}: " + ", ".join(f"tally {t}: total {a:+.2e} moved {b:.2e}"
                                                        for t, (a, b) in enumerate(out)), flush=True)
    return out


def paired_fp32_fp64(ctx, prob, first, n, fp64="fp64_persistent", rel_round=2e-5, label=""):
    """Both GPU policies over the same history ids with records, then paired_check."""
    print(f"[case] paired {label or prob.name} n={n} first={first}", flush=True)
    r32, rec32, st32 = gpu_run(ctx, prob, first=first, n=n, precision="fp32")
    r64, rec64, st64 = gpu_run(ctx, prob, first=first, n=n, precision=fp64)
    assert st32["histories"] == st64["histories"] == n
    assert st32["capped"] == 0
    return paired_check(prob, r32, rec32, r64, rec64, rel_round, label)
