"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark and the runner use (the stored FP32-mixed tuning of each workload, or
FP64 plain), checked on sampled
histories the oracle recomputes one by one, against closed forms, and against
oracle samples through the tally agreement test.
"""
import dataclasses

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2304_06226_amd import binding as B
from paper_2304_06226_amd import workloads as W
from paper_2304_06226_amd.tuning import TUNED

from parity import ORACLE_FIRST, compare_records_fp64, tally_stat_test

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = B.Context(device=0, seed=4096)
    yield c
    c.close()


def total_sigma(mat, lam):
    xs = O.macro_xs(mat, lam)
    return xs[0] + xs[1] + xs[2]


def _tuned(ctx, name):
    """Apply the stored tuning of workload `name`; returns the previous one."""
    base = ctx.get_tuning()
    ctx.set_tuning(**TUNED[name])
    return base


def test_biased_sample_full_1e7_fp32(ctx):
    import torch
    prob = W.biased_sample()
    n = prob.n_histories
    print(f"[case] biased sample fp32 n={n}", flush=True)
    sim = B.Simulation(ctx, prob)
    base = _tuned(ctx, "sample")
    try:
        ctx.reset_stats()
        sim.run(first=0, n=n, precision="fp32")
        torch.cuda.synchronize()
        res = sim.results()
        st = ctx.read_stats()
    finally:
        ctx.set_tuning(**base)
    assert st["histories"] == n and st["capped"] == 0
    # Beer-Lambert through the 10 mm diameter
    T = np.exp(-total_sigma(prob.materials[0], 1.8) * 10.0)
    sw, sw2, nh = res[1]
    m = sw[0] / nh
    v = (sw2[0] / nh - m * m) / (nh - 1)
    assert abs(m - T) / np.sqrt(v) < 4.0
    # every tally against an oracle sample of 2e6 histories
    o = O.run(prob, first=ORACLE_FIRST, n=2_000_000, threads=16)
    for t, (gw, gw2, gn) in enumerate(res):
        p, z = tally_stat_test(gw, gw2, gn, o.sumw[t], o.sumw2[t], o.n)
        assert p > 1e-3, (t, p)


def test_biased_sample_full_1e7_fp64_sampled_histories(ctx):
    import torch
    prob = W.biased_sample()
    n = prob.n_histories
    print(f"[case] biased sample fp64 n={n} with records", flush=True)
    sim = B.Simulation(ctx, prob)
    rec = torch.zeros(n * B.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    sim.run(first=0, n=n, precision="fp64", records=rec)
    torch.cuda.synchronize()
    g = B.records_to_numpy(rec, n)
    del rec
    ids = np.sort(np.random.default_rng(7).choice(n, size=2000, replace=False))
    o = np.concatenate([O.run(prob, first=int(h), n=1, threads=1, records=True).records for h in ids])
    same = compare_records_fp64(g[ids], o)
    assert same.mean() >= 0.999
    assert np.all(g["term"] > 0)


def test_vessel_full_1e8_fp32(ctx):
    import torch
    prob = W.vessel_sample()
    n = prob.n_histories
    print(f"[case] vessel fp32 n={n}", flush=True)
    sim = B.Simulation(ctx, prob)
    base = _tuned(ctx, "vessel")
    try:
        ctx.reset_stats()
        sim.run(first=0, n=n, precision="fp32")
        torch.cuda.synchronize()
        res = sim.results()
        st = ctx.read_stats()
    finally:
        ctx.set_tuning(**base)
    assert st["histories"] == n and st["capped"] == 0
    o = O.run(prob, first=ORACLE_FIRST, n=3_000_000, threads=16)
    for t, (gw, gw2, gn) in enumerate(res):
        if t == 0:
            # 2theta(3600) x lambda(1000): compare on 2theta(360) x lambda(50) blocks
            def coarse(a):
                return a.reshape(360, 10, 50, 20).sum(axis=(1, 3)).ravel()
            p, z = tally_stat_test(coarse(gw), coarse(gw2), gn, coarse(o.sumw[t]), coarse(o.sumw2[t]), o.n)
        else:
            p, z = tally_stat_test(gw, gw2, gn, o.sumw[t], o.sumw2[t], o.n)
        assert p > 1e-3, (t, p)


def _guide_coarse(ctx, tally, fine=(200, 200, 100, 100), coarse=(50, 50, 20, 20)):
    """Read a 4-D guide tally in slices of the first axis and sum it to coarse bins."""
    f0, f1, f2, f3 = fine
    c0, c1, c2, c3 = coarse
    r0, r1, r2, r3 = f0 // c0, f1 // c1, f2 // c2, f3 // c3
    outw = np.zeros(coarse)
    outw2 = np.zeros(coarse)
    row = f1 * f2 * f3
    for i in range(f0):
        w, w2 = ctx.read_tally_range(tally, i * row, row)
        outw[i // r0] += w.reshape(c1, r1, c2, r2, c3, r3).sum(axis=(1, 3, 5))
        outw2[i // r0] += w2.reshape(c1, r1, c2, r2, c3, r3).sum(axis=(1, 3, 5))
    return outw.ravel(), outw2.ravel()


def test_guide_full_1e8_fp32_full_tally(ctx):
    import torch
    prob = W.m3_guide()
    n = prob.n_histories
    print(f"[case] guide fp32 n={n}, 4e8-bin tally", flush=True)
    sim = B.Simulation(ctx, prob)
    assert ctx.tally_nbins(sim.tallies[0]) == 400_000_000
    base = _tuned(ctx, "guide")
    try:
        ctx.reset_stats()
        sim.run(first=0, n=n, precision="fp32")
        torch.cuda.synchronize()
        st = ctx.read_stats()
    finally:
        ctx.set_tuning(**base)
    assert st["histories"] == n and st["capped"] == 0
    gw, gw2 = _guide_coarse(ctx, sim.tallies[0])
    # the sparse 4-D tally is compared on coarse bins (x,y 50x50, divergences 20x20)
    # merged to >= 100 entries per group, where the per-group z is close to normal
    small = W.m3_guide(nbins_xy=50, nbins_div=20)
    o = O.run(small, first=ORACLE_FIRST, n=10_000_000, threads=16)
    p, z = tally_stat_test(gw, gw2, n, o.sumw[0], o.sumw2[0], o.n, min_count=100)
    assert p > 1e-3, p
    # surviving fraction: killed + escaped = all
    assert st["escaped"] + st["killed"] == n
    # the FP64 policy on the same histories (common random numbers): the FP32
    # rounding moves little weight (the paired statistical test with per-history
    # variances runs at 1e6 histories in test_gpu_paired)
    sim64 = B.Simulation(ctx, small)
    sim64.run(first=0, n=n, precision="fp64")
    torch.cuda.synchronize()
    w64, w64_2, _ = ctx.read_tally(sim64.tallies[0])
    assert abs(gw.sum() - w64.sum()) / w64.sum() < 1e-6
    assert np.abs(gw - w64).sum() / w64.sum() < 1e-3


def test_batch_full_closed_forms(ctx):
    import torch
    batch = W.sample_batch()
    print(f"[case] full batch: {len(batch.problems)} simulations, {batch.total_histories} histories", flush=True)
    br = B.BatchRun(ctx, batch)
    base = _tuned(ctx, "batch")
    try:
        ctx.reset_stats()
        br.run()
        torch.cuda.synchronize()
        st = ctx.read_stats()
    finally:
        ctx.set_tuning(**base)
    assert st["histories"] == batch.total_histories and st["capped"] == 0
    # transmitted counter of every powder simulation: exp(-Sigma_S 2r - Sigma_V 2 mm)
    zs = []
    for s, prob in zip(br.sims[:-1], batch.problems[:-1]):
        lam = prob.source.lam0
        r = prob.volumes[1].size[0]
        tau = total_sigma(prob.materials[0], lam) * 2 * r
        if len(prob.materials) > 1:
            tau += total_sigma(prob.materials[1], lam) * 2.0
        T = np.exp(-tau)
        sw, sw2, nh = s.ctx.read_tally(s.tallies[1])
        m = sw[0] / nh
        v = max(sw2[0] / nh - m * m, 0.0) / (nh - 1)
        if v > 0:
            zs.append((m - T) / np.sqrt(v))
    zs = np.array(zs)
    assert len(zs) > 200
    assert stats.chi2.sf((zs ** 2).sum(), len(zs)) > 1e-3
    assert np.abs(zs).max() < 5
    # imaging: unscattered image against the integral of exp(-tau(x, y)) over each 32x32 block
    prob = batch.problems[-1]
    s = br.sims[-1]
    sw, sw2, nh = s.ctx.read_tally(s.tallies[1])
    img = sw.reshape(512, 512)
    sig = [total_sigma(m, 2.0) for m in prob.materials]
    expect = unscattered_block_fraction(prob, sig, nblk=16)
    got = img.reshape(16, 32, 16, 32).sum(axis=(1, 3)) / nh            # unscattered fraction per block
    z = (got - expect) / np.sqrt(expect * (1 - expect) / nh)
    assert np.abs(z).max() < 4.5, np.abs(z).max()
    assert stats.chi2.sf((z ** 2).sum(), z.size) > 1e-3


def unscattered_block_fraction(prob, sig, nblk, half=250.0):
    """Exact probability that a source neutron (uniform over the 500x500 mm beam)
    reaches each of nblk x nblk detector blocks unscattered: exp(-tau(x, y)) is
    constant on the rectangles cut by the box edges and block boundaries, so the
    integral is a finite sum over those rectangles (tau from 2-D difference arrays)."""
    boxes = prob.volumes[1:-1]
    bounds = np.linspace(-half, half, nblk + 1)
    xe = [bounds]
    ye = [bounds]
    for v in boxes:
        cx, cy, _ = v.center
        sx, sy, _ = v.size
        xe.append(np.clip([cx - sx / 2, cx + sx / 2], -half, half))
        ye.append(np.clip([cy - sy / 2, cy + sy / 2], -half, half))
    xs = np.unique(np.concatenate(xe))
    ys = np.unique(np.concatenate(ye))
    diff = np.zeros((len(xs), len(ys)))
    for v in boxes:
        cx, cy, _ = v.center
        sx, sy, sz = v.size
        i0, i1 = np.searchsorted(xs, np.clip([cx - sx / 2, cx + sx / 2], -half, half))
        j0, j1 = np.searchsorted(ys, np.clip([cy - sy / 2, cy + sy / 2], -half, half))
        t = sig[v.material] * sz
        diff[i0, j0] += t
        diff[i1, j0] -= t
        diff[i0, j1] -= t
        diff[i1, j1] += t
    tau = np.cumsum(np.cumsum(diff, axis=0), axis=1)[:-1, :-1]
    area = np.outer(np.diff(xs), np.diff(ys))
    xc = 0.5 * (xs[1:] + xs[:-1])
    yc = 0.5 * (ys[1:] + ys[:-1])
    bi = np.minimum((xc + half) / (2 * half) * nblk, nblk - 1).astype(int)
    bj = np.minimum((yc + half) / (2 * half) * nblk, nblk - 1).astype(int)
    out = np.zeros((nblk, nblk))
    np.add.at(out, (bi[:, None].repeat(len(yc), 1), bj[None, :].repeat(len(xc), 0)), np.exp(-tau) * area)
    return out / (2 * half) ** 2


def test_paper_guide_full_1e8_fp32(ctx):
    """The paper's guide benchmark at its own size, 1e8 neutrons: the detected
    fraction and the rear-detector image (20x20 blocks) against a 1e7-history
    oracle sample."""
    import torch
    prob = W.paper_guide()
    n = prob.n_histories
    print(f"[case] paper guide fp32 n={n}", flush=True)
    sim = B.Simulation(ctx, prob)
    base = _tuned(ctx, "paper_guide")
    try:
        ctx.reset_stats()
        sim.run(first=0, n=n, precision="fp32")
        torch.cuda.synchronize()
        res = sim.results()
        st = ctx.read_stats()
    finally:
        ctx.set_tuning(**base)
    assert st["histories"] == n and st["capped"] == 0
    assert st["detected"] + st["escaped"] + st["absorbed"] + st["killed"] == n
    o = O.run(prob, first=ORACLE_FIRST, n=10_000_000, threads=16)

    def coarse(a):
        return a.reshape(20, 5, 20, 5).sum(axis=(1, 3)).ravel()
    gw, gw2, gn = res[0]
    p, z = tally_stat_test(coarse(gw), coarse(gw2), gn, coarse(o.sumw[0]), coarse(o.sumw2[0]), o.n)
    assert p > 1e-3, p
    gw, gw2, gn = res[1]
    p, z = tally_stat_test(gw, gw2, gn, o.sumw[1], o.sumw2[1], o.n)
    assert p > 1e-3, p
