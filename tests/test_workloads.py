"""Checks of the synthetic input generators (no transport arithmetic here)."""
import numpy as np

from paper_2304_06226_amd import workloads as W


def cubic_multiplicity(h, k, l):
    """Textbook m-3m multiplicities: {h00} 6, {hh0} 12, {hhh} 8, {hk0} 24, {hhl} 24, {hkl} 48."""
    n_zero = [h, k, l].count(0)
    distinct = len({h, k, l} - {0})
    if n_zero == 2:
        return 6
    if n_zero == 1:
        return 12 if distinct == 1 else 24
    if h == k == l:
        return 8
    if h == k or k == l or h == l:
        return 24
    return 48


def test_fcc_families_a4():
    d, m, reps = W.fcc_families(4.0, 0.5)
    assert len(d) == 26
    assert len(np.unique(np.round(d, 12))) == 22
    assert m.sum() == 536
    for (h, k, l), mm in zip(reps, m):
        assert h >= k >= l >= 0
        assert len({h % 2, k % 2, l % 2}) == 1
        assert mm == cubic_multiplicity(h, k, l)
    assert np.all(np.diff(d) <= 0)
    assert reps[0] == (1, 1, 1) and reps[1] == (2, 0, 0)
    # equal d: 511 before 333 (representatives descending)
    i511, i333 = reps.index((5, 1, 1)), reps.index((3, 3, 3))
    assert i511 + 1 == i333


def test_family_count_range():
    for a in (3.5, 4.05, 6.0):
        d, m, _ = W.fcc_families(a, 0.5)
        assert 19 <= len(d) <= 71
        assert d.min() >= 0.5


def test_seeded_materials_reproducible():
    a = W.sample_material()
    b = W.sample_material()
    assert np.array_equal(a.f2, b.f2)
    assert a.f2.min() >= 1.0 and a.f2.max() <= 10.0
    v = W.vessel_material()
    assert not np.array_equal(a.f2[:10], v.f2[:10])
    assert abs(v.number_density - 4 / 4.05 ** 3) < 1e-15


def test_configs_shapes():
    assert W.analog_sample().tallies[0].nbins == 1800
    assert W.biased_sample().tallies[0].shape == (1800, 100)
    assert W.vessel_sample().tallies[0].shape == (3600, 1000)
    assert W.m3_guide().tallies[0].nbins == 200 * 200 * 100 * 100
