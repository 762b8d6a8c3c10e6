"""Pins of the oracle's ray-solid intersection against brute-force ray marching.

For random rays, the union of the oracle's intervals must equal the set of
ray parameters whose points lie inside the solid, with inside-ness decided here
by a separate numpy point test written from the solid definitions (box of full
sides, finite cylinder, open-ended cylindrical shell, sphere, spherical shell).
Face ids are checked at the interval ends.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_06226_amd.workloads import Volume


def inside_np(v, pts):
    q = pts - np.asarray(v.center)
    if v.kind == "box":
        return np.all(np.abs(q) <= 0.5 * np.asarray(v.size[:3]), axis=1)
    a = v.axis
    b, c = (a + 1) % 3, (a + 2) % 3
    if v.kind == "cylinder":
        return (q[:, b] ** 2 + q[:, c] ** 2 <= v.size[0] ** 2) & (np.abs(q[:, a]) <= 0.5 * v.size[1])
    if v.kind == "cyl_shell":
        rho2 = q[:, b] ** 2 + q[:, c] ** 2
        return (rho2 >= v.size[0] ** 2) & (rho2 <= v.size[1] ** 2) & (np.abs(q[:, a]) <= 0.5 * v.size[2])
    r2 = (q ** 2).sum(axis=1)
    if v.kind == "sphere":
        return r2 <= v.size[0] ** 2
    return (r2 >= v.size[0] ** 2) & (r2 <= v.size[1] ** 2)


SOLIDS = [
    Volume("box", (1.0, -2.0, 3.0), (10.0, 4.0, 7.0)),
    Volume("cylinder", (0.5, 0.0, -1.0), (5.0, 20.0), axis=1),
    Volume("cylinder", (0.0, 0.0, 0.0), (3.0, 6.0), axis=0),
    Volume("cyl_shell", (0.0, 1.0, 0.0), (10.0, 11.0, 40.0), axis=1),
    Volume("cyl_shell", (0.0, 0.0, 0.0), (4.0, 9.0, 8.0), axis=2),
    Volume("sphere", (0.0, 0.0, 2.0), (7.0,)),
    Volume("sph_shell", (1.0, 1.0, 1.0), (5.0, 8.0)),
]


@pytest.mark.parametrize("vol", SOLIDS, ids=[f"{v.kind}{i}" for i, v in enumerate(SOLIDS)])
def test_intervals_match_ray_marching(vol):
    rng = np.random.default_rng(11)
    span = 60.0
    ts = np.linspace(-span, span, 24001)
    dt = ts[1] - ts[0]
    checked = 0
    for _ in range(300):
        p = rng.uniform(-15, 15, 3)
        u = rng.normal(size=3)
        if rng.random() < 0.6:   # aim at a point near the solid's centre
            u = np.asarray(vol.center) + rng.normal(scale=3.0, size=3) - p
        if rng.random() < 0.2:   # rays parallel to a coordinate axis exercise the u == 0 branches
            u = np.zeros(3)
            u[rng.integers(3)] = rng.choice([-1.0, 1.0])
        u /= np.linalg.norm(u)
        iv = O.intervals(vol, p, u)
        pts = p[None, :] + ts[:, None] * u[None, :]
        ins = inside_np(vol, pts)
        mask = np.zeros_like(ins)
        for a, b, fa, fb in iv:
            assert a <= b
            mask |= (ts >= a) & (ts <= b)
        near = np.zeros_like(ins)
        for a, b, _, _ in iv:
            near |= (np.abs(ts - a) < 2 * dt) | (np.abs(ts - b) < 2 * dt)
        bad = (ins != mask) & ~near
        assert not bad.any(), (vol.kind, p, u, iv)
        # midpoints are inside, pieces are disjoint and ordered
        for i, (a, b, _, _) in enumerate(iv):
            if np.isfinite(a) and np.isfinite(b) and b - a > 1e-9:
                assert inside_np(vol, (p + 0.5 * (a + b) * u)[None, :])[0]
            if i > 0:
                assert iv[i - 1][1] <= a
        checked += len(iv)
    assert checked > 50


def _face_of_point(vol, x):
    """Which face constraint is active at point x (independent of the oracle)."""
    q = x - np.asarray(vol.center)
    if vol.kind == "box":
        s = 0.5 * np.asarray(vol.size)
        k = int(np.argmax(np.abs(np.abs(q) - s) * -1))
        return 2 * k + (1 if q[k] > 0 else 0)
    a = vol.axis
    b, c = (a + 1) % 3, (a + 2) % 3
    if vol.kind in ("cylinder", "cyl_shell"):
        h = vol.size[1] if vol.kind == "cylinder" else vol.size[2]
        rho = np.hypot(q[b], q[c])
        d_cap = abs(abs(q[a]) - 0.5 * h)
        d_out = abs(rho - (vol.size[0] if vol.kind == "cylinder" else vol.size[1]))
        d_in = abs(rho - vol.size[0]) if vol.kind == "cyl_shell" else np.inf
        m = min(d_cap, d_out, d_in)
        if m == d_cap:
            return 2 if q[a] > 0 else 1
        return 0 if m == d_out else 3
    r = np.linalg.norm(q)
    if vol.kind == "sphere":
        return 0
    return 0 if abs(r - vol.size[1]) < abs(r - vol.size[0]) else 3


@pytest.mark.parametrize("vol", SOLIDS, ids=[f"{v.kind}{i}" for i, v in enumerate(SOLIDS)])
def test_face_ids(vol):
    rng = np.random.default_rng(5)
    n = 0
    for _ in range(400):
        p = rng.uniform(-15, 15, 3)
        u = np.asarray(vol.center) + rng.normal(scale=3.0, size=3) - p
        u /= np.linalg.norm(u)
        for a, b, fa, fb in O.intervals(vol, p, u):
            if b - a < 1e-6:
                continue
            assert fa == _face_of_point(vol, p + a * u)
            assert fb == _face_of_point(vol, p + b * u)
            n += 1
    assert n > 50


def test_contains_agrees_with_numpy():
    rng = np.random.default_rng(3)
    for vol in SOLIDS:
        pts = rng.uniform(-15, 15, (500, 3))
        ref = inside_np(vol, pts)
        got = np.array([O.contains(vol, x) for x in pts])
        assert (ref == got).all()
