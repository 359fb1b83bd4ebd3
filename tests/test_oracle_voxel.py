"""Pins of the oracle's voxelisers (Pekar mask: a P component is updated iff
its own Yee point, Sec. III Table I, lies strictly inside the metal)."""
import numpy as np

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W


def _positions(shape, comp):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = x.astype(float); y = y.astype(float); z = z.astype(float)
    if comp == 0: x += 0.5
    if comp == 1: y += 0.5
    if comp == 2: z += 0.5
    return x, y, z


def test_sphere_mask_matches_brute_force_distance():
    n, dx = 40, 0.25e-9
    rng = np.random.default_rng(11)
    spheres = np.array([[19.3 * dx, 20.1 * dx, 18.7 * dx, 7.3 * dx],
                        [10.2 * dx, 9.6 * dx, 11.0 * dx, 3.1 * dx]])
    spheres[:, :3] += rng.uniform(-0.2, 0.2, size=(2, 3)) * dx
    m = orc.voxelize_spheres(n, n, n, dx, spheres)
    for comp in range(3):
        x, y, z = _positions((n, n, n), comp)
        inside = np.zeros(x.shape, bool)
        near = np.zeros(x.shape, bool)
        for cx, cy, cz, r in spheres / dx:
            d2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
            inside |= d2 < r * r
            near |= np.abs(d2 - r * r) < 1e-6 * r * r
        bit = ((m >> comp) & 1).astype(bool)
        assert np.array_equal(bit[~near], inside[~near])
        assert bit.sum() > 0
    # count vs volume of the big sphere
    r = spheres[0, 3] / dx
    count = int(((m >> 0) & 1).sum())
    vol = 4.0 / 3.0 * np.pi * (r ** 3 + (spheres[1, 3] / dx) ** 3)
    assert abs(count / vol - 1.0) < 3.0 / r


def test_star_mask_geometry():
    w = W.config3(seed=1, n=200, dx=0.4e-9)
    d = w.star
    m = orc.voxelize_star(w.nx, w.ny, w.nz, w.dx, d)
    c = d[:3]; R = d[3]; rt = d[4]
    # sphere interior: every P_x point within 0.9 R of the centre is metal
    x, y, z = _positions(m.shape, 0)
    r2 = (x * w.dx - c[0]) ** 2 + (y * w.dx - c[1]) ** 2 + (z * w.dx - c[2]) ** 2
    bit = (m & 1).astype(bool)
    assert bit[r2 < (0.9 * R) ** 2].all()
    # nothing farther than the longest tip
    Lmax = max(d[8 + 4 * t + 3] for t in range(6))
    assert not bit[r2 > (R + Lmax + 0.1e-9) ** 2].any()
    # points on each tip axis: inside just below the apex, outside beyond it
    for t in range(6):
        a = d[8 + 4 * t: 11 + 4 * t]; L = d[11 + 4 * t]
        for frac, expect in ((R + L - 0.7 * rt, 7), (R + L + 0.6 * rt, 0)):
            p = c + frac * a
            i, j, k = np.round(p / w.dx).astype(int)
            # the nearest node's three P points are within half a cell of p
            bits = int(m[k, j, i])
            if expect:
                assert bits != 0, (t, frac)
            else:
                assert bits == 0, (t, frac)
