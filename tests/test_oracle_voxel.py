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


def _round_cone_distance(s, q, h, r1, r2, th):
    """Signed distance, in the (axial s, radial q >= 0) half-plane, to the
    convex hull of the balls B(0, r1) and B(h e, r2) whose common tangent
    cone has half-angle th (r1 - r2 = h sin th): behind the tangent point
    of the first ball its sphere, beyond that of the second ball its
    sphere, in between the straight flank."""
    a = s * np.cos(th) - q * np.sin(th)
    d = s * np.sin(th) + q * np.cos(th) - r1
    d = np.where(a < 0.0, np.sqrt(s * s + q * q) - r1, d)
    d = np.where(a > h * np.cos(th), np.sqrt((s - h) ** 2 + q * q) - r2, d)
    return d


def test_star_mask_matches_round_cone_distance():
    """Every P point of the star farther than 1e-3 dx from the surface is
    inside the oracle's mask iff its signed distance to the star is negative.

    The star is built here from its description alone: a sphere of radius R
    and, per tip, a cone of half-angle th ending in a rounded apex of radius
    r_tip whose far point lies L past the sphere surface.  The tip solid is
    the convex hull of the apex ball (centre h = R + L - r_tip on the axis)
    and the ball at the centre of radius r_tip + h sin th, which has the same
    flank; the two solids differ only inside the central sphere (checked
    below), so the union is the same set.  A sine used for a tangent (or the
    reverse) anywhere in the cone radius moves the flank by whole cells."""
    w = W.config3(seed=1, n=200, dx=0.4e-9)
    d = w.star
    th = np.radians(15.0)  # the workload's half-angle
    assert np.isclose(d[5], np.tan(th)) and np.isclose(d[6], np.sin(th))
    c, R, rt = d[:3] / w.dx, d[3] / w.dx, d[4] / w.dx
    m = orc.voxelize_star(w.nx, w.ny, w.nz, w.dx, d)
    near_total = 0
    for comp in range(3):
        x, y, z = _positions(m.shape, comp)
        ox, oy, oz = x - c[0], y - c[1], z - c[2]
        r2 = ox * ox + oy * oy + oz * oz
        dist = np.sqrt(r2) - R
        for t in range(int(d[7])):
            ax = d[8 + 4 * t: 11 + 4 * t]
            L = d[11 + 4 * t] / w.dx
            h = R + L - rt
            r1 = rt + h * np.sin(th)
            # the hull's base ball and the cone's base disc lie inside the sphere
            assert r1 < R and (h + rt / np.sin(th)) * np.tan(th) < R
            s = ox * ax[0] + oy * ax[1] + oz * ax[2]
            q = np.sqrt(np.maximum(r2 - s * s, 0.0))
            dist = np.minimum(dist, _round_cone_distance(s, q, h, r1, rt, th))
        far = np.abs(dist) > 1e-3
        near_total += int((~far).sum())
        bit = ((m >> comp) & 1).astype(bool)
        assert np.array_equal(bit[far], (dist < 0)[far]), comp
        assert bit.sum() > 0
    assert near_total < 1e-4 * 3 * m.size
