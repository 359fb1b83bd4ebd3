"""Pins of the oracle's design-density path and of its dual-number derivative.

The adjoint gradient of the library is checked against the oracle's exact
directional derivative (dual numbers carried through every step).  These
tests pin that oracle machinery to things other than itself:

* the dual-number derivative of sigma_ext equals central differences of the
  plain (real-valued) oracle objective, along a random design direction and
  along single voxels;
* the density interpolation (wp^2 -> rho wp^2, beta^2 -> rho beta^2, D -> rho
  D, gamma unchanged): a uniform density rho reproduces a plain metal run
  with those scaled parameters; rho = 1 reproduces the plain metal bitwise;
  rho = 0 leaves P_f identically zero and E equal to the empty grid's.
"""
import numpy as np

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask, oracle_mask_and_weight, oracle_problem, rel_l2

THREADS = 2


def design(steps=200, **kw):
    w = W.early_pulse(W.dimer_design(0, n=34, r=0.75e-9, gap=0.25e-9, design=8, npml=4,
                                     steps=steps, precision="fp64", **kw))
    w.omega = W.spectrum_omegas(6, 2.0, 4.5)
    return w


def objective(w, mask, weight, m):
    s = orc.OracleSim(oracle_problem(w, threads=THREADS), mask, weight)
    s.run(w.steps)
    v = s.spectra()["ext"][m]
    s.close()
    return v


def test_dual_derivative_matches_central_differences():
    """d sigma_ext / dt along w + t v: dual numbers against (L(+h) - L(-h)) / 2h
    of the real-valued run.  The central difference has an O(h^2) error; with
    h = 1e-4 on O(1) weights it is far below the 1e-6 bound."""
    w = design()
    m = 3
    mask, weight = oracle_mask_and_weight(w)
    p = oracle_problem(w, threads=THREADS)
    (x0, y0, z0), (x1, y1, z1) = w.design_lo, w.design_hi
    dirs = []
    v = np.zeros_like(weight)
    v[z0:z1, y0:y1, x0:x1] = W.design_direction(np.asarray(w.rho).shape, 7)
    dirs.append(("random", v))
    # single voxels: the one in the gap on the axis, and one at a corner
    for q in (((z0 + z1) // 2, (y0 + y1) // 2, (x0 + x1) // 2), (z0, y0 + 1, x1 - 1)):
        e = np.zeros_like(weight)
        e[q] = 1.0
        dirs.append((f"voxel {q}", e))
    h = 1e-4
    for name, v in dirs:
        val, der = orc.directional(p, mask, weight, v, w.steps, m)
        lp = objective(w, mask, weight + h * v, m)
        lm = objective(w, mask, weight - h * v, m)
        fd = (lp - lm) / (2 * h)
        print(f"{name}: dual {der:.12e} fd {fd:.12e}")
        assert abs(val - objective(w, mask, weight, m)) <= 1e-14 * abs(val)
        assert der != 0.0
        assert abs(der - fd) <= 1e-6 * abs(fd), (name, der, fd)


def _run(w, mask, weight, steps):
    s = orc.OracleSim(oracle_problem(w, threads=THREADS), mask, weight)
    s.run(steps)
    out = {f: s.get(f) for f in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Px", "Py", "Pz")}
    out["spec"] = s.spectra()
    s.close()
    return out


def test_uniform_density_equals_scaled_material():
    """rho = 0.5 on the design box equals a plain metal box whose wp^2, beta^2
    and D are halved (gamma unchanged): the interpolation of the design
    reading.  A density that also scaled gamma, or missed beta^2 or D, moves
    the fields by far more than the 1e-12 bound."""
    w = design(steps=300)
    mask, weight = oracle_mask_and_weight(w)
    (x0, y0, z0), (x1, y1, z1) = w.design_lo, w.design_hi
    # design box only (the fixed dimer outside it removed), so that the whole
    # metal carries the one density
    box = np.zeros_like(mask)
    box[z0:z1, y0:y1, x0:x1] = 7
    wt = np.zeros_like(weight)
    wt[z0:z1, y0:y1, x0:x1] = 0.5
    a = _run(w, box, wt, w.steps)
    ws = design(steps=300)
    ws.wp, ws.beta, ws.diff = w.wp * np.sqrt(0.5), w.beta * np.sqrt(0.5), w.diff * 0.5
    b = _run(ws, box, None, w.steps)
    for f in ("Ex", "Ez", "Hy", "Px", "Pz"):
        e = rel_l2(a[f], b[f])
        print(f"{f}: {e:.2e}")
        assert e <= 1e-12, f
    assert np.abs(a["Pz"]).max() > 0  # the longitudinal (nonlocal) part is active
    # the same density with gamma halved as well is visibly different
    ws.gamma = w.gamma * 0.5
    c = _run(ws, box, None, w.steps)
    assert rel_l2(a["Px"], c["Px"]) > 1e-6


def test_density_one_is_plain_metal_and_zero_is_vacuum():
    w = design(steps=250)
    (x0, y0, z0), (x1, y1, z1) = w.design_lo, w.design_hi
    box = np.zeros(oracle_mask(w).shape, np.uint8)
    box[z0:z1, y0:y1, x0:x1] = 7
    one = np.zeros(box.shape)
    one[z0:z1, y0:y1, x0:x1] = 1.0
    a = _run(w, box, one, w.steps)
    b = _run(w, box, None, w.steps)
    for f in a:
        if f == "spec":
            for k in a[f]:
                assert np.array_equal(a[f][k], b[f][k]), k
        else:
            assert np.array_equal(a[f], b[f]), f
    zero = np.zeros(box.shape)
    c = _run(w, box, zero, w.steps)
    empty = _run(w, np.zeros_like(box), None, w.steps)
    for f in ("Px", "Py", "Pz"):
        assert not np.any(c[f]), f
    # E_y, E_z, H_x, H_z of the empty grid are rounding-level (x-polarised
    # normal incidence): measure every difference against the field's scale
    escale, hscale = np.linalg.norm(empty["Ex"]), np.linalg.norm(empty["Hy"])
    for f in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"):
        scale = escale if f[0] == "E" else hscale
        assert np.linalg.norm(c[f] - empty[f]) <= 1e-13 * scale, f
    assert escale > 0 and hscale > 0
