"""Pins of the oracle's dielectric substrate: a half-space z > sub_k of
relative permittivity eps_sub beside the background eps_b (the layered
backgrounds of Sec. V's comparisons, and the substrates for which Sec. III
discusses source and boundary treatment).  E_x and E_y on the interface plane
take the mean of the two permittivities; the 1D incident line carries the
same layers, so the TF/SF source injects the layered plane-wave solution.

1. With no particle, the total field inside the TF box is the line's field
   through the interface, and the scattered-field region stays at rounding.
2. The line's reflection from the interface (run with the substrate minus
   the run without, over the incident spectrum) has the Fresnel magnitude
   |(n_b - n_s) / (n_b + n_s)| at normal incidence, to the discretisation
   error of a few cells per wavelength.
"""
import math

import numpy as np

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_problem

EPS_SUB = 2.25  # n = 1.5, a glass-like substrate


def test_substrate_keeps_the_scattered_region_empty():
    n = 30
    dx = 5e-9
    w = W.early_pulse(W.sphere_problem("substrate_tfsf", n, dx, 4, [(n - 1) / 2.0] * 3, 3 * dx))
    w.eps_sub, w.sub_k = EPS_SUB, n // 2  # the interface crosses the TF box
    p = oracle_problem(w, flux=False, omega=np.zeros(0))
    s = orc.OracleSim(p, np.zeros((n, n, n), np.uint8))
    lo, hi = w.tf_lo, w.tf_hi
    assert lo[2] < w.sub_k < hi[2]
    off = int(orc.constants()["aux_off"])
    worst_sf = worst_tf = peak = 0.0
    for _ in range(12):
        s.run(40)
        Ex = s.get("Ex")
        e1, _h1 = s.aux()
        tf = np.zeros_like(Ex, dtype=bool)
        tf[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0]] = True
        inc = e1[np.arange(n) + off][:, None, None] * np.ones((1, n, n))
        worst_sf = max(worst_sf, np.abs(Ex[~tf]).max(), np.abs(s.get("Ey")).max(), np.abs(s.get("Ez")).max())
        worst_tf = max(worst_tf, np.abs(Ex[tf] - inc[tf]).max())
        peak = max(peak, np.abs(e1).max())
    assert peak > 0.1
    assert worst_sf <= 1e-13 * peak, worst_sf / peak
    assert worst_tf <= 1e-13 * peak, worst_tf / peak


def _line_series(eps_sub, steps, z_obs):
    n, nz, dx = 16, 200, 2e-9
    w = W.Workload(name="line", nx=n, ny=n, nz=nz, dx=dx, npml=4)
    w.tf_lo, w.tf_hi = (5, 5, 5), (10, 10, nz - 6)
    w.norm_k = 5
    w.eps_sub, w.sub_k = eps_sub, 120
    p = oracle_problem(w, flux=False, omega=np.zeros(0))
    s = orc.OracleSim(p, np.zeros((nz, n, n), np.uint8))
    off = int(orc.constants()["aux_off"])
    out = np.empty(steps)
    for q in range(steps):
        s.run(1)
        out[q] = s.aux()[0][z_obs + off]
    return out, s.dt


def test_line_reflection_has_the_fresnel_magnitude():
    steps, z_obs = 3000, 40
    with_sub, dt = _line_series(EPS_SUB, steps, z_obs)
    without, _ = _line_series(0.0, steps, z_obs)
    refl = with_sub - without  # the reflected wave at the observation plane
    assert np.abs(refl).max() > 1e-3 * np.abs(without).max()
    nb, ns = 1.0, math.sqrt(EPS_SUB)
    r = abs((nb - ns) / (nb + ns))
    t = np.arange(steps) * dt
    worst = 0.0
    for ev in np.linspace(1.5, 4.0, 11):
        om = W.ev_to_rad(ev)
        ph = np.exp(1j * om * t)
        ratio = abs(np.sum(refl * ph)) / abs(np.sum(without * ph))
        worst = max(worst, abs(ratio - r))
    print(f"Fresnel |r| = {r:.5f}; worst deviation 1.5-4 eV: {worst:.2e}")
    assert worst <= 1e-3
