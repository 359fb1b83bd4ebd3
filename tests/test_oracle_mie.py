"""Pins of the oracle against Mie theory for spheres (Sec. V compares the
FDTD spectra of small spheres with Mie results, local and nonlocal).

1. Local Drude sphere (beta = D = 0): the oracle's extinction cross section
   (induced-current route, TF/SF source) against the full Mie series for the
   same permittivity eps(w) = 1 - wp^2 / (w (w + i gamma)) in vacuum.
2. Hydrodynamic sphere (D = 0): the blueshift of the dipole resonance with
   respect to the local sphere against the quasi-static nonlocal dipole
   polarisability, at radii 10 and 6 nm: the shift grows as the radius
   shrinks, in the theory's proportion.

The grids are coarse (dx = 1 nm, spheres of 10 and 6 cells) and beta is
exaggerated (2e7 m/s) so that the longitudinal decay length
beta / sqrt(wp^2 - w^2), about 2.4 nm, spans a few cells.  The local
resonance then agrees with Mie to about 1 %.  The blueshift converges from
below as the decay length is resolved: 0.53, 0.75 and 0.81 of the dipole
theory at beta = 1e7, 2e7 and 3e7 m/s on this grid, so it is held to
[0.6, 1.05] of the theory; the ratio of the shifts at the two radii does
not depend on that factor and matches the theory's within 10 % (measured
1.98 against 1.99).  Plausible mistakes move the local resonance by far
more (wp^2 off by 2: 30 %), change the cross section by a factor
(normalisation), or shift the nonlocal resonance the wrong way (the sign
of the pressure term).
"""
import math

import numpy as np
from scipy.special import spherical_jn, spherical_yn

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask, oracle_problem

WP, GAMMA, BETA = 1.0e16, 2.0e15, 2.0e7
C0 = 299792458.0
OMEGA = W.spectrum_omegas(191, 2.8, 6.6)


def eps_drude(w):
    return 1.0 - WP ** 2 / (w * (w + 1j * GAMMA))


def mie_extinction(eps, a, w, nmax=8):
    """Full Mie extinction cross section (m^2) of a sphere of radius a and
    relative permittivity eps in vacuum; Riccati-Bessel functions
    psi_n(z) = z j_n(z), xi_n(z) = z h_n^(1)(z), time factor e^{-i w t}."""
    k = w / C0
    x = k * a
    m = np.sqrt(eps + 0j)
    mx = m * x
    s = 0.0
    for n in range(1, nmax + 1):
        jx, djx = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
        yx, dyx = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
        jm, djm = spherical_jn(n, mx), spherical_jn(n, mx, derivative=True)
        psi_x, dpsi_x = x * jx, jx + x * djx
        xi_x, dxi_x = x * (jx + 1j * yx), (jx + 1j * yx) + x * (djx + 1j * dyx)
        psi_m, dpsi_m = mx * jm, jm + mx * djm
        an = (m * psi_m * dpsi_x - psi_x * dpsi_m) / (m * psi_m * dxi_x - xi_x * dpsi_m)
        bn = (psi_m * dpsi_x - m * psi_x * dpsi_m) / (psi_m * dxi_x - m * xi_x * dpsi_m)
        s += (2 * n + 1) * (an + bn).real
    return 2.0 * math.pi / k ** 2 * s


def quasistatic_extinction(a, w, beta):
    """Dipole extinction k Im(alpha) + k^4 |alpha|^2 / (6 pi) of a small
    sphere; with beta > 0 the hydrodynamic (nonlocal) dipole polarisability
    alpha = 4 pi a^3 (eps - (1 + d)) / (eps + 2 (1 + d)),
    d = (eps - 1) j_1(kL a) / (kL a j_1'(kL a)), kL^2 = (w (w + i gamma) - wp^2) / beta^2
    (eps_inf = 1, vacuum background); d = 0 is the local sphere."""
    eps = eps_drude(w)
    d = 0.0
    if beta > 0:
        z = np.sqrt((w * (w + 1j * GAMMA) - WP ** 2) + 0j) / beta * a
        d = (eps - 1.0) * spherical_jn(1, z) / (z * spherical_jn(1, z, derivative=True))
    alpha = 4.0 * math.pi * a ** 3 * (eps - (1.0 + d)) / (eps + 2.0 * (1.0 + d))
    k = w / C0
    return k * alpha.imag + k ** 4 * abs(alpha) ** 2 / (6.0 * math.pi)


def peak(w, s):
    """Resonance frequency: the maximum refined by a parabola through its
    neighbours."""
    i = int(np.argmax(s))
    assert 0 < i < len(s) - 1, "resonance at the edge of the band"
    y0, y1, y2 = s[i - 1], s[i], s[i + 1]
    t = 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)
    return w[i] + t * (w[i + 1] - w[i])


_RUNS = {}


def oracle_extinction(n, a_cells, beta):
    key = (n, a_cells, beta)
    if key not in _RUNS:
        dx = 1.0e-9
        w = W.sphere_problem(f"mie_{n}_{a_cells}", n, dx, 6, [(n - 1) / 2.0] * 3, a_cells * dx,
                             steps=6000, precision="fp64")
        w = W.early_pulse(w)
        w.wp, w.gamma, w.beta, w.diff, w.eps_inf = WP, GAMMA, beta, 0.0, 1.0
        w.omega = OMEGA
        w.flux = False
        s = orc.OracleSim(oracle_problem(w, threads=8), oracle_mask(w))
        s.run(w.steps)
        _RUNS[key] = np.asarray(s.spectra()["ext"], dtype=np.float64)
        s.close()
    return _RUNS[key]


def test_mie_series_reduces_to_the_dipole_limit():
    """The reference itself: for ka -> 0 the Mie series equals the local
    quasi-static dipole result."""
    a = 1.0e-9
    for w in OMEGA[::10]:
        m = mie_extinction(eps_drude(w), a, w)
        q = quasistatic_extinction(a, w, 0.0)
        assert abs(m - q) <= 2e-3 * abs(q), (w, m, q)


def test_local_drude_sphere_against_mie():
    a_cells = 10
    ext = oracle_extinction(46, a_cells, 0.0)
    a = a_cells * 1.0e-9
    mie = np.array([mie_extinction(eps_drude(w), a, w) for w in OMEGA])
    wf, wm = peak(OMEGA, ext), peak(OMEGA, mie)
    print(f"local a = 10 nm: FDTD peak {wf:.4e}, Mie {wm:.4e} rad/s; "
          f"heights {ext.max():.3e} / {mie.max():.3e} m^2")
    assert abs(wf - wm) <= 0.03 * wm
    assert abs(ext.max() - mie.max()) <= 0.15 * mie.max()
    assert np.linalg.norm(ext - mie) <= 0.25 * np.linalg.norm(mie)


def test_hydrodynamic_blueshift_against_nonlocal_dipole_theory():
    shifts, theory = {}, {}
    for n, a_cells in ((46, 10), (38, 6)):
        a = a_cells * 1.0e-9
        loc = peak(OMEGA, oracle_extinction(n, a_cells, 0.0))
        nl = peak(OMEGA, oracle_extinction(n, a_cells, BETA))
        q_loc = peak(OMEGA, np.array([quasistatic_extinction(a, w, 0.0) for w in OMEGA]))
        q_nl = peak(OMEGA, np.array([quasistatic_extinction(a, w, BETA) for w in OMEGA]))
        fd, th = nl - loc, q_nl - q_loc
        shifts[a_cells], theory[a_cells] = fd, th
        print(f"a = {a_cells} nm: FDTD blueshift {fd:.3e}, nonlocal dipole theory {th:.3e} rad/s "
              f"(ratio {fd / th:.2f})")
        assert th > 0
        assert 0.6 * th <= fd <= 1.05 * th
    scaling, scaling_th = shifts[6] / shifts[10], theory[6] / theory[10]
    print(f"shift ratio a = 6 / a = 10 nm: FDTD {scaling:.3f}, theory {scaling_th:.3f}")
    assert abs(scaling - scaling_th) <= 0.1 * scaling_th
