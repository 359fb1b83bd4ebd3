"""Pins of the oracle's near-field and free-electron density maps (the field and
density distributions of Sec. V; the density is n - n0 = div P_NL / e, Eq.
Nsol).

1. The maps are running transforms by definition: recording E at points of
   the plane and the whole P_f after every step, and transforming with numpy
   (factor every * dt, e^{+i w t}, E stamped (n+1) dt, the density from P_f^n
   stamped n dt), reproduces them.
2. Local response keeps the charge on the surface (Sec. V): with beta = D = 0
   each P_c follows E_c through the same causal recursion at every metal
   point, so where all six P points around a node lie in the metal, div P is
   a filtered div E, and Gauss's law (div (eps0 eps_inf E + P) = 0, kept by
   the Yee update) forces both to vanish.  The hydrodynamic pressure term
   spreads the charge inward.
"""
import numpy as np

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask, oracle_problem

QE = 1.602176634e-19


def divergence_at_nodes(P, dx):
    """Backward-difference divergence of (Px, Py, Pz) at the nodes, zero
    outside the grid; arrays (nz, ny, nx)."""
    px, py, pz = P
    d = px.copy()
    d[:, :, 1:] -= px[:, :, :-1]
    d += py
    d[:, 1:, :] -= py[:, :-1, :]
    d += pz
    d[1:, :, :] -= pz[:-1, :, :]
    return d / dx


def problem(w, steps_every, omegas, beta=None):
    p = oracle_problem(w, threads=8, map_axis=1, map_index=int(round(w.spheres[0, 1] / w.dx)),
                       map_every=steps_every, map_omega=omegas)
    if beta is not None:
        p.beta = beta
        p.diff = 0.0
    return p


def test_maps_are_running_transforms_of_the_fields():
    w = W.early_pulse(W.config1(2))
    om = W.spectrum_omegas(3, 2.5, 4.0)
    every, steps = 3, 240
    p = problem(w, every, om)
    s = orc.OracleSim(p, oracle_mask(w))
    j0 = p.map_index
    rng = np.random.default_rng(0)
    cz = int(round(w.spheres[0, 2] / w.dx))
    cx = int(round(w.spheres[0, 0] / w.dx))
    pts = [(cz + dz, cx + dx_) for dz, dx_ in rng.integers(-9, 10, size=(12, 2))]  # (k, i)
    dt = s.dt
    acc = {k: np.zeros((len(om), len(pts)), complex) for k in ("Ex", "Ey", "Ez", "n")}
    inc = np.zeros(len(om), complex)
    off = int(orc.constants()["aux_off"])
    for n in range(steps):
        s.run(1)
        if n % every:
            continue
        tE, tN = (n + 1) * dt, n * dt
        phE = every * dt * np.exp(1j * om * tE)
        phN = every * dt * np.exp(1j * om * tN)
        for c in ("Ex", "Ey", "Ez"):
            f = s.get(c)
            acc[c] += phE[:, None] * np.array([f[k, j0, i] for k, i in pts])[None, :]
        dens = divergence_at_nodes([s.get("Pmx"), s.get("Pmy"), s.get("Pmz")], w.dx) / QE
        acc["n"] += phN[:, None] * np.array([dens[k, j0, i] for k, i in pts])[None, :]
        e1, _ = s.aux()
        inc += phE * e1[w.norm_k + off]
    mp = s.maps()
    assert np.abs(acc["n"]).max() > 0 and np.abs(acc["Ex"]).max() > 0
    for c in ("Ex", "Ey", "Ez", "n"):
        got = np.array([[mp[c][m, k, i] for k, i in pts] for m in range(len(om))])
        scale = np.abs(acc[c]).max()
        assert np.abs(got - acc[c]).max() <= 1e-12 * scale, c
    assert np.abs(mp["inc"] - inc).max() <= 1e-12 * np.abs(inc).max()


def test_local_response_keeps_the_charge_on_the_surface():
    w = W.early_pulse(W.config1(0))
    om = W.spectrum_omegas(2, 3.0, 3.6)
    mask = oracle_mask(w)
    # nodes whose six neighbouring P points all lie in the metal
    inner = ((mask & 1) != 0) & ((mask & 2) != 0) & ((mask & 4) != 0)
    inner[:, :, 1:] &= (mask[:, :, :-1] & 1) != 0
    inner[:, 1:, :] &= (mask[:, :-1, :] & 2) != 0
    inner[1:, :, :] &= (mask[:-1, :, :] & 4) != 0
    inner[:, :, 0] = inner[:, 0, :] = inner[0, :, :] = False
    fractions = {}
    for beta in (0.0, W.BETA):
        p = problem(w, 1, om, beta=beta)
        s = orc.OracleSim(p, mask)
        s.run(w.steps)
        dens = np.abs(s.maps()["n"])  # (nmap, nz, nx) on the plane j0
        j0 = p.map_index
        sel = inner[:, j0, :]
        assert sel.sum() > 20
        fractions[beta] = dens[:, sel].max() / dens.max()
        s.close()
    assert fractions[0.0] <= 1e-9, fractions
    assert fractions[W.BETA] >= 1e-2, fractions
