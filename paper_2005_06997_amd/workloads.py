"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws and lays out problem parameters -- grid sizes, sphere
and star geometry, material constants, the source pulse, monitor boxes and
frequency lists.  It holds none of the FDTD arithmetic.  Both the GPU library
and the CPU oracle receive exactly these parameters; each voxelises the
geometry itself.

Geometry coordinates are metres measured from node (0, 0, 0); a grid of n
cells per axis has nodes 0 .. n-1 and includes the CPML layers.

The workloads stand in for the paper's silver spheres (Sec. V: 200^3 cells
plus CPML, dx = D/100) and its star-shaped particle (Sec. VI: 600^3 cells,
dx = 0.1 nm) with a gold-like Drude metal.  Draw order for each seed is fixed
and stated beside each generator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

HBAR_EV_S = 6.582119569e-16  # reduced Planck constant in eV s
C0 = 299792458.0             # speed of light, m/s (used only to size the pulse window)

# gold-like Drude metal of the benchmark configurations
WP = 1.37e16       # rad/s
GAMMA = 1.06e14    # rad/s
BETA = 1.0e6       # m/s (beta itself; beta^2 = 1e12 m^2/s^2)
DIFF = 1.9e-4      # m^2/s
# Two synthetic critical points (A, Omega [rad/s], Gamma [rad/s], phi [rad])
# with the magnitudes of noble-metal interband fits (poles near 2.6 and 3.7
# eV, widths of 0.4-1.2 eV, negative phases); not a fit to measured data.
CP_SYNTH = ((0.65, 4.0e15, 6.5e14, -1.2), (1.4, 5.6e15, 1.9e15, -1.1))
EPS_INF_SYNTH = 1.1


def ev_to_rad(e: float) -> float:
    return e / HBAR_EV_S


def spectrum_omegas(n: int = 100, e_lo: float = 1.0, e_hi: float = 6.0) -> np.ndarray:
    """omega_m = (e_lo + (e_hi - e_lo) m / (n - 1)) eV / hbar, m = 0 .. n-1."""
    m = np.arange(n, dtype=np.float64)
    return (e_lo + (e_hi - e_lo) * m / max(n - 1, 1)) / HBAR_EV_S


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    courant: float = 0.5
    npml: int = 8
    pml_order: float = 3.0
    pml_sigma_scale: float = 0.8
    pml_kappa_max: float = 1.0
    pml_alpha_max: float = 0.0
    eps_b: float = 1.0
    # dielectric substrate: the half-space z > sub_k (node planes) has relative
    # permittivity eps_sub (0: none)
    eps_sub: float = 0.0
    sub_k: int = 0
    # total-field operation: no TF/SF box; a soft plane source on E_x of node
    # plane source_k; metal may reach into the absorbing layers (local Drude
    # there)
    total_field: bool = False
    source_k: int = 0
    tf_lo: Tuple[int, int, int] = (0, 0, 0)
    tf_hi: Tuple[int, int, int] = (0, 0, 0)
    # material
    wp: float = WP
    gamma: float = GAMMA
    beta: float = BETA
    diff: float = DIFF
    eps_inf: float = 1.0
    # critical points (Eq. CritPoint): (A, Omega, Gamma, phi) per pole
    cp: Tuple = ()
    # near-field / density maps on the plane map_index normal to map_axis
    map_axis: int = 1
    map_index: int = 0
    map_every: int = 1
    map_omega: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # source: 1 modulated Gaussian, 2 raised cosine
    src_kind: int = 1
    e0: float = 1.0
    omega_c: float = ev_to_rad(3.5)
    tau: float = 2.0 * math.sqrt(math.log(10.0)) / ev_to_rad(2.5)
    t0: float = 3.0 * 2.0 * math.sqrt(math.log(10.0)) / ev_to_rad(2.5)
    omega_max: float = 1.26e16
    # monitors
    omega: np.ndarray = field(default_factory=spectrum_omegas)
    dft_every: int = 1
    norm_k: int = 0
    flux: bool = True
    abs_lo: Tuple[int, int, int] = (0, 0, 0)
    abs_hi: Tuple[int, int, int] = (0, 0, 0)
    sca_lo: Tuple[int, int, int] = (0, 0, 0)
    sca_hi: Tuple[int, int, int] = (0, 0, 0)
    # geometry: "spheres" -> (n, 4) array [cx, cy, cz, r]; "star" -> descriptor
    geometry: str = "spheres"
    spheres: Optional[np.ndarray] = None
    star: Optional[np.ndarray] = None
    steps: int = 600
    precision: str = "fp64"
    # optional design region (node-index box [lo, hi)) and density
    design_lo: Optional[Tuple[int, int, int]] = None
    design_hi: Optional[Tuple[int, int, int]] = None
    rho: Optional[np.ndarray] = None

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dt(self) -> float:
        return self.courant * self.dx / C0


def _boxes(w: Workload, lo_m: np.ndarray, hi_m: np.ndarray, margin: int = 3) -> Workload:
    """TF box = analytic metal extent (cells) + `margin`; absorption box one cell
    inside it; scattering box two cells outside it."""
    lo = np.floor(lo_m / w.dx).astype(int) - margin
    hi = np.ceil(hi_m / w.dx).astype(int) + margin
    w.tf_lo = tuple(int(v) for v in lo)
    w.tf_hi = tuple(int(v) for v in hi)
    w.abs_lo = tuple(int(v) + 1 for v in lo)
    w.abs_hi = tuple(int(v) - 1 for v in hi)
    w.sca_lo = tuple(int(v) - 2 for v in lo)
    w.sca_hi = tuple(int(v) + 2 for v in hi)
    n = (w.nx, w.ny, w.nz)
    for a in range(3):
        # the scattering box samples H half a cell on either side of its faces;
        # all of them must lie outside the absorbing layers
        if w.sca_lo[a] < w.npml + 1 or w.sca_hi[a] > n[a] - 2 - w.npml:
            raise ValueError(f"{w.name}: monitor boxes do not fit between the particle and the CPML")
    return w


def sphere_problem(name: str, n: int, dx: float, npml: int, centre_cells, radius: float,
                   **kw) -> Workload:
    c = np.asarray(centre_cells, dtype=np.float64) * dx
    w = Workload(name=name, nx=n, ny=n, nz=n, dx=dx, npml=npml, **kw)
    w.geometry = "spheres"
    w.spheres = np.array([[c[0], c[1], c[2], radius]])
    w.norm_k = int(round(c[2] / dx))
    return _boxes(w, c - radius, c + radius)


def config1(seed: int = 0) -> Workload:
    """Single gold-like sphere r = 2 nm +- U(0.1 nm) centred in a 48^3 grid at
    dx = 0.25 nm, 8-cell CPML, FP64, 600 steps.  Draws: radius jitter, then
    the three centre offsets (each U(-0.5, 0.5) cell)."""
    g = np.random.Generator(np.random.PCG64(seed))
    r = 2.0e-9 + g.uniform(-0.1e-9, 0.1e-9)
    off = g.uniform(-0.5, 0.5, size=3)
    n = 48
    centre = (n - 1) / 2.0 + off
    return sphere_problem(f"sphere_r2nm_48^3_seed{seed}", n, 0.25e-9, 8, centre, r,
                          steps=600, precision="fp64")


def config2(precision: str = "fp32") -> Workload:
    """Single sphere r = 10 nm, 320^3 grid at dx = 0.1 nm, 12-cell CPML, 20000 steps."""
    n = 320
    return sphere_problem("sphere_r10nm_320^3", n, 0.1e-9, 12, [(n - 1) / 2.0] * 3, 10.0e-9,
                          steps=20000, precision=precision)


def config2_coarse(precision: str = "fp32") -> Workload:
    """The same particle on a 2x coarser grid: 160^3 at dx = 0.2 nm, 10000 steps
    (same physical time), 8-cell CPML."""
    n = 160
    return sphere_problem("sphere_r10nm_160^3", n, 0.2e-9, 8, [(n - 1) / 2.0] * 3, 10.0e-9,
                          steps=10000, precision=precision)


def star_descriptor(centre, R: float, r_tip: float, half_angle_deg: float,
                    axes: np.ndarray, lengths: np.ndarray) -> np.ndarray:
    """[cx, cy, cz, R, r_tip, tan(half), sin(half), ntips, (ax, ay, az, L) x ntips]."""
    th = math.radians(half_angle_deg)
    head = [centre[0], centre[1], centre[2], R, r_tip, math.tan(th), math.sin(th), float(len(lengths))]
    body = []
    for a, L in zip(axes, lengths):
        body += [a[0], a[1], a[2], L]
    return np.array(head + body, dtype=np.float64)


_BASE_AXES = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                      dtype=np.float64)


def _perp_pair(e: np.ndarray):
    # two unit vectors orthogonal to e (fixed choice per axis)
    t = np.array([0.0, 0.0, 1.0]) if abs(e[2]) < 0.5 else np.array([1.0, 0.0, 0.0])
    u = np.cross(e, t)
    u /= np.linalg.norm(u)
    v = np.cross(e, u)
    return u, v


def star_tips(g: np.random.Generator, L0: float, dL: float, max_tilt_deg: float):
    """Per tip (order +x, -x, +y, -y, +z, -z): length L0 + U(-dL, dL), then tilt
    angle U(0, max_tilt) and azimuth U(0, 2 pi)."""
    axes, lengths = [], []
    for e in _BASE_AXES:
        L = L0 + g.uniform(-dL, dL)
        tilt = math.radians(g.uniform(0.0, max_tilt_deg))
        phi = g.uniform(0.0, 2.0 * math.pi)
        u, v = _perp_pair(e)
        a = math.cos(tilt) * e + math.sin(tilt) * (math.cos(phi) * u + math.sin(phi) * v)
        a /= np.linalg.norm(a)
        axes.append(a)
        lengths.append(L)
    return np.array(axes), np.array(lengths)


def config3(seed: int = 0, n: int = 640, dx: float = 0.2e-9, precision: str = "fp32") -> Workload:
    """Sphere R = 15 nm with six sphere-capped cones along +-x, +-y, +-z: length
    12 +- U(2) nm past the surface, apex radius 0.5 nm, half-angle 15 deg, each
    axis tilted by U(0, 10 deg) in a uniform azimuth; 640^3 at dx = 0.2 nm,
    12-cell CPML, 30000 steps."""
    g = np.random.Generator(np.random.PCG64(seed))
    axes, lengths = star_tips(g, 12.0e-9, 2.0e-9, 10.0)
    R = 15.0e-9
    centre = np.array([(n - 1) / 2.0 * dx] * 3)
    w = Workload(name=f"star_R15nm_{n}^3_seed{seed}", nx=n, ny=n, nz=n, dx=dx, npml=12,
                 steps=30000, precision=precision)
    w.geometry = "star"
    w.star = star_descriptor(centre, R, 0.5e-9, 15.0, axes, lengths)
    ext = R + float(np.max(lengths)) + 1.0e-9
    w.norm_k = int(round(centre[2] / dx))
    return _boxes(w, centre - ext, centre + ext)


def config4(seed: int = 0, count: int = 64) -> List[Workload]:
    """Batched sweep.  Per instance draws, in order: type (sphere or gap dimer
    with p = 1/2; dimer axis along x), radius U(1, 8) nm, gap U(0.5, 2) nm,
    beta U(0.8e6, 1.2e6) m/s, D U(0, 4e-4) m^2/s.  dx = 0.2 nm; cube side =
    clamp(8 ceil((extent + 10 nm) / dx / 8), 40, 200) with an 8-cell CPML;
    FP32, 8000 steps each."""
    g = np.random.Generator(np.random.PCG64(seed))
    dx = 0.2e-9
    out = []
    for idx in range(count):
        dimer = g.uniform() < 0.5
        r = g.uniform(1.0e-9, 8.0e-9)
        gap = g.uniform(0.5e-9, 2.0e-9)
        beta = g.uniform(0.8e6, 1.2e6)
        diff = g.uniform(0.0, 4.0e-4)
        extent = (4 * r + gap) if dimer else 2 * r
        side = 8 * math.ceil((extent + 10.0e-9) / dx / 8)
        side = max(40, min(200, side))
        c = np.array([(side - 1) / 2.0 * dx] * 3)
        w = Workload(name=f"batch{idx}_{'dimer' if dimer else 'sphere'}_{side}^3", nx=side, ny=side,
                     nz=side, dx=dx, npml=8, beta=beta, diff=diff, steps=8000, precision="fp32",
                     flux=False)
        if dimer:
            off = r + gap / 2.0
            w.spheres = np.array([[c[0] - off, c[1], c[2], r], [c[0] + off, c[1], c[2], r]])
            lo = c - np.array([off + r, r, r])
            hi = c + np.array([off + r, r, r])
        else:
            w.spheres = np.array([[c[0], c[1], c[2], r]])
            lo, hi = c - r, c + r
        w.norm_k = int(round(c[2] / dx))
        out.append(_boxes(w, lo, hi))
    return out


def dimer_design(seed: int = 0, n: int = 160, dx: float = 0.25e-9, r: float = 5.0e-9,
                 gap: float = 1.0e-9, design: int = 60, npml: int = 8, steps: int = 6000,
                 precision: str = "fp32") -> Workload:
    """Gold-like dimer (two spheres along x) with a cubic design region of side
    `design` cells centred on the gap; density rho ~ U(0, 1) (seeded, drawn
    in x-fastest order) replaces the fixed metal there."""
    g = np.random.Generator(np.random.PCG64(seed))
    c = np.array([(n - 1) / 2.0 * dx] * 3)
    off = r + gap / 2.0
    w = Workload(name=f"dimer_design_{n}^3", nx=n, ny=n, nz=n, dx=dx, npml=npml, steps=steps,
                 precision=precision, flux=False)
    w.spheres = np.array([[c[0] - off, c[1], c[2], r], [c[0] + off, c[1], c[2], r]])
    ci = int(round(c[0] / dx))
    lo = ci - design // 2
    w.design_lo = (lo, lo, lo)
    w.design_hi = (lo + design, lo + design, lo + design)
    w.rho = g.uniform(0.0, 1.0, size=(design, design, design)).astype(np.float32)
    ext_lo = np.minimum(c - np.array([off + r, r, r]), np.array(w.design_lo) * dx)
    ext_hi = np.maximum(c + np.array([off + r, r, r]), np.array(w.design_hi) * dx)
    w.norm_k = int(round(c[2] / dx))
    return _boxes(w, ext_lo, ext_hi)


def config5(seed: int = 0) -> Workload:
    """Adjoint design gradient: 160^3 at dx = 0.25 nm, r = 5 nm dimer with a 1 nm
    gap, 60^3 design region, objective sigma_ext at 2.5 eV, 6000 steps."""
    return dimer_design(seed)


def config5_small(seed: int = 0) -> Workload:
    """48^3 copy of the design problem: same dx, geometry x 0.3, design 18^3."""
    return dimer_design(seed, n=48, r=1.5e-9, gap=0.3e-9, design=18, npml=4, steps=6000,
                        precision="fp64")


def design_direction(shape, seed: int) -> np.ndarray:
    """A seeded direction in design-density space (standard normal entries,
    shape (z, y, x)) along which a gradient is projected."""
    g = np.random.Generator(np.random.PCG64(seed))
    return g.standard_normal(size=tuple(shape))


def small_sphere(n: int = 32, dx: float = 0.25e-9, radius: float = 1.2e-9, npml: int = 4,
                 seed: int = 0, steps: int = 200, **kw) -> Workload:
    """Small test problem: one sphere near the grid centre (offset U(-0.5, 0.5) cell)."""
    g = np.random.Generator(np.random.PCG64(seed))
    off = g.uniform(-0.5, 0.5, size=3)
    centre = (n - 1) / 2.0 + off
    return sphere_problem(f"small_sphere_{n}^3_seed{seed}", n, dx, npml, centre, radius,
                          steps=steps, **kw)


def with_critical_points(w: Workload, poles=CP_SYNTH, eps_inf: float = EPS_INF_SYNTH) -> Workload:
    """The same problem with bound electrons: the two synthetic critical points
    and eps_inf > 1 in the metal (eps_b stays 1)."""
    return replace(w, name=w.name + "_cp", cp=tuple(tuple(float(x) for x in q) for q in poles),
                   eps_inf=eps_inf)


def with_maps(w: Workload, omegas, every: int = 1, axis: int = 1) -> Workload:
    """Maps on the plane through the first particle's centre, normal to
    `axis` (the xz plane for axis 1: polarisation and propagation)."""
    c = w.spheres[0, :3] if w.geometry == "spheres" else w.star[:3]
    return replace(w, map_axis=axis, map_index=int(round(c[axis] / w.dx)), map_every=every,
                   map_omega=np.asarray(omegas, dtype=np.float64))


def early_pulse(w: Workload) -> Workload:
    """Move the pulse peak to 1.2 tau so that short runs see the field."""
    return replace(w, t0=1.2 * w.tau)
