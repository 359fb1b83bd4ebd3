"""Shared test helpers: workload -> oracle problem, norms."""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc


def oracle_problem(w, **over) -> "orc.Problem":
    """Copy a workload's parameters into the oracle's own problem record."""
    p = orc.Problem(
        nx=w.nx, ny=w.ny, nz=w.nz, dx=w.dx, courant=w.courant, eps_b=w.eps_b, npml=w.npml,
        pml_order=w.pml_order, pml_sigma_scale=w.pml_sigma_scale, pml_kappa_max=w.pml_kappa_max,
        pml_alpha_max=w.pml_alpha_max, tfsf=True, tf_lo=w.tf_lo, tf_hi=w.tf_hi, model=0,
        wp=w.wp, gamma=w.gamma, beta=w.beta, diff=w.diff, eps_inf=w.eps_inf, src_kind=w.src_kind,
        e0=w.e0, omega_c=w.omega_c, tau=w.tau, t0=w.t0, omega_max=w.omega_max,
        omega=np.asarray(w.omega, dtype=np.float64), dft_every=w.dft_every, norm_k=w.norm_k,
        flux=bool(w.flux), abs_lo=w.abs_lo, abs_hi=w.abs_hi, sca_lo=w.sca_lo, sca_hi=w.sca_hi,
        cp=tuple(w.cp), map_axis=w.map_axis, map_index=w.map_index, map_every=w.map_every,
        map_omega=np.asarray(w.map_omega, dtype=np.float64), eps_sub=w.eps_sub, sub_k=w.sub_k,
        total_field=bool(w.total_field), source_k=w.source_k)
    if w.total_field:
        p.tfsf = False
    for k, v in over.items():
        setattr(p, k, v)
    return p


def oracle_mask(w) -> np.ndarray:
    if w.geometry == "star":
        return orc.voxelize_star(w.nx, w.ny, w.nz, w.dx, w.star)
    return orc.voxelize_spheres(w.nx, w.ny, w.nz, w.dx, w.spheres)


def oracle_mask_and_weight(w):
    """Mask and per-cell metal weight; a design region, if any, is fully
    active with weight rho."""
    m = oracle_mask(w)
    wt = (m != 0).astype(np.float64)
    if w.design_lo is not None:
        (x0, y0, z0), (x1, y1, z1) = w.design_lo, w.design_hi
        m[z0:z1, y0:y1, x0:x1] = 7
        wt[z0:z1, y0:y1, x0:x1] = np.asarray(w.rho)  # rho is stored (z, y, x), x fastest
    return m, wt


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den = np.linalg.norm(b)
    if den == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / den)
