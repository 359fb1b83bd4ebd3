"""ctypes front end of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  It loads ``libgnor_oracle.so`` (built from ``gnor_oracle.cpp``
with g++) and never touches the GPU library.

The oracle implements the hydrodynamic FDTD step of Baxter, Cala Lesina &
Ramunno (arXiv:2005.06997) literally: the Yee positions of Sec. III Table I,
the update order H -> E -> P_f, Eq. (NonlocalUpdate) / Eq. (GNORUpdate) for
P_f with Eq. (GradDiv) written term by term, and the two E-update equations
obtained from Eq. (discreteamperes).  Everything is SI and FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gnor_oracle.cpp")
LIB = os.path.join(HERE, "libgnor_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP contraction off, OpenMP available)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
               SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(OrConfig), C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_run.argtypes = [C.c_void_p, C.c_long]
        L.or_step_index.restype = C.c_long
        L.or_step_index.argtypes = [C.c_void_p]
        L.or_dt.restype = C.c_double
        L.or_dt.argtypes = [C.c_void_p]
        L.or_get.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.or_set.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.or_get_aux.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_aux_len.restype = C.c_int
        L.or_aux_len.argtypes = [C.c_void_p]
        L.or_get_dft.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.or_spectra.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.or_get_maps.restype = C.c_long
        L.or_get_maps.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_box_flux.restype = C.c_double
        L.or_box_flux.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.or_face_flux.restype = C.c_double
        L.or_face_flux.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.or_directional.argtypes = [C.POINTER(OrConfig), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_long, C.c_int, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
        L.or_voxelize_spheres.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                          C.c_void_p, C.c_void_p]
        L.or_voxelize_star.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_void_p,
                                       C.c_void_p]
        L.or_constants.restype = C.c_double
        L.or_constants.argtypes = [C.c_int]
        _lib = L
    return _lib


class OrConfig(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("periodic", C.c_int32),
        ("dx", C.c_double), ("courant", C.c_double), ("eps_b", C.c_double),
        ("npml", C.c_int32),
        ("pml_order", C.c_double), ("pml_sigma_scale", C.c_double),
        ("pml_kappa_max", C.c_double), ("pml_alpha_max", C.c_double),
        ("tfsf", C.c_int32), ("tf_lo", C.c_int32 * 3), ("tf_hi", C.c_int32 * 3),
        ("model", C.c_int32),
        ("wp", C.c_double), ("gamma", C.c_double), ("beta", C.c_double),
        ("diff", C.c_double), ("eps_inf", C.c_double),
        ("src_kind", C.c_int32),
        ("e0", C.c_double), ("omega_c", C.c_double), ("tau", C.c_double),
        ("t0", C.c_double), ("omega_max", C.c_double),
        ("nfreq", C.c_int32), ("dft_every", C.c_int32), ("norm_k", C.c_int32),
        ("flux", C.c_int32),
        ("abs_lo", C.c_int32 * 3), ("abs_hi", C.c_int32 * 3),
        ("sca_lo", C.c_int32 * 3), ("sca_hi", C.c_int32 * 3),
        ("threads", C.c_int32),
        ("ncp", C.c_int32),
        ("cp_A", C.c_double * 4), ("cp_Omega", C.c_double * 4),
        ("cp_Gamma", C.c_double * 4), ("cp_phi", C.c_double * 4),
        ("map_axis", C.c_int32), ("map_index", C.c_int32), ("nmap", C.c_int32),
        ("map_every", C.c_int32), ("map_omega", C.c_double * 8),
        ("eps_sub", C.c_double), ("sub_k", C.c_int32),
        ("total_field", C.c_int32), ("source_k", C.c_int32),
        ("periodic_xy", C.c_int32),
    ]


@dataclass
class Problem:
    """Everything the oracle needs (SI units; grid counts include the CPML)."""
    nx: int
    ny: int
    nz: int
    dx: float
    courant: float = 0.5
    eps_b: float = 1.0
    npml: int = 8
    pml_order: float = 3.0
    pml_sigma_scale: float = 0.8
    pml_kappa_max: float = 1.0
    pml_alpha_max: float = 0.0
    periodic: bool = False
    tfsf: bool = True
    tf_lo: Sequence[int] = (0, 0, 0)
    tf_hi: Sequence[int] = (0, 0, 0)
    model: int = 0  # 0 GNOR, 1 nonlocal Drude (Eq. NonlocalUpdate)
    wp: float = 0.0
    gamma: float = 0.0
    beta: float = 0.0
    diff: float = 0.0
    eps_inf: float = 1.0
    src_kind: int = 1  # 0 none, 1 modulated Gaussian, 2 raised cosine
    e0: float = 1.0
    omega_c: float = 0.0
    tau: float = 0.0
    t0: float = 0.0
    omega_max: float = 0.0
    omega: np.ndarray = field(default_factory=lambda: np.zeros(0))
    dft_every: int = 1
    norm_k: int = 0
    flux: bool = False
    abs_lo: Sequence[int] = (0, 0, 0)
    abs_hi: Sequence[int] = (0, 0, 0)
    sca_lo: Sequence[int] = (0, 0, 0)
    sca_hi: Sequence[int] = (0, 0, 0)
    threads: int = 0
    # critical points, Eq. (CritPoint): up to 4 poles (A_p, Omega_p, Gamma_p, phi_p)
    cp: Sequence[Sequence[float]] = ()
    # near-field / density maps on the plane map_index normal to map_axis
    map_axis: int = 1
    map_index: int = 0
    map_every: int = 1
    map_omega: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # dielectric substrate: the half-space z > sub_k has permittivity eps_sub
    # (0: none)
    eps_sub: float = 0.0
    sub_k: int = 0
    # total-field operation: no TF/SF, a soft plane source on E_x of node
    # plane source_k; metal inside the absorbing layers follows the local
    # Drude model there
    total_field: bool = False
    source_k: int = 0
    # periodic in x and y, CPML on the z faces only (test mode)
    periodic_xy: bool = False

    def to_c(self) -> OrConfig:
        c = OrConfig()
        for name, _ in OrConfig._fields_:
            if name == "nfreq":
                c.nfreq = int(len(self.omega))
                continue
            if name == "ncp":
                if len(self.cp) > 4:
                    raise ValueError("at most 4 critical points")
                c.ncp = len(self.cp)
                continue
            if name == "nmap":
                if len(self.map_omega) > 8:
                    raise ValueError("at most 8 map frequencies")
                c.nmap = len(self.map_omega)
                continue
            if name == "map_omega":
                c.map_omega[:] = [float(x) for x in self.map_omega] + [0.0] * (8 - len(self.map_omega))
                continue
            if name.startswith("cp_"):
                col = {"cp_A": 0, "cp_Omega": 1, "cp_Gamma": 2, "cp_phi": 3}[name]
                getattr(c, name)[:] = [float(pole[col]) for pole in self.cp] + [0.0] * (4 - len(self.cp))
                continue
            v = getattr(self, name)
            if name in ("tf_lo", "tf_hi", "abs_lo", "abs_hi", "sca_lo", "sca_hi"):
                getattr(c, name)[:] = [int(x) for x in v]
            elif name == "threads":
                c.threads = int(v) if v else int(os.environ.get("ORACLE_THREADS", "1"))
            else:
                setattr(c, name, type(getattr(c, name))(v))
        return c


FIELD_INDEX = {
    "Ex": 0, "Ey": 1, "Ez": 2, "Hx": 3, "Hy": 4, "Hz": 5, "Jx": 6, "Jy": 7, "Jz": 8,
    "Px": 9, "Py": 10, "Pz": 11, "Pmx": 12, "Pmy": 13, "Pmz": 14,
    "Emx": 15, "Emy": 16, "Emz": 17, "GD1x": 18, "GD1y": 19, "GD1z": 20,
    "GD2x": 21, "GD2y": 22, "GD2z": 23,
}
# critical-point polarisations: "PC<q><c>" (P_CP,q^n), "PCm<q><c>" (P_CP,q^{n-1})
for _q in range(4):
    for _i, _c in enumerate("xyz"):
        FIELD_INDEX[f"PC{_q}{_c}"] = 24 + 6 * _q + _i
        FIELD_INDEX[f"PCm{_q}{_c}"] = 27 + 6 * _q + _i


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleSim:
    """One oracle simulation; arrays are (nz, ny, nx) C-order, x fastest."""

    def __init__(self, prob: Problem, mask: np.ndarray, weight: Optional[np.ndarray] = None):
        self.prob = prob
        self.shape = (prob.nz, prob.ny, prob.nx)
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(self.shape)
        assert m.shape == self.shape
        self._mask = m
        self._w = None if weight is None else np.ascontiguousarray(weight, dtype=np.float64).reshape(self.shape)
        self._om = np.ascontiguousarray(prob.omega, dtype=np.float64)
        self._cfg = prob.to_c()
        self.h = lib().or_create(C.byref(self._cfg), _ptr(m),
                                 None if self._w is None else _ptr(self._w), _ptr(self._om))

    def close(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def dt(self) -> float:
        return lib().or_dt(self.h)

    @property
    def step(self) -> int:
        return lib().or_step_index(self.h)

    def run(self, nsteps: int):
        lib().or_run(self.h, int(nsteps))

    def get(self, name: str) -> np.ndarray:
        out = np.empty(self.shape, np.float64)
        assert lib().or_get(self.h, FIELD_INDEX[name], _ptr(out)) == 0
        return out

    def set(self, name: str, arr: np.ndarray):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self.shape)
        assert lib().or_set(self.h, FIELD_INDEX[name], _ptr(a)) == 0

    def aux(self):
        n = lib().or_aux_len(self.h)
        e = np.empty(n)
        hh = np.empty(n)
        lib().or_get_aux(self.h, _ptr(e), _ptr(hh))
        return e, hh

    def dft(self):
        nf = len(self._om)
        arrs = [np.empty((self.prob.nz, nf)) for _ in range(4)]
        lib().or_get_dft(self.h, *[_ptr(a) for a in arrs])
        return (arrs[0] + 1j * arrs[1], arrs[2] + 1j * arrs[3])

    def maps(self):
        """Map transforms: dict Ex, Ey, Ez, n -> complex (nmap, mv, mu) arrays,
        and inc -> complex (nmap,) incident transforms at norm_k."""
        p = self.prob
        nm = len(p.map_omega)
        ns = (p.nx, p.ny, p.nz)
        ua = 1 if p.map_axis == 0 else 0
        va = 1 if p.map_axis == 2 else 2
        mu, mv = ns[ua], ns[va]
        f = np.empty((8, nm, mv, mu))
        inc = np.empty((nm, 2))
        assert lib().or_get_maps(self.h, _ptr(f), _ptr(inc)) == mu * mv
        out = {k: f[2 * q] + 1j * f[2 * q + 1] for q, k in enumerate(("Ex", "Ey", "Ez", "n"))}
        out["inc"] = inc[:, 0] + 1j * inc[:, 1]
        return out

    def spectra(self):
        nf = len(self._om)
        out = [np.empty(nf) for _ in range(4)]
        lib().or_spectra(self.h, *[_ptr(a) for a in out])
        return dict(inc=out[0], ext=out[1], abs=out[2], sca=out[3])

    def box_flux(self, box: int, m: int) -> float:
        """Outward flux of Re(E x H*) through box 0 (absorption) or 1 (scattering)."""
        return lib().or_box_flux(self.h, box, m)

    def face_flux(self, box: int, face: int, m: int) -> float:
        """Outward flux through one face; faces ordered -x, +x, -y, +y, -z, +z."""
        return lib().or_face_flux(self.h, box, face, m)


def directional(prob: Problem, mask: np.ndarray, weight: np.ndarray, direction: np.ndarray,
                nsteps: int, m_target: int):
    """sigma_ext(omega[m_target]) and its exact derivative along `direction`
    (dual-number forward mode through every step)."""
    shape = (prob.nz, prob.ny, prob.nx)
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(shape)
    w = np.ascontiguousarray(weight, dtype=np.float64).reshape(shape)
    d = np.ascontiguousarray(direction, dtype=np.float64).reshape(shape)
    om = np.ascontiguousarray(prob.omega, dtype=np.float64)
    cfg = prob.to_c()
    v = C.c_double()
    dv = C.c_double()
    lib().or_directional(C.byref(cfg), _ptr(m), _ptr(w), _ptr(d), _ptr(om), int(nsteps),
                         int(m_target), C.byref(v), C.byref(dv))
    return v.value, dv.value


def voxelize_spheres(nx: int, ny: int, nz: int, dx: float, spheres: np.ndarray) -> np.ndarray:
    """spheres: (n, 4) array of centre x, y, z and radius in metres (origin at node 0)."""
    s = np.ascontiguousarray(spheres, dtype=np.float64).reshape(-1, 4)
    out = np.empty((nz, ny, nx), np.uint8)
    lib().or_voxelize_spheres(nx, ny, nz, float(dx), int(s.shape[0]), _ptr(s), _ptr(out))
    return out


def voxelize_star(nx: int, ny: int, nz: int, dx: float, desc: np.ndarray) -> np.ndarray:
    d = np.ascontiguousarray(desc, dtype=np.float64)
    out = np.empty((nz, ny, nx), np.uint8)
    lib().or_voxelize_star(nx, ny, nz, float(dx), _ptr(d), _ptr(out))
    return out


def constants() -> dict:
    L = lib()
    return dict(c0=L.or_constants(0), mu0=L.or_constants(1), eps0=L.or_constants(2),
                eta0=L.or_constants(3), aux_pml=int(L.or_constants(4)),
                aux_off=int(L.or_constants(5)), aux_src=int(L.or_constants(6)))
