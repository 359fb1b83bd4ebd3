"""Python binding of libgnorfdtd (ctypes; argument marshalling only).

Every step of the time loop runs in the HIP kernels of ``libgnorfdtd.so``.
PyTorch provides the device buffer the library carves its state from and the
HIP stream it enqueues on.  If the library has not been built, or no GPU is
present, constructing a :class:`Sim` raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgnorfdtd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gnor_fdtd.h")

GNOR_FP32, GNOR_FP64 = 0, 1
STATUS = {0: "GNOR_OK", 1: "GNOR_E_INVALID_ARG", 2: "GNOR_E_UNSTABLE", 3: "GNOR_E_OUT_OF_MEMORY",
          4: "GNOR_E_DEVICE", 5: "GNOR_E_STATE", 6: "GNOR_E_BUFFER_TOO_SMALL", 7: "GNOR_E_NONFINITE"}
FIELDS = {"Ex": 0, "Ey": 1, "Ez": 2, "Hx": 3, "Hy": 4, "Hz": 5, "Jx": 6, "Jy": 7, "Jz": 8,
          "n": 21}  # n: free-electron density n - n0 at the nodes (GNOR_FIELD_DENSITY)
# critical-point polarisation P_CP,p^n: "PC<p><c>"
FIELDS.update({f"PC{p}{c}": 9 + 3 * p + i for p in range(4) for i, c in enumerate("xyz")})


class GnorError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("courant", C.c_double), ("npml", C.c_int32),
                ("pml_order", C.c_double), ("pml_sigma_scale", C.c_double),
                ("pml_kappa_max", C.c_double), ("pml_alpha_max", C.c_double),
                ("eps_background", C.c_double),
                ("tf_lo", C.c_int32 * 3), ("tf_hi", C.c_int32 * 3), ("precision", C.c_int32),
                ("eps_substrate", C.c_double), ("substrate_k", C.c_int32),
                ("total_field", C.c_int32), ("source_k", C.c_int32)]


MAX_CP = 4


class MaterialDesc(C.Structure):
    _fields_ = [("wp", C.c_double), ("gamma", C.c_double), ("beta", C.c_double),
                ("diffusion", C.c_double), ("eps_inf", C.c_double),
                ("ncp", C.c_int32),
                ("cp_A", C.c_double * MAX_CP), ("cp_Omega", C.c_double * MAX_CP),
                ("cp_Gamma", C.c_double * MAX_CP), ("cp_phi", C.c_double * MAX_CP)]


class MapDesc(C.Structure):
    _fields_ = [("axis", C.c_int32), ("index", C.c_int32), ("nmap", C.c_int32),
                ("every", C.c_int32), ("omega", C.POINTER(C.c_double))]


class SourceDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("e0", C.c_double), ("omega_c", C.c_double),
                ("tau", C.c_double), ("t0", C.c_double), ("omega_max", C.c_double)]


class MonitorDesc(C.Structure):
    _fields_ = [("nfreq", C.c_int32), ("omega", C.POINTER(C.c_double)), ("norm_k", C.c_int32),
                ("dft_every", C.c_int32), ("flux_enabled", C.c_int32),
                ("abs_lo", C.c_int32 * 3), ("abs_hi", C.c_int32 * 3),
                ("sca_lo", C.c_int32 * 3), ("sca_hi", C.c_int32 * 3)]


_lib = None


def header_functions():
    """Names of the functions declared in include/gnor_fdtd.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gnor_[a-z_0-9]+)\s*\(", txt)))


def load() -> C.CDLL:
    """Load libgnorfdtd.so (built in-tree by ``paper_2005_06997_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2005_06997_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    dp = C.POINTER(C.c_double)
    sig = {
        "gnor_create": (i32, [C.POINTER(GridDesc), C.POINTER(vp)]),
        "gnor_destroy": (None, [vp]),
        "gnor_set_material": (i32, [vp, vp, C.POINTER(MaterialDesc)]),
        "gnor_set_source": (i32, [vp, C.POINTER(SourceDesc)]),
        "gnor_set_monitors": (i32, [vp, C.POINTER(MonitorDesc)]),
        "gnor_set_maps": (i32, [vp, C.POINTER(MapDesc)]),
        "gnor_get_maps": (i32, [vp, vp, vp, sz]),
        "gnor_required_bytes": (sz, [vp]),
        "gnor_bind_memory": (i32, [vp, vp, sz, vp]),
        "gnor_reset": (i32, [vp]),
        "gnor_run": (i32, [vp, i64]),
        "gnor_set_watchdog": (i32, [vp, i32]),
        "gnor_synchronize": (i32, [vp]),
        "gnor_step_index": (i64, [vp]),
        "gnor_set_graph_chunk": (i32, [vp, i32]),
        "gnor_get_spectra": (i32, [vp, dp, dp, dp, dp]),
        "gnor_flush_spectra": (i32, [vp]),
        "gnor_get_dft": (i32, [vp, dp, dp, dp, dp]),
        "gnor_get_field": (i32, [vp, i32, dp, sz]),
        "gnor_get_aux": (i32, [vp, dp, dp, sz]),
        "gnor_state_bytes": (sz, [vp]),
        "gnor_save_state": (i32, [vp, vp, sz]),
        "gnor_load_state": (i32, [vp, vp, sz]),
        "gnor_check_finite": (i32, [vp]),
        "gnor_profile_kernels": (i32, [vp, i64, dp, i32]),
        "gnor_tile_classes": (i32, [vp, C.POINTER(C.c_int32)]),
        "gnor_tile_class_cells": (i32, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
        "gnor_set_fused": (i32, [vp, i32]),
        "gnor_set_class_streams": (i32, [vp, i32]),
        "gnor_set_tiling": (i32, [vp, i32, i32, i32]),
        "gnor_autotune": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), dp]),
        "gnor_voxelize_spheres": (i32, [i32, i32, i32, dbl, i32, vp, vp]),
        "gnor_voxelize_star": (i32, [i32, i32, i32, dbl, vp, i32, vp]),
        "gnor_set_design": (i32, [vp, C.POINTER(i32), C.POINTER(i32), vp]),
        "gnor_update_design": (i32, [vp, vp]),
        "gnor_gradient_required_bytes": (sz, [vp, i64, i32]),
        "gnor_gradient": (i32, [vp, i64, i32, i32, vp, sz, dp, vp]),
        "gnor_batch_required_bytes": (sz, [i32, vp]),
        "gnor_batch_create": (i32, [i32, vp, vp, vp, sz, C.POINTER(vp)]),
        "gnor_batch_create_static": (i32, [i32, vp, vp, C.POINTER(vp)]),
        "gnor_batch_run": (i32, [vp, i64]),
        "gnor_batch_synchronize": (i32, [vp]),
        "gnor_batch_set_graph_chunk": (i32, [vp, i32]),
        "gnor_batch_set_form": (i32, [vp, i32]),
        "gnor_batch_last_error": (C.c_char_p, [vp]),
        "gnor_batch_destroy": (None, [vp]),
        "gnor_status_string": (C.c_char_p, [i32]),
        "gnor_last_error": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def voxelize(w) -> np.ndarray:
    """The library's own voxeliser for a workload's geometry (x-fastest mask)."""
    L = load()
    out = np.zeros((w.nz, w.ny, w.nx), np.uint8)
    if w.geometry == "star":
        d = np.ascontiguousarray(w.star, dtype=np.float64)
        st = L.gnor_voxelize_star(w.nx, w.ny, w.nz, w.dx, d.ctypes.data, len(d), out.ctypes.data)
    else:
        s = np.ascontiguousarray(w.spheres, dtype=np.float64).reshape(-1, 4)
        st = L.gnor_voxelize_spheres(w.nx, w.ny, w.nz, w.dx, s.shape[0], s.ctypes.data, out.ctypes.data)
    if st:
        raise GnorError(st, "voxeliser rejected the geometry")
    return out


class Sim:
    """One simulation on one GPU.  `w` is a workload record (see
    :mod:`paper_2005_06997_amd.workloads`); `mask` overrides the voxelised
    geometry."""

    def __init__(self, w, precision: Optional[str] = None, device: str = "cuda:0",
                 mask: Optional[np.ndarray] = None, graph_chunk: int = 64):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libgnorfdtd needs a GPU: torch.cuda.is_available() is False")
        self.L = load()
        self.w = w
        prec = (precision or w.precision).lower()
        self.precision = prec
        g = GridDesc(nx=w.nx, ny=w.ny, nz=w.nz, dx=w.dx, courant=w.courant, npml=w.npml,
                     pml_order=w.pml_order, pml_sigma_scale=w.pml_sigma_scale,
                     pml_kappa_max=w.pml_kappa_max, pml_alpha_max=w.pml_alpha_max,
                     eps_background=w.eps_b, precision=GNOR_FP32 if prec == "fp32" else GNOR_FP64,
                     eps_substrate=getattr(w, "eps_sub", 0.0), substrate_k=getattr(w, "sub_k", 0),
                     total_field=int(bool(getattr(w, "total_field", False))),
                     source_k=int(getattr(w, "source_k", 0)))
        g.tf_lo[:] = list(w.tf_lo)
        g.tf_hi[:] = list(w.tf_hi)
        h = C.c_void_p()
        st = self.L.gnor_create(C.byref(g), C.byref(h))
        if st:
            raise GnorError(st, "gnor_create rejected the grid")
        self.h = h
        self.mode = 0
        self.mask = voxelize(w) if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        mat = MaterialDesc(wp=w.wp, gamma=w.gamma, beta=w.beta, diffusion=w.diff, eps_inf=w.eps_inf)
        cp = tuple(getattr(w, "cp", ()))
        if len(cp) > MAX_CP:
            raise ValueError(f"at most {MAX_CP} critical points")
        mat.ncp = len(cp)
        for u, (A, Om, Ga, ph) in enumerate(cp):
            mat.cp_A[u], mat.cp_Omega[u], mat.cp_Gamma[u], mat.cp_phi[u] = A, Om, Ga, ph
        self._check(self.L.gnor_set_material(h, self.mask.ctypes.data, C.byref(mat)))
        self.design_shape = None
        if getattr(w, "design_lo", None) is not None:
            lo = (C.c_int32 * 3)(*w.design_lo)
            hi = (C.c_int32 * 3)(*w.design_hi)
            rho = np.ascontiguousarray(w.rho, dtype=np.float32)
            self.design_shape = tuple(int(b - a) for a, b in zip(w.design_lo[::-1], w.design_hi[::-1]))
            assert rho.shape == self.design_shape, (rho.shape, self.design_shape)
            self._check(self.L.gnor_set_design(h, lo, hi, rho.ctypes.data))
        src = SourceDesc(kind=w.src_kind, e0=w.e0, omega_c=w.omega_c, tau=w.tau, t0=w.t0,
                         omega_max=w.omega_max)
        self._check(self.L.gnor_set_source(h, C.byref(src)))
        self._omega = np.ascontiguousarray(w.omega, dtype=np.float64)
        mon = MonitorDesc(nfreq=len(self._omega), omega=_dp(self._omega), norm_k=w.norm_k,
                          dft_every=w.dft_every, flux_enabled=int(bool(w.flux)))
        mon.abs_lo[:] = list(w.abs_lo); mon.abs_hi[:] = list(w.abs_hi)
        mon.sca_lo[:] = list(w.sca_lo); mon.sca_hi[:] = list(w.sca_hi)
        self._check(self.L.gnor_set_monitors(h, C.byref(mon)))
        self._map_omega = np.ascontiguousarray(getattr(w, "map_omega", np.zeros(0)), dtype=np.float64)
        if len(self._map_omega):
            md = MapDesc(axis=w.map_axis, index=w.map_index, nmap=len(self._map_omega),
                         every=w.map_every, omega=_dp(self._map_omega))
            self._check(self.L.gnor_set_maps(h, C.byref(md)))
        nbytes = int(self.L.gnor_required_bytes(h))
        self.device = torch.device(device)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        self._check(self.L.gnor_set_graph_chunk(h, int(graph_chunk)))
        self._check(self.L.gnor_bind_memory(h, self.buffer.data_ptr(), nbytes,
                                            C.c_void_p(self.stream.cuda_stream)))
        self.nbytes = nbytes

    # ------------------------------------------------------------------ utils
    def _check(self, st: int):
        if st:
            raise GnorError(st, self.L.gnor_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            try:
                self.stream.synchronize()
            except Exception:
                pass
            self.L.gnor_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # -------------------------------------------------------------- stepping
    @property
    def step(self) -> int:
        return int(self.L.gnor_step_index(self.h))

    @property
    def dt(self) -> float:
        return self.w.courant * self.w.dx / 299792458.0

    def run(self, nsteps: int):
        self._check(self.L.gnor_run(self.h, int(nsteps)))

    def synchronize(self):
        self._check(self.L.gnor_synchronize(self.h))

    def flush_spectra(self):
        """Enqueue the fold of the flux samples staged since the last fold."""
        self._check(self.L.gnor_flush_spectra(self.h))

    def reset(self):
        self._check(self.L.gnor_reset(self.h))

    def set_watchdog(self, on: bool):
        """Non-finite scan of E after every chunk of steps inside run()."""
        self._check(self.L.gnor_set_watchdog(self.h, 1 if on else 0))

    def check_finite(self) -> bool:
        st = self.L.gnor_check_finite(self.h)
        if st == 7:
            return False
        self._check(st)
        return True

    # ---------------------------------------------------------------- output
    def field(self, name: str) -> np.ndarray:
        out = np.empty((self.w.nz, self.w.ny, self.w.nx), np.float64)
        self._check(self.L.gnor_get_field(self.h, FIELDS[name], _dp(out), out.size))
        return out

    def aux(self):
        n1 = self.w.nz + 50
        e1 = np.empty(n1); h1 = np.empty(n1)
        self._check(self.L.gnor_get_aux(self.h, _dp(e1), _dp(h1), n1))
        return e1, h1

    def dft(self):
        nf = len(self._omega)
        a = [np.empty((self.w.nz, nf)) for _ in range(4)]
        self._check(self.L.gnor_get_dft(self.h, *[_dp(x) for x in a]))
        return a[0] + 1j * a[1], a[2] + 1j * a[3]

    def maps(self) -> Dict[str, np.ndarray]:
        """Map transforms: Ex, Ey, Ez, n -> complex (nmap, nv, nu); inc ->
        complex (nmap,), the incident transform at norm_k."""
        w = self.w
        nm = len(self._map_omega)
        n = (w.nx, w.ny, w.nz)
        nu, nv = n[1 if w.map_axis == 0 else 0], n[1 if w.map_axis == 2 else 2]
        f = np.empty((8, nm, nv, nu))
        inc = np.empty((nm, 2))
        self._check(self.L.gnor_get_maps(self.h, _dp(f), _dp(inc), f.size))
        out = {k: f[2 * q] + 1j * f[2 * q + 1] for q, k in enumerate(("Ex", "Ey", "Ez", "n"))}
        out["inc"] = inc[:, 0] + 1j * inc[:, 1]
        return out

    def spectra(self) -> Dict[str, np.ndarray]:
        nf = len(self._omega)
        out = [np.empty(nf) for _ in range(4)]
        self._check(self.L.gnor_get_spectra(self.h, *[_dp(x) for x in out]))
        return dict(inc=out[0], ext=out[1], abs=out[2], sca=out[3])

    def save_state(self) -> bytearray:
        n = int(self.L.gnor_state_bytes(self.h))
        buf = bytearray(n)
        self._check(self.L.gnor_save_state(self.h, (C.c_char * n).from_buffer(buf), n))
        return buf

    def load_state(self, buf: bytearray):
        n = len(buf)
        self._check(self.L.gnor_load_state(self.h, (C.c_char * n).from_buffer(buf), n))

    def profile(self, nsteps: int) -> Dict[str, float]:
        """Average ms per launch of the H sweep, E/J sweep, spectra+staging and
        (amortised per step) flux accumulation, from HIP events."""
        ms = np.zeros(14)
        self._check(self.L.gnor_profile_kernels(self.h, int(nsteps), _dp(ms), 14))
        return dict(h=float(ms[0]), ej=float(ms[1]), dft=float(ms[2]), step=float(ms[3]),
                    flux_acc=float(ms[4]), h_cls=[float(v) for v in ms[5:9]],
                    ej_cls=[float(v) for v in ms[9:13]], aux=float(ms[13]), fused=bool(ms[3] > 0))

    def set_class_streams(self, on: bool):
        """Concurrent tile-class launches (default) or one after another."""
        self._check(self.L.gnor_set_class_streams(self.h, 1 if on else 0))

    def set_fused(self, on: bool):
        """One-pass fused step, or the two-sweep form."""
        self.set_mode(1 if on else 0)

    def set_mode(self, mode: int):
        """Step form: 0 two sweeps, 1 fused one-pass step, 2 hybrid (fused
        where no CPML slab is met, two sweeps elsewhere), 3 one-pass kernel
        for the plain tiles only."""
        self._check(self.L.gnor_set_fused(self.h, int(mode)))
        self.mode = int(mode)

    def tile_classes(self):
        """Tiles per class (plain Yee, CPML, metal, metal + CPML) of the current tiling."""
        c = (C.c_int32 * 4)()
        self._check(self.L.gnor_tile_classes(self.h, c))
        return [int(v) for v in c]

    def tile_class_cells(self):
        """Per class: grid cells its tiles cover, and (cell, axis) pairs among
        them inside that axis's CPML slab."""
        c = (C.c_int64 * 4)()
        d = (C.c_int64 * 4)()
        self._check(self.L.gnor_tile_class_cells(self.h, c, d))
        return [int(v) for v in c], [int(v) for v in d]

    def update_design(self, rho):
        """New design densities (z, y, x) in [0, 1] from a device tensor on this
        simulation's GPU (float32, contiguous) or any array (copied to the
        device first); the state is not reset."""
        import torch
        if isinstance(rho, torch.Tensor) and rho.device == self.device and rho.dtype == torch.float32:
            r = rho.contiguous()
        else:
            r = torch.as_tensor(np.asarray(rho, dtype=np.float32)).to(self.device)
        assert tuple(r.shape) == self.design_shape, (tuple(r.shape), self.design_shape)
        # the library reads r in stream order on the simulation's stream; wait
        # for that read, so that the caller may reuse rho at once
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.L.gnor_update_design(self.h, C.c_void_p(r.data_ptr())))
        self.stream.synchronize()

    def gradient(self, nsteps: int, ckpt_every: int, m_target: int, as_tensor: bool = False):
        """sigma_ext(omega[m_target]) of nsteps steps from rest and its exact
        adjoint gradient w.r.t. the design densities, shape (z, y, x): a numpy
        array, or with as_tensor a float64 device tensor."""
        import torch
        nbytes = int(self.L.gnor_gradient_required_bytes(self.h, int(nsteps), int(ckpt_every)))
        if nbytes == 0:
            raise GnorError(5, "no design region or memory not bound")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        g = torch.empty(self.design_shape, dtype=torch.float64, device=self.device)
        obj = C.c_double()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.L.gnor_gradient(self.h, int(nsteps), int(ckpt_every), int(m_target),
                                         C.c_void_p(ws.data_ptr()), nbytes, C.byref(obj),
                                         C.c_void_p(g.data_ptr())))
        del ws  # the call synchronised its stream
        return obj.value, (g if as_tensor else g.cpu().numpy())

    def set_tiling(self, ty: int, kz: int, xcd: int = 0):
        self._check(self.L.gnor_set_tiling(self.h, int(ty), int(kz), int(xcd)))

    def autotune(self, trial_steps: int = 20, cache: Optional[str] = None):
        """Pick the sweep tiling of the current step form by timing every
        candidate (library autotuner); results are cached in a JSON file keyed
        by grid shape, precision, metal-cell count and step form (default
        ~/.cache/gnorfdtd/tiling.json)."""
        import json
        path = cache or os.path.join(os.path.expanduser("~"), ".cache", "gnorfdtd", "tiling.json")
        key = (f"{self.w.nx}x{self.w.ny}x{self.w.nz}:{self.precision}:{int(np.count_nonzero(self.mask))}"
               f":form{self.mode}")
        table = {}
        if os.path.exists(path):
            try:
                table = json.load(open(path))
            except (OSError, ValueError):
                table = {}
        if key in table:
            e = table[key]
            self.set_tiling(e["ty"], e["kz"], e["xcd"])
            return dict(e, cached=True)
        ty, kz, xcd, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        self._check(self.L.gnor_autotune(self.h, int(trial_steps), C.byref(ty), C.byref(kz),
                                         C.byref(xcd), C.byref(ms)))
        table[key] = dict(ty=ty.value, kz=kz.value, xcd=xcd.value, ms=ms.value)
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as fh:
                json.dump(table, fh, indent=1)
        except OSError:
            pass
        return dict(table[key], cached=False)


class Batch:
    """Independent simulations stepped in lockstep; each phase of a step is one
    launch over the tiles of every instance (see gnor_batch_create)."""

    def __init__(self, sims, tiling=(2, 5, 2), graph_chunk: int = 64, form: int = 0):
        import torch
        L = load()
        self.L = L
        self.sims = list(sims)
        for s in self.sims:
            s.set_tiling(*tiling)
        arr = (C.c_void_p * len(self.sims))(*[s.h.value for s in self.sims])
        nbytes = int(L.gnor_batch_required_bytes(len(self.sims), arr))
        self.table = torch.empty(nbytes, dtype=torch.uint8, device=self.sims[0].device)
        h = C.c_void_p()
        st = L.gnor_batch_create(len(self.sims), arr, C.c_void_p(self.sims[0].stream.cuda_stream),
                                 C.c_void_p(self.table.data_ptr()), nbytes, C.byref(h))
        if st:
            raise GnorError(st, "gnor_batch_create rejected the instances")
        self.h = h
        self._check(L.gnor_batch_set_graph_chunk(h, int(graph_chunk)))
        for s in self.sims:
            s.mode = 0  # the library sets the instances to the batch's form
        self.set_form(form)

    def set_form(self, form: int):
        """Step form of the batch and of its instances: 0 two sweeps, 3 the
        tiles in one pass but those with metal and a y or z slab (as
        Sim.set_mode)."""
        self._check(self.L.gnor_batch_set_form(self.h, int(form)))
        self.form = int(form)
        for s in self.sims:
            s.mode = int(form)

    def _check(self, st: int):
        if st:
            raise GnorError(st, self.L.gnor_batch_last_error(self.h).decode())

    def run(self, nsteps: int):
        self._check(self.L.gnor_batch_run(self.h, int(nsteps)))

    def synchronize(self):
        self._check(self.L.gnor_batch_synchronize(self.h))

    @property
    def cells(self) -> int:
        return sum(s.w.cells for s in self.sims)

    def close(self):
        if getattr(self, "h", None):
            self.L.gnor_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def extinction_objective():
    """A torch.autograd.Function: sigma_ext at one frequency as a function of
    the design density tensor, differentiated by the library's adjoint."""
    import torch

    class ExtinctionObjective(torch.autograd.Function):
        """rho stays on the simulation's device; the adjoint runs in forward
        only when rho requires a gradient (otherwise only the objective's
        forward run)."""

        @staticmethod
        def forward(ctx, rho, sim, nsteps, ckpt_every, m_target):
            sim.update_design(rho.detach().to(device=sim.device, dtype=torch.float32))
            if ctx.needs_input_grad[0]:
                obj, grad = sim.gradient(nsteps, ckpt_every, m_target, as_tensor=True)
                ctx.save_for_backward(grad.to(device=rho.device, dtype=rho.dtype))
            else:
                sim.reset()
                sim.run(nsteps)
                obj = float(sim.spectra()["ext"][m_target])
            return rho.new_tensor(obj)

        @staticmethod
        def backward(ctx, gout):
            (g,) = ctx.saved_tensors
            return gout * g, None, None, None, None

    return ExtinctionObjective
