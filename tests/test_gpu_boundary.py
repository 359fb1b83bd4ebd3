"""The C-ABI's ownership and read-out contract on the GPU:

* the free-electron density n - n0 = div P_f^n / e at the nodes (Eq. Nsol),
  read through gnor_get_field, equals the oracle's P_f^n differenced on the
  host by the definition (backward differences at the nodes);
* design densities enter from a device array: equal to the same densities
  given at set-up, bit for bit; out-of-range values are refused and leave
  the densities unchanged;
* the gradient's workspace and a batch's tables are caller buffers whose
  size the library states (a short one is refused);
* the non-finite watchdog inside gnor_run reports a NaN planted in E from
  the host, and stays quiet when switched off.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask, oracle_problem

pytestmark = pytest.mark.gpu

QE = 1.602176634e-19  # C


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_06997_amd import binding
    return binding


def density_from_p(px, py, pz, dx):
    """div P at the nodes by backward differences (zero beyond the grid), / e."""
    d = px.copy()
    d[:, :, 1:] -= px[:, :, :-1]
    d += py
    d[:, 1:, :] -= py[:, :-1, :]
    d += pz
    d[1:, :, :] -= pz[:-1, :, :]
    return d / (dx * QE)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_density_matches_oracle(B, prec, tol):
    w = W.early_pulse(W.config1(2))
    steps = 420
    print(f"case density read-out {prec}: {w.name}, {steps} steps", flush=True)
    g = B.Sim(w, precision=prec)
    g.run(steps)
    n_gpu = g.field("n")
    o = orc.OracleSim(oracle_problem(w, threads=8), oracle_mask(w))
    o.run(steps)
    n_ref = density_from_p(o.get("Px"), o.get("Py"), o.get("Pz"), w.dx)
    o.close()
    e = np.linalg.norm(n_gpu - n_ref) / np.linalg.norm(n_ref)
    print(f"  rel-L2 {e:.2e}, peak {np.abs(n_ref).max():.3e} m^-3", flush=True)
    assert np.abs(n_ref).max() > 0
    assert e <= tol


def small_design(steps=300):
    w = W.early_pulse(W.config5_small(0))
    w.omega = W.spectrum_omegas(6, 2.0, 4.5)
    w.steps = steps
    return w


def test_design_from_device_equals_setup_and_refuses_bad_values(B):
    import torch
    from dataclasses import replace
    w = small_design()
    rho2 = np.asarray(W.design_direction(np.asarray(w.rho).shape, 5))
    rho2 = (1.0 / (1.0 + np.exp(-rho2))).astype(np.float32)  # a second density field in (0, 1)
    print("case design densities from a device array", flush=True)
    ref = B.Sim(replace(w, rho=rho2), precision="fp64")
    ref.run(w.steps)
    want = {f: ref.field(f) for f in ("Ex", "Hy", "Jx", "Jz")}
    s = B.Sim(w, precision="fp64")
    s.update_design(torch.from_numpy(rho2).to(s.device))
    s.run(w.steps)
    for f, v in want.items():
        assert np.array_equal(s.field(f), v), f
    # refused: a value above 1 and a NaN; the densities stay rho2
    for bad in (1.5, np.nan):
        r = rho2.copy()
        r[3, 4, 5] = bad
        with pytest.raises(B.GnorError) as ei:
            s.update_design(torch.from_numpy(r).to(s.device))
        assert ei.value.status == 1
    s.reset()
    s.run(w.steps)
    for f, v in want.items():
        assert np.array_equal(s.field(f), v), f


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_design_density_in_the_one_pass_metal_tiles(B, prec, tol):
    """Fractional densities (a design region) in step form 3, whose metal
    tiles without a slab take one pass with their weight of wp^2, beta^2 and D
    per point: fields, current and spectra equal the two-sweep form's up to
    rounding."""
    # the 160^3 design problem (its metal tiles away from the layers are
    # slab-free), with the pulse moved early
    w = W.early_pulse(W.config5(0))
    w.omega = W.spectrum_omegas(6, 2.0, 4.5)
    w.steps = 400
    print(f"case design densities 160^3, step form 3 vs 0, {prec}", flush=True)
    runs = []
    for form in (0, 3):
        g = B.Sim(w, precision=prec)
        g.set_mode(form)
        g.run(w.steps)
        runs.append(g)
    assert runs[1].tile_classes()[2] > 0
    for f in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz"):
        a, b = runs[1].field(f), runs[0].field(f)
        scale = max(np.linalg.norm(runs[0].field(h)) for h in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz",
                                                              "Jx", "Jy", "Jz") if h[0] == f[0])
        d = np.linalg.norm(a - b) / scale
        print(f"  {f}: {d:.2e}", flush=True)
        assert d <= tol, f
    assert np.abs(runs[0].field("Jx")).max() > 0
    sa, sb = runs[1].spectra(), runs[0].spectra()
    for k in ("inc", "ext"):
        assert np.linalg.norm(sa[k] - sb[k]) <= tol * np.linalg.norm(sb[k]), k


def test_caller_buffers_are_sized_by_the_library(B):
    import torch
    w = small_design(64)
    s = B.Sim(w, precision="fp32")
    L = s.L
    need = int(L.gnor_gradient_required_bytes(s.h, 64, 32))
    assert need > 0
    assert int(L.gnor_gradient_required_bytes(s.h, 64, 0)) == 0
    ws = torch.empty(need - 4096, dtype=torch.uint8, device=s.device)
    g = torch.empty(s.design_shape, dtype=torch.float64, device=s.device)
    obj = C.c_double()
    st = L.gnor_gradient(s.h, 64, 32, 1, C.c_void_p(ws.data_ptr()), need - 4096, C.byref(obj),
                         C.c_void_p(g.data_ptr()))
    assert st == 6  # GNOR_E_BUFFER_TOO_SMALL
    arr = (C.c_void_p * 1)(s.h.value)
    tb = int(L.gnor_batch_required_bytes(1, arr))
    assert tb > 0
    t = torch.empty(tb, dtype=torch.uint8, device=s.device)
    h = C.c_void_p()
    assert L.gnor_batch_create(1, arr, None, C.c_void_p(t.data_ptr()), tb - 256, C.byref(h)) == 6
    assert L.gnor_batch_create(1, arr, None, C.c_void_p(t.data_ptr()), tb, C.byref(h)) == 0
    L.gnor_batch_destroy(h)


def test_watchdog_reports_a_planted_nan(B):
    """A NaN written into E_x^0 (the first array of the saved state) before
    stepping: gnor_run returns GNOR_E_NONFINITE once the first chunk's scan
    has been read (while the second chunk runs), or gnor_synchronize does;
    with the watchdog off neither call complains and the explicit check finds
    the NaN."""
    w = W.early_pulse(W.config1(1))
    for on in (True, False):
        print(f"case watchdog {'on' if on else 'off'}: NaN planted in E_x", flush=True)
        s = B.Sim(w, precision="fp32")
        s.set_watchdog(on)
        buf = s.save_state()
        e = np.frombuffer(buf, dtype=np.float32, count=w.cells, offset=8)
        e.setflags(write=True)
        q = (w.nz // 2 * w.ny + w.ny // 2) * w.nx + w.nx // 2
        e[q] = np.nan
        s.load_state(buf)
        if on:
            with pytest.raises(B.GnorError) as ei:
                s.run(600)
                s.synchronize()
            assert ei.value.status == 7
            # the flag is sticky until reset
            with pytest.raises(B.GnorError):
                s.synchronize()
                s.run(600)
                s.synchronize()
            s.reset()
            s.run(600)
            s.synchronize()
            assert s.check_finite()
        else:
            s.run(600)
            s.synchronize()
            assert not s.check_finite()
        s.close()


@pytest.mark.parametrize("form", [0, 3])
def test_tile_class_cells_cover_the_grid(B, form):
    """Per-class cell counts (the bench's algorithmic bytes come from them):
    the tiles of the four classes cover every cell once, and the slab
    (cell, axis) pairs add up to the CPML's, 2 npml N / n per axis."""
    w = W.small_sphere(n=52, npml=6, seed=3)
    w.nx = 150  # three x tiles, the last ragged
    print(f"case tile class cells, form {form}", flush=True)
    g = B.Sim(w, precision="fp32")
    g.set_mode(form)
    g.set_tiling(4, 5, 2)
    cells, dirs = g.tile_class_cells()
    N = w.nx * w.ny * w.nz
    assert sum(cells) == N
    assert sum(dirs) == sum(2 * w.npml * N // n for n in (w.nx, w.ny, w.nz))
    assert cells[0] > 0 and cells[2] + cells[3] > 0
    g.close()
