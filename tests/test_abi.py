"""C-ABI contract checks that need no GPU: the library loads and exports every
function include/gnor_fdtd.h declares; host-side validation returns the
documented status codes; the library's voxelisers match the oracle's
independent voxelisers bit for bit."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2005_06997_amd import binding as B
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask


@pytest.fixture(scope="module")
def lib():
    return B.load()


def test_exports_every_declared_function(lib):
    names = B.header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for code in range(8):
        assert lib.gnor_status_string(code)


def _grid(w, **over):
    g = B.GridDesc(nx=w.nx, ny=w.ny, nz=w.nz, dx=w.dx, courant=w.courant, npml=w.npml,
                   pml_order=3.0, pml_sigma_scale=0.8, pml_kappa_max=1.0, pml_alpha_max=0.0,
                   eps_background=1.0, precision=B.GNOR_FP64)
    g.tf_lo[:] = list(w.tf_lo)
    g.tf_hi[:] = list(w.tf_hi)
    for k, v in over.items():
        setattr(g, k, v)
    return g


def _create(lib, g):
    h = C.c_void_p()
    st = lib.gnor_create(C.byref(g), C.byref(h))
    return st, h


def test_create_rejects_unstable_courant(lib):
    w = W.config1(0)
    st, h = _create(lib, _grid(w, courant=0.6))
    assert st == 2  # GNOR_E_UNSTABLE
    st, h = _create(lib, _grid(w, courant=0.0))
    assert st == 2
    st, h = _create(lib, _grid(w, courant=0.5))
    assert st == 0
    lib.gnor_destroy(h)


def test_create_rejects_bad_sizes_and_boxes(lib):
    w = W.config1(0)
    assert _create(lib, _grid(w, nx=0))[0] == 1
    assert _create(lib, _grid(w, dx=-1.0))[0] == 1
    assert _create(lib, _grid(w, precision=7))[0] == 1
    g = _grid(w)
    g.tf_lo[0] = w.npml  # TF box touching the CPML
    assert _create(lib, g)[0] == 1
    # substrate: negative permittivity or a plane outside the grid
    assert _create(lib, _grid(w, eps_substrate=-1.0))[0] == 1
    assert _create(lib, _grid(w, eps_substrate=2.25, substrate_k=w.nz))[0] == 1
    st, h = _create(lib, _grid(w, eps_substrate=2.25, substrate_k=w.nz - 1))
    assert st == 0
    lib.gnor_destroy(h)


def test_material_outside_tf_rejected_and_run_before_bind(lib):
    w = W.config1(0)
    st, h = _create(lib, _grid(w))
    assert st == 0
    mask = np.zeros((w.nz, w.ny, w.nx), np.uint8)
    mask[w.tf_lo[2] + 1, 24, 24] = 1  # one cell inside the TF box: too close to its face
    mat = B.MaterialDesc(wp=W.WP, gamma=W.GAMMA, beta=W.BETA, diffusion=W.DIFF, eps_inf=1.0)
    assert lib.gnor_set_material(h, mask.ctypes.data, C.byref(mat)) == 1
    assert b"TF box" in lib.gnor_last_error(h)
    mask[:] = 0
    mask[24, 24, 24] = 8  # bits above 2 are not allowed
    assert lib.gnor_set_material(h, mask.ctypes.data, C.byref(mat)) == 1
    mask[:] = 0
    mask[24, 24, 24] = 7
    assert lib.gnor_set_material(h, mask.ctypes.data, C.byref(mat)) == 0
    assert lib.gnor_run(h, 1) == 5  # GNOR_E_STATE: nothing bound
    assert lib.gnor_required_bytes(h) > 0
    lib.gnor_destroy(h)


@pytest.mark.parametrize("seed", range(5))
def test_sphere_masks_bit_exact_vs_oracle(seed):
    w = W.config1(seed)
    assert np.array_equal(B.voxelize(w), oracle_mask(w))


def test_dimer_and_batch_masks_bit_exact_vs_oracle():
    for w in W.config4(seed=0, count=6):
        assert np.array_equal(B.voxelize(w), oracle_mask(w))


@pytest.mark.parametrize("seed", [0, 1])
def test_star_mask_bit_exact_vs_oracle(seed):
    w = W.config3(seed=seed, n=200, dx=0.4e-9)
    a = B.voxelize(w)
    b = oracle_mask(w)
    assert a.any()
    assert np.array_equal(a, b)


def test_binding_structs_match_the_header(tmp_path):
    """sizeof and field offsets of the ABI structs as the C compiler lays them
    out, against the ctypes mirrors in the binding."""
    import os
    import subprocess

    structs = {"gnor_grid_desc": B.GridDesc, "gnor_material_desc": B.MaterialDesc,
               "gnor_source_desc": B.SourceDesc, "gnor_monitor_desc": B.MonitorDesc,
               "gnor_map_desc": B.MapDesc}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gnor_fdtd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_material_rejects_bad_critical_points(lib):
    w = W.config1(0)
    st, h = _create(lib, _grid(w))
    assert st == 0
    mask = oracle_mask(w)
    m = B.MaterialDesc(wp=w.wp, gamma=w.gamma, beta=w.beta, diffusion=w.diff, eps_inf=1.0)
    m.ncp = 5
    mp = mask.ctypes.data_as(C.c_void_p)
    assert lib.gnor_set_material(h, mp, C.byref(m)) == 1  # GNOR_E_INVALID_ARG
    m.ncp = 1
    m.cp_A[0], m.cp_Omega[0], m.cp_Gamma[0], m.cp_phi[0] = 1.0, 4e15, -1.0, 0.0
    assert lib.gnor_set_material(h, mp, C.byref(m)) == 1
    m.cp_Gamma[0] = 5e14
    assert lib.gnor_set_material(h, mp, C.byref(m)) == 0
    assert lib.gnor_set_fused(h, 1) == 1
    lib.gnor_destroy(h)


def test_new_entry_points_validate_on_the_host(lib):
    """Host-side checks of the caller-buffer and watchdog entry points (no
    device work: each returns before any HIP call)."""
    w = W.config1(0)
    st, h = _create(lib, _grid(w))
    assert st == 0
    assert lib.gnor_set_watchdog(h, 2) == 1
    assert lib.gnor_set_watchdog(h, 0) == 0
    assert lib.gnor_gradient_required_bytes(h, 100, 10) == 0  # not bound, no design region
    assert lib.gnor_batch_required_bytes(0, None) == 0
    arr = (C.c_void_p * 1)(h.value)
    out = C.c_void_p()
    assert lib.gnor_batch_create(1, arr, None, None, 0, C.byref(out)) == 1  # no table
    assert lib.gnor_batch_set_form(None, 3) == 1  # no batch
    assert lib.gnor_update_design(h, None) == 5  # not bound
    assert lib.gnor_flush_spectra(h) == 5
    lib.gnor_destroy(h)


def test_total_field_operation_validates_on_the_host(lib):
    """Total-field grids: the source plane must lie between the absorbing
    layers; no substrate, flux boxes, design region or fused form 1; metal may
    reach into the layers but not onto the outer node planes."""
    w = W.config1(0)
    n, L = w.nz, w.npml
    for k, ok in ((L, False), (L + 1, True), (n - 2 - L, True), (n - 1 - L, False)):
        st, h = _create(lib, _grid(w, total_field=1, source_k=k, tf_lo=(0, 0, 0), tf_hi=(0, 0, 0)))
        assert (st == 0) == ok, k
        if st == 0:
            lib.gnor_destroy(h)
    st, h = _create(lib, _grid(w, total_field=2, source_k=L + 1))
    assert st == 1
    st, h = _create(lib, _grid(w, total_field=1, source_k=L + 1, eps_substrate=2.25, substrate_k=n // 2))
    assert st == 1
    st, h = _create(lib, _grid(w, total_field=1, source_k=L + 1))
    assert st == 0
    mat = B.MaterialDesc(wp=w.wp, gamma=w.gamma, beta=w.beta, diffusion=w.diff, eps_inf=1.0)
    m = np.zeros((w.nz, w.ny, w.nx), np.uint8)
    m[n // 2:n // 2 + 4, 1:w.ny - 1, 1:w.nx - 1] = 7  # through the x and y layers
    assert lib.gnor_set_material(h, m.ctypes.data_as(C.c_void_p), C.byref(mat)) == 0
    m[n // 2, 0, 5] = 7  # on an outer node plane
    assert lib.gnor_set_material(h, m.ctypes.data_as(C.c_void_p), C.byref(mat)) == 1
    m[n // 2, 0, 5] = 0
    assert lib.gnor_set_material(h, m.ctypes.data_as(C.c_void_p), C.byref(mat)) == 0
    assert lib.gnor_set_fused(h, 1) == 1
    for form in (0, 2, 3):
        assert lib.gnor_set_fused(h, form) == 0
    lo = (C.c_int32 * 3)(10, 10, 10)
    hi = (C.c_int32 * 3)(12, 12, 12)
    rho = np.full(8, 0.5, np.float32)
    assert lib.gnor_set_design(h, lo, hi, rho.ctypes.data_as(C.c_void_p)) == 1
    om = np.array([4e15])
    mon = B.MonitorDesc(nfreq=1, omega=om.ctypes.data_as(C.POINTER(C.c_double)), norm_k=L + 1,
                        dft_every=1, flux_enabled=1)
    assert lib.gnor_set_monitors(h, C.byref(mon)) == 1
    mon.flux_enabled = 0
    assert lib.gnor_set_monitors(h, C.byref(mon)) == 0
    lib.gnor_destroy(h)
