"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

FP64 path: fields E^n, H^{n-1/2}, J^{n-1/2} and the four spectra agree with the
oracle to rel-L2 <= 1e-10 (the two implementations differ only in rounding:
the oracle's three-level P recursion and Eq. (GradDiv) term by term, the GPU's
current form with node scalars).  FP32 path: <= 1e-4 on the spectra.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

FIELDS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_06997_amd import binding
    return binding


def oracle_run(w, steps, **over):
    p = oracle_problem(w, threads=8, **over)
    s = orc.OracleSim(p, oracle_mask(w))
    s.run(steps)
    return s


def compare(gpu, ora, ftol, stol, fields=FIELDS, spectra=("inc", "ext", "abs", "sca")):
    """rel-L2 per field; a component that is rounding noise on both sides (e.g.
    E_y with no particle) is measured against 1e-3 of the largest component
    of the same field."""
    worst = {}
    pairs = {f: (gpu.field(f), ora.get(f)) for f in fields}
    for f, (a, b) in pairs.items():
        kin = [g for g in pairs if g[0] == f[0]]
        floor = 1e-3 * max(np.linalg.norm(pairs[g][1]) for g in kin)
        den = max(np.linalg.norm(b), floor)
        e = float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))
        worst[f] = e
        assert np.isfinite(a).all()
    sg, so = gpu.spectra(), ora.spectra()
    for k in spectra:
        worst[k] = rel_l2(sg[k], so[k])
    say("  rel-L2: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    for f in fields:
        assert worst[f] <= ftol, (f, worst[f])
    for k in spectra:
        assert worst[k] <= stol, (k, worst[k])
    return worst


@pytest.mark.parametrize("seed", range(5))
def test_fp64_config1_parity(B, seed):
    w = W.config1(seed)
    say(f"case fp64 config1 seed {seed}: {w.nx}^3, {w.steps} steps")
    g = B.Sim(w, precision="fp64")
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    worst = compare(g, o, 1e-10, 1e-10)
    say(f"  worst rel-L2 {max(worst.values()):.3e}")


def test_fp64_early_pulse_parity(B):
    w = W.early_pulse(W.config1(0))
    say("case fp64 config1 early pulse")
    g = B.Sim(w, precision="fp64")
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    assert np.abs(o.get("Jx")).max() > 1e3  # the metal responds strongly
    compare(g, o, 1e-10, 1e-10)


def test_flux_folds_split_at_any_step(B):
    """The flux-box transforms do not depend on where the staging windows are
    folded: a run read out or flushed at steps before, on and across the
    256-step window boundaries (each a fold of a partly filled window), then
    continued, ends with the spectra of an unbroken run to the rounding of
    the split sums, and with the oracle's."""
    w = W.early_pulse(W.config1(0))
    cuts = (5, 256, 300, 511, w.steps)
    say(f"case fp64 config1 early pulse, folds at steps {cuts}")
    a = B.Sim(w, precision="fp64")
    a.run(w.steps)
    sa = a.spectra()
    b = B.Sim(w, precision="fp64")
    done = 0
    for i, n in enumerate(cuts):
        b.run(n - done)
        done = n
        if i % 2:
            b.flush_spectra()
        else:
            b.spectra()
    sb = b.spectra()
    for k in ("inc", "ext", "abs", "sca"):
        e = rel_l2(sb[k], sa[k])
        say(f"  {k}: split vs unbroken {e:.2e}")
        assert e <= 1e-12, (k, e)
    assert np.abs(sa["sca"]).max() > 0
    o = oracle_run(w, w.steps)
    so = o.spectra()
    for k in ("abs", "sca"):
        assert rel_l2(sb[k], so[k]) <= 1e-10, k


def test_fp64_ragged_grid_and_general_cpml(B):
    """Sizes that are not multiples of the block shape; kappa > 1, alpha > 0;
    strong nonlocality (beta, D) and eps_inf != 1."""
    w = W.sphere_problem("ragged", 37, 0.25e-9, 5, [18.3, 17.2, 18.9], 1.3e-9, steps=300)
    w.ny = 38
    w.nz = 39
    w = W._boxes(w, w.spheres[0, :3] - 1.3e-9, w.spheres[0, :3] + 1.3e-9)
    w.pml_kappa_max = 3.0
    w.pml_alpha_max = 0.05
    w.beta = 2.0e6
    w.diff = 6.0e-4
    w.eps_inf = 1.7
    w = W.early_pulse(w)
    w.omega = W.spectrum_omegas(24)
    say("case fp64 ragged 37x38x39, kappa/alpha CPML, eps_inf 1.7")
    g = B.Sim(w, precision="fp64")
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    compare(g, o, 1e-10, 1e-10)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dielectric_background_n13(B, prec):
    """A sphere in a background of index 1.3 (eps_b = 1.69, the setting of the
    paper's Sec. V comparison with experiment): CPML, TF/SF line and the
    vacuum update all take eps_b; the metal keeps eps_inf = 1."""
    w = W.early_pulse(W.config1(4))
    w.eps_b = 1.69
    w.omega = W.spectrum_omegas(24)
    say(f"case background n = 1.3, {prec}")
    g = B.Sim(w, precision=prec)
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    tol = (1e-10, 1e-10) if prec == "fp64" else (1e-3, 1e-4)
    compare(g, o, *tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_and_two_sweep_forms_agree(B, prec):
    """The one-pass fused step and the two-sweep form (H sweep, then E/J
    sweep) compute the same update; both match the oracle."""
    w = W.early_pulse(W.config1(0))
    w.omega = W.spectrum_omegas(20)
    steps = 300
    say(f"case fused vs two-sweep, {prec}")
    runs = []
    for fused in (True, False):
        g = B.Sim(w, precision=prec)
        g.set_fused(fused)
        g.run(steps)
        runs.append(g)
    o = oracle_run(w, steps)
    tol = (1e-10, 1e-10) if prec == "fp64" else (1e-3, 1e-4)
    for g in runs:
        compare(g, o, *tol)
    # relative to the largest component of the same field (a component that
    # is rounding noise, e.g. H_x here, is compared at that scale)
    agree = 1e-12 if prec == "fp64" else 1e-5
    fa = {f: runs[0].field(f) for f in FIELDS}
    fb = {f: runs[1].field(f) for f in FIELDS}
    for f in FIELDS:
        scale = max(np.linalg.norm(fb[g]) for g in FIELDS if g[0] == f[0])
        d = np.linalg.norm(fa[f] - fb[f]) / scale
        say(f"  {f}: fused vs two-sweep {d:.2e}")
        assert d <= agree, f
    assert runs[0].profile(2)["fused"] and not runs[1].profile(2)["fused"]


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_metal_across_x_tiles_vs_oracle(B, mode):
    """A sphere straddling the boundary between x tiles 0 and 1 of a 160-wide
    grid: tile 0 holds the low x slab (class metal + CPML), tile 1 no slab
    (class metal).  Step forms: two sweeps, fused, hybrid (the metal tile
    fused, its metal + CPML neighbour two-sweep: each reads the other's H and
    node scalars), fused plain tiles (plain tiles in one pass beside
    two-sweep metal and CPML tiles)."""
    n, dx, r = 160, 0.25e-9, 2.0e-9
    c = np.array([62.3, 23.5, 23.2])
    w = W.sphere_problem("wrap", n, dx, 8, c, r, steps=300)
    w.ny = w.nz = 48
    w = W._boxes(w, c * dx - r, c * dx + r)
    w = W.early_pulse(w)
    w.omega = W.spectrum_omegas(20)
    say(f"case metal across x tiles 160x48x48, step form {mode}")
    g = B.Sim(w, precision="fp64")
    g.set_mode(mode)
    g.set_tiling(4, 16, 2)
    # (in form 3 the metal tiles that meet only the x slab join class 2)
    assert g.tile_classes()[2] > 0 and (mode == 3 or g.tile_classes()[3] > 0)
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    compare(g, o, 1e-10, 1e-10)


@pytest.mark.parametrize("prec,mode", [("fp32", 2), ("fp64", 2), ("fp32", 3), ("fp64", 3)])
def test_hybrid_and_two_sweep_forms_agree(B, prec, mode):
    """A 192 x 96 x 80 grid with a sphere across x tiles 0 and 1: every tile
    class occurs; the hybrid form (fused where no CPML slab is met), the form
    with fused plain tiles and the two-sweep form give the same fields and
    spectra up to rounding, through graph chunks and eager steps."""
    n, dx, r = 192, 0.25e-9, 3.0e-9
    c = np.array([66.3, 47.6, 39.2])
    w = W.sphere_problem("hybrid", n, dx, 8, c, r, steps=260)
    w.ny, w.nz = 96, 80
    w = W._boxes(w, c * dx - r, c * dx + r)
    w = W.early_pulse(w)
    w.omega = W.spectrum_omegas(16)
    say(f"case step form {mode} vs two-sweep 192x96x80, {prec}")
    runs = []
    for m in (0, mode):
        g = B.Sim(w, precision=prec)
        g.set_mode(m)
        g.run(w.steps)
        runs.append(g)
    # every class occurs (in form 3 the metal tiles that meet only the x slab
    # join class 2, and class 3 may be empty)
    assert min(runs[1].tile_classes()[:3 if mode == 3 else 4]) > 0
    agree = 1e-12 if prec == "fp64" else 1e-5
    fa = {f: runs[0].field(f) for f in FIELDS}
    fb = {f: runs[1].field(f) for f in FIELDS}
    for f in FIELDS:
        scale = max(np.linalg.norm(fa[g]) for g in FIELDS if g[0] == f[0])
        d = np.linalg.norm(fa[f] - fb[f]) / scale
        say(f"  {f}: form {mode} vs two-sweep {d:.2e}")
        assert d <= agree, f
    sa, sb = runs[0].spectra(), runs[1].spectra()
    for k in ("inc", "ext", "abs", "sca"):
        assert rel_l2(sb[k], sa[k]) <= agree, k


@pytest.mark.parametrize("prec,tol,tiling", [("fp64", (1e-10, 1e-10), (2, 4, 0)),
                                             ("fp64", (1e-10, 1e-10), (8, 3, 1)),
                                             ("fp32", (1e-3, 1e-4), (2, 4, 0)),
                                             ("fp32", (1e-3, 1e-4), (4, 5, 2))])
def test_fused_plain_tiles_at_the_grid_walls_vs_oracle(B, prec, tol, tiling):
    """No CPML (a PEC box): the plain tiles of the one-pass kernel touch the
    walls on every face, and the grid is ragged in x (72 = 64 + 8) and y (41
    rows: partial blocks of 4 and 8 rows), so the kernel's range guards, its
    idle lanes and rows, the shared rows and the recomputed halos all act;
    against the oracle, with a sphere inside the TF box."""
    c = np.array([35.3, 20.2, 21.6])
    w = W.sphere_problem("walls", 72, 0.25e-9, 0, c, 1.6e-9, steps=240)
    w.ny, w.nz = 41, 44
    w = W._boxes(w, c * 0.25e-9 - 1.6e-9, c * 0.25e-9 + 1.6e-9)
    w = W.early_pulse(w)
    w.omega = W.spectrum_omegas(16)
    say(f"case fused plain tiles at the walls 72x41x44, {prec}, tiling {tiling}")
    g = B.Sim(w, precision=prec)
    g.set_mode(3)
    g.set_tiling(*tiling)
    assert g.tile_classes()[0] > 0
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    compare(g, o, *tol)


@pytest.mark.parametrize("prec,tol,tiling", [("fp64", (1e-10, 1e-10), (2, 4, 0)),
                                             ("fp64", (1e-10, 1e-10), (4, 5, 2)),
                                             ("fp64", (1e-10, 1e-10), (8, 3, 1)),
                                             ("fp32", (1e-3, 1e-4), (2, 3, 2))])
def test_one_pass_cpml_tiles_vs_oracle(B, prec, tol, tiling):
    """Step form 3 runs the CPML tiles (a y or z slab, maybe an x slab too)
    in one pass as well.  A 72 x 41 x 44 grid, ragged in x and y, with a
    6-cell CPML and the TF box one cell from the layers (the least distance
    allowed), so that the shell of the box, and with it the TF/SF launch of
    the CPML class, reaches into CPML tiles; a sphere inside.  Against the
    oracle, at tilings whose tiles straddle the slab boundaries in y and z."""
    c = np.array([35.3, 20.2, 21.6])
    w = W.sphere_problem("cpml_one_pass", 72, 0.25e-9, 6, c, 1.6e-9, steps=260)
    w.ny, w.nz = 41, 44
    w = W._boxes(w, c * 0.25e-9 - 1.6e-9, c * 0.25e-9 + 1.6e-9)
    w.flux = False
    w.tf_lo = (7, 7, 7)
    w.tf_hi = (w.nx - 8, w.ny - 8, w.nz - 8)
    w = W.early_pulse(w)
    w.omega = W.spectrum_omegas(16)
    say(f"case one-pass CPML tiles 72x41x44, {prec}, tiling {tiling}")
    g = B.Sim(w, precision=prec)
    g.set_mode(3)
    g.set_tiling(*tiling)
    assert g.tile_classes()[1] > 0
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    compare(g, o, *tol, spectra=("inc", "ext"))


def test_fp64_vacuum_no_metal(B):
    w = W.early_pulse(W.small_sphere(n=30, radius=1.0e-9, npml=4, seed=4))
    w.omega = W.spectrum_omegas(10)
    say("case fp64 vacuum (no metal)")
    mask = np.zeros((w.nz, w.ny, w.nx), np.uint8)
    g = B.Sim(w, precision="fp64", mask=mask)
    g.run(250)
    p = oracle_problem(w, threads=8)
    o = orc.OracleSim(p, mask)
    o.run(250)
    compare(g, o, 1e-10, 1e-10, fields=("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"), spectra=("inc", "abs"))
    assert np.abs(g.spectra()["ext"]).max() == 0.0


def test_fp32_config1_vs_oracle(B):
    w = W.early_pulse(W.config1(1))
    say("case fp32 config1 early pulse vs fp64 oracle")
    g = B.Sim(w, precision="fp32")
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    worst = compare(g, o, 1e-3, 1e-4)
    say(f"  fp32 worst field {max(worst[f] for f in FIELDS):.3e} spectra "
        f"{max(worst[k] for k in ('inc', 'ext', 'abs', 'sca')):.3e}")


@pytest.mark.parametrize("ty,kz,xcd", [(2, 8, 1), (8, 13, 0), (4, 48, 1), (4, 8, 2), (2, 2, 2),
                                        (4, 5, 2)])
def test_tilings_agree_with_oracle(B, ty, kz, xcd):
    """Every sweep tiling (including a kz that does not divide nz) reproduces
    the oracle; only reduction orders of the spectra differ."""
    w = W.early_pulse(W.config1(1))
    w.omega = W.spectrum_omegas(20)
    say(f"case tiling ty={ty} kz={kz} xcd={xcd}")
    g = B.Sim(w, precision="fp64")
    g.set_tiling(ty, kz, xcd)
    g.run(300)
    o = oracle_run(w, 300)
    compare(g, o, 1e-10, 1e-10)


def test_autotuner_picks_a_tiling_and_resets(B, tmp_path):
    w = W.early_pulse(W.config1(2))
    say("case autotuner")
    g = B.Sim(w, precision="fp32")
    r = g.autotune(trial_steps=3, cache=str(tmp_path / "tiles.json"))
    assert r["ty"] in (2, 4, 8) and 1 <= r["kz"] <= w.nz and not r["cached"]
    assert g.step == 0
    r2 = g.autotune(cache=str(tmp_path / "tiles.json"))
    assert r2["cached"] and (r2["ty"], r2["kz"]) == (r["ty"], r["kz"])
    g.run(100)
    h = B.Sim(w, precision="fp32")
    h.set_tiling(r["ty"], r["kz"], r["xcd"])
    h.run(100)
    for f in FIELDS:
        assert np.array_equal(g.field(f), h.field(f)), f


def test_graph_replay_equals_eager_bitwise(B):
    w = W.early_pulse(W.config1(2))
    say("case graph chunks vs eager launches")
    a = B.Sim(w, precision="fp64", graph_chunk=0)
    b = B.Sim(w, precision="fp64", graph_chunk=64)
    a.run(7); a.run(190)
    b.run(7); b.run(190)  # odd start: eager steps until aligned, then graphs
    for f in FIELDS:
        assert np.array_equal(a.field(f), b.field(f)), f
    sa, sb = a.spectra(), b.spectra()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k


def test_serial_classes_profiled_steps_and_reset_are_bitwise_neutral(B):
    """The tile classes of a sweep update disjoint tiles: launching them one
    after another instead of concurrently on their streams, stepping through
    the profiler (events around every sweep) and rerunning after gnor_reset
    change no bit of the fields or spectra."""
    w = W.early_pulse(W.config1(1))
    w.omega = W.spectrum_omegas(16)
    steps = w.steps
    say(f"case serial classes, profiled steps and reset vs concurrent classes, {steps} steps")
    ref = B.Sim(w, precision="fp32")
    ref.run(steps)
    want = ({f: ref.field(f) for f in FIELDS}, ref.spectra())
    ser = B.Sim(w, precision="fp32")
    ser.set_class_streams(False)
    ser.run(steps)
    pro = B.Sim(w, precision="fp32")
    pr = pro.profile(steps)
    assert pro.step == steps and pr["h"] > 0
    ref.reset()
    assert ref.step == 0
    ref.run(steps)
    for name, s in (("serial", ser), ("profiled", pro), ("reset", ref)):
        for f in FIELDS:
            assert np.array_equal(s.field(f), want[0][f]), (name, f)
        for k, v in s.spectra().items():
            assert np.array_equal(v, want[1][k]), (name, k)
    assert np.abs(want[0]["Jx"]).max() > 0


def test_resume_from_snapshot_is_bitwise(B):
    w = W.early_pulse(W.config1(3))
    say("case save/load state resume")
    a = B.Sim(w, precision="fp32")
    a.run(200)
    snap = a.save_state()
    a.run(150)
    ref = {f: a.field(f) for f in FIELDS}
    sref = a.spectra()
    b = B.Sim(w, precision="fp32")
    b.load_state(snap)
    assert b.step == 200
    b.run(150)
    for f in FIELDS:
        assert np.array_equal(b.field(f), ref[f]), f
    for k, v in b.spectra().items():
        assert np.array_equal(v, sref[k]), k


def test_step_forms_switch_mid_run_and_resume(B):
    """Switching step forms at odd and even steps keeps every double-buffered
    state array (fields, currents, node scalars, CPML memories) where the
    next form reads it (against the oracle), and a snapshot taken in the
    fused form resumes bit for bit in a fresh simulation that continues in
    the hybrid and two-sweep forms."""
    w = W.early_pulse(W.config1(1))
    w.omega = W.spectrum_omegas(16)
    say("case step forms 0 -> 1 (step 101) -> snapshot (160) -> 2 -> 0 (212), fp64")
    g = B.Sim(w, precision="fp64")
    g.run(101)
    g.set_mode(1)
    g.run(59)
    snap = g.save_state()
    g.set_mode(2)
    g.run(52)
    g.set_mode(0)
    g.run(88)
    compare(g, oracle_run(w, 300), 1e-10, 1e-10)
    h = B.Sim(w, precision="fp64")
    h.load_state(snap)
    assert h.step == 160
    h.set_mode(2)
    h.run(52)
    h.set_mode(0)
    h.run(88)
    for f in FIELDS:
        assert np.array_equal(h.field(f), g.field(f)), f
    sg, sh = g.spectra(), h.spectra()
    for k in sg:
        assert np.array_equal(sh[k], sg[k]), k


def test_nonfinite_watchdog(B):
    """A NaN planted from the host in a snapshot is reported (no kernel is
    made to fail)."""
    w = W.config1(4)
    say("case non-finite watchdog")
    a = B.Sim(w, precision="fp64")
    a.run(4)
    assert a.check_finite()
    snap = a.save_state()
    arr = np.frombuffer(snap, dtype=np.uint8)
    # the E^n component x starts the state region (after the 8-byte step index)
    # at parity 0 (4 steps done): plant a NaN in its middle
    n = w.nx * w.ny * w.nz
    e = np.frombuffer(snap, dtype=np.float64, count=n, offset=8)
    e.setflags(write=True)
    e[n // 2] = np.nan
    a.load_state(snap)
    assert not a.check_finite()
