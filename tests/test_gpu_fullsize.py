"""Checks at the benchmark configurations' full sizes: a short run of the
320^3 grid against the oracle, element by element, and, where the oracle is
too slow, properties that hold at any size and FP32-vs-FP64 agreement.

* 320^3 grid in the benchmark's launch configuration, sphere moved down in z
  so the pulse reaches it within 100 steps: FP64 and FP32 paths against the
  FP64 oracle, every element of E, H and J and the spectra.

* 320^3 sphere (the benchmark workload, autotuned launch configuration):
  FP32 spectra within 1e-4 of the FP64 GPU path after 2400 steps and after
  the full 20 000; div H invariant in the FP64 run away from the TF surface
  and the CPML.
* The sphere workload's 2x-coarsened copy (160^3 at dx = 0.2 nm, 10 000
  steps): FP64 and FP32 spectra against the oracle's spectra of the same
  copy, stored by an oracle-only script.
* 640^3 star: the library's and the oracle's voxelisers agree bit for bit;
  FP32 vs FP64 spectra (all four) after a short early-pulse run.
* 160^3 design problem over its full 6000 steps: the FP64 adjoint gradient
  against central differences on 32 random voxels (each error against its
  own difference), the FP32 adjoint against the FP64 one.
* 64-instance batch in the benchmark's launch configuration: sampled
  instances equal their single runs bit for bit.
"""
import numpy as np
import pytest

from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_06997_amd import binding
    return binding


def test_sphere320_vs_oracle_in_the_benchmark_launch(B):
    """The benchmark grid (320^3, dx = 0.1 nm, 12-cell CPML, r = 10 nm sphere,
    GNOR metal) in the benchmark's launch configurations: tilings (4, 3, 2)
    in FP32 and (2, 4, 2) in FP64 (the ones the counters were taken at), and
    (2, 3, 2); graph chunks of 64 steps, concurrent tile classes.  The sphere
    sits as low in z as the monitor boxes allow (scattering box one cell above
    the CPML), so the incident pulse, launched three cells below the grid,
    enters the TF box after about 36 steps and the metal after about 43; 100
    steps then exercise every tile class (in step form 3 the metal tiles that
    meet only an x slab are class 2, and class 3 is empty here).  The oracle
    takes about a minute for them on 16 host threads."""
    import torch
    from oracle import oracle as orc
    from tests.helpers import oracle_problem
    n, dx, r = 320, 0.1e-9, 10.0e-9
    c = [(n - 1) / 2.0, (n - 1) / 2.0, 118.5]
    w = W.early_pulse(W.sphere_problem("sphere_r10nm_320^3_low", n, dx, 12, c, r, steps=100,
                                       precision="fp64"))
    w.omega = W.spectrum_omegas(20)
    w.norm_k = 20  # a plane the pulse has crossed (the centre plane has not seen it yet)
    assert w.sca_lo[2] == w.npml + 1
    steps = 100
    fields = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz")
    print(f"case 320^3 low sphere vs oracle, {steps} steps", flush=True)
    o = orc.OracleSim(oracle_problem(w, threads=16), oracle_mask(w))
    o.run(steps)
    ref = {f: o.get(f) for f in fields}
    sref = o.spectra()
    o.close()
    assert np.abs(ref["Jx"]).max() > 0  # the field has reached the metal
    assert np.abs(sref["inc"]).min() > 0
    # FP32 spectra: 1e-3 here.  After 100 steps the scattered flux is barely
    # above the FP32 rounding of the total-minus-incident cancellation at the
    # TF surface (measured 1.3e-4 for sigma_sca, 1e-8 for ext and abs); the
    # 1e-4 bound of full-length runs is checked below at 2400 steps.
    for prec, ftol, stol, mode, til in (("fp64", 1e-10, 1e-10, 0, (2, 3, 2)), ("fp32", 1e-3, 1e-3, 0, (2, 3, 2)),
                                        ("fp64", 1e-10, 1e-10, 3, (2, 4, 2)), ("fp32", 1e-3, 1e-3, 3, (4, 3, 2))):
        g = B.Sim(w, precision=prec)
        g.set_mode(mode)
        g.set_tiling(*til)
        cls = g.tile_classes()
        assert all(v > 0 for v in (cls[:3] if mode == 3 else cls)), cls
        g.run(steps)
        worst = {}
        for f in fields:
            a, b = g.field(f), ref[f]
            kin = max(np.linalg.norm(ref[h]) for h in fields if h[0] == f[0])
            worst[f] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-3 * kin))
        sg = g.spectra()
        for k in ("inc", "ext", "abs", "sca"):
            worst[k] = rel_l2(sg[k], sref[k])
        print(f"  {prec} step form {mode} tiling {til} rel-L2: " +
              ", ".join(f"{k} {v:.1e}" for k, v in worst.items()), flush=True)
        for f in fields:
            assert worst[f] <= ftol, (prec, f, worst[f])
        for k in ("inc", "ext", "abs", "sca"):
            assert worst[k] <= stol, (prec, k, worst[k])
        g.close()
        torch.cuda.empty_cache()


def test_sphere320_fp32_vs_fp64_and_div_h(B):
    import torch
    w = W.early_pulse(W.config2())
    steps = 2400
    print(f"case 320^3 sphere fp32 vs fp64, {steps} steps", flush=True)
    s32 = B.Sim(w, precision="fp32")
    s32.autotune(trial_steps=4)
    s32.run(steps)
    sp32 = s32.spectra()
    s32.close()
    torch.cuda.empty_cache()
    s64 = B.Sim(w, precision="fp64")
    s64.run(steps)
    sp64 = s64.spectra()
    for k in ("ext", "abs", "sca"):
        e = rel_l2(sp32[k], sp64[k])
        print(f"  {k}: fp32 vs fp64 rel-L2 {e:.3e}", flush=True)
        assert e <= 1e-4
    assert np.abs(sp64["ext"]).max() > 0
    # div H at cell centres stays zero away from the TF surface and the CPML
    Hx, Hy, Hz = s64.field("Hx"), s64.field("Hy"), s64.field("Hz")
    dh = ((Hx[:-1, :-1, 1:] - Hx[:-1, :-1, :-1]) + (Hy[:-1, 1:, :-1] - Hy[:-1, :-1, :-1]) +
          (Hz[1:, :-1, :-1] - Hz[:-1, :-1, :-1]))
    lo, hi = np.array(w.tf_lo), np.array(w.tf_hi)
    sl = tuple(slice(int(lo[a]) + 2, int(hi[a]) - 2) for a in (2, 1, 0))
    assert np.abs(dh[sl]).max() <= 1e-12 * np.abs(Hy).max()


def test_sphere320_full_length_fp32_vs_fp64(B):
    """The benchmark workload over its full 20 000 steps (about 3.3 ps, the
    resonance decayed): FP32 spectra within 1e-4 rel-L2 of the FP64 path,
    both in the benchmark's launch configuration (step form 3 at tilings
    (4, 3, 2) and (2, 4, 2), graph chunks, streamed stores)."""
    import torch
    w = W.config2()
    assert w.steps == 20000
    print(f"case 320^3 sphere fp32 vs fp64, {w.steps} steps", flush=True)
    spectra = {}
    for prec, til in (("fp32", (4, 3, 2)), ("fp64", (2, 4, 2))):
        s = B.Sim(w, precision=prec)
        s.set_mode(3)
        s.set_tiling(*til)
        s.run(w.steps)
        spectra[prec] = s.spectra()
        assert s.check_finite()
        s.close()
        torch.cuda.empty_cache()
    for k in ("ext", "abs", "sca"):
        e = rel_l2(spectra["fp32"][k], spectra["fp64"][k])
        print(f"  {k}: fp32 vs fp64 rel-L2 {e:.3e}", flush=True)
        assert e <= 1e-4
    ext = spectra["fp64"]["ext"]
    assert np.all(np.isfinite(ext)) and ext.max() > 0


def read_golden_spectra(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = np.array([[float(v) for v in line.split()] for line in open(path)
                     if line.strip() and not line.startswith("#")])
    return dict(omega=rows[:, 0], inc=rows[:, 1], ext=rows[:, 2], abs=rows[:, 3], sca=rows[:, 4])


def test_sphere_coarse_copy_vs_oracle_golden(B):
    """The 320^3 sphere workload's 2x-coarsened copy (160^3 at dx = 0.2 nm,
    8-cell CPML, the same particle, 10 000 steps = the same 3.3 fs) against
    the FP64 oracle's spectra of the same copy (tests/golden, written by an
    oracle-only script) on inc, ext, abs and sca: FP32 to 1e-4; FP64 to 1e-9
    here (1e-10 in the parity runs of at most 600 steps).  Over 10^4 steps
    the oracle's three-level P recursion, which forms P^{n+1} - P^n from
    values an O(w dt) fraction apart, loses about three digits of the current
    per step to FP64 rounding; the GPU's current form does not.  Measured
    2.7e-10 on sca, 9.4e-11 on ext, 4.8e-11 on abs."""
    import torch
    gold = read_golden_spectra("config2_coarse_oracle_spectra.txt")
    w = W.config2_coarse()
    assert w.steps == 10000 and np.allclose(gold["omega"], w.omega, rtol=1e-15)
    worst = {}
    for prec in ("fp64", "fp32"):
        print(f"case 160^3 coarsened sphere, {w.steps} steps, {prec} vs oracle golden", flush=True)
        s = B.Sim(w, precision=prec)
        s.run(w.steps)
        sp = s.spectra()
        s.close()
        torch.cuda.empty_cache()
        for k in ("inc", "ext", "abs", "sca"):
            worst[(prec, k)] = rel_l2(sp[k], gold[k])
            print(f"  {k}: rel-L2 {worst[(prec, k)]:.3e}", flush=True)
    for (prec, k), e in worst.items():
        assert e <= (1e-9 if prec == "fp64" else 1e-4), (prec, k, e)
    assert gold["ext"].max() > 0 and gold["sca"].max() > 0


def test_star640_masks_and_fp32_vs_fp64(B):
    import torch
    w = W.early_pulse(W.config3(seed=0))
    w.omega = W.spectrum_omegas(40)
    print("case 640^3 star: masks, fp32 vs fp64", flush=True)
    m_lib = B.voxelize(w)
    m_orc = oracle_mask(w)
    assert np.array_equal(m_lib, m_orc)
    del m_orc
    # 1000 steps: the scattered flux is then far above the FP32 rounding of
    # the total-minus-incident cancellation at the TF surface (after 600
    # steps sigma_sca differed by 9.9e-5 between FP32 and FP64)
    steps = 1000
    out = {}
    for prec in ("fp32", "fp64"):
        s = B.Sim(w, precision=prec, mask=m_lib)
        s.run(steps)
        out[prec] = (s.spectra(), s.check_finite())
        s.close()
        torch.cuda.empty_cache()
    assert out["fp32"][1] and out["fp64"][1]
    for k in ("inc", "ext", "abs", "sca"):
        e = rel_l2(out["fp32"][0][k], out["fp64"][0][k])
        print(f"  {k}: fp32 vs fp64 rel-L2 {e:.3e}", flush=True)
        assert e <= 1e-4
    assert np.abs(out["fp64"][0]["sca"]).max() > 0


def test_design160_gradient_vs_fd_on_32_voxels(B):
    """The adjoint workload as stated: 160^3, 60^3 design region, objective
    sigma_ext at 2.5 eV, 6000 steps, checkpoints every 500.  The FP64 adjoint
    against FP64 central differences (step 1/2048) on 32 seeded random
    voxels, each error measured against that voxel's own difference (floor:
    the objective's FP64 rounding over the run divided by the step); the FP32
    adjoint against the FP64 adjoint over the whole region and voxel by
    voxel."""
    import torch
    w = W.config5(0)
    w.omega = W.spectrum_omegas(9, 2.0, 3.0)  # 2.5 eV is index 4
    m = 4
    steps = w.steps
    assert steps == 6000
    print(f"case 160^3 design gradient ({steps} steps, checkpoints every 500): fp64 adjoint vs fd "
          "on 32 voxels, fp32 adjoint vs fp64", flush=True)
    s64 = B.Sim(w, precision="fp64")
    obj64, g64 = s64.gradient(steps, 500, m)
    s32 = B.Sim(w, precision="fp32")
    obj32, g32 = s32.gradient(steps, 500, m)
    s32.close()
    torch.cuda.empty_cache()
    e32 = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    gmax = float(np.abs(g64).max())
    print(f"  objective fp64 {obj64:.6e} fp32 {obj32:.6e}; gradient fp32 vs fp64 rel-L2 {e32:.2e}",
          flush=True)
    assert abs(obj32 - obj64) <= 1e-4 * abs(obj64)
    assert e32 <= 5e-3
    assert np.all(np.abs(g32 - g64) <= 0.05 * np.abs(g64) + 5e-3 * gmax)
    rho0 = np.array(w.rho, dtype=np.float32)
    rng = np.random.default_rng(11)

    def central(q, h):
        vals, pts = [], []
        for sgn in (+1, -1):
            r = rho0.copy()
            r[q] = np.float32(rho0[q] + sgn * h)
            pts.append(float(r[q]))  # the step actually taken in FP32
            s64.update_design(r)
            s64.reset()
            s64.run(steps)
            vals.append(s64.spectra()["ext"][m])
        return (vals[0] - vals[1]) / (pts[0] - pts[1])

    # central differences with h = 1/2048: their O(h^2) truncation, 3e-4 of
    # the derivative at h = 1/256 on some voxels, is 64 times smaller; the
    # floor is the objective's FP64 rounding over the run divided by the step
    h0 = 1.0 / 2048.0
    for t in range(32):
        q = tuple(int(rng.integers(0, n)) for n in g64.shape)
        h = min(h0, float(rho0[q]) / 2, (1.0 - float(rho0[q])) / 2)
        fd = central(q, h)
        floor = 1e-13 * abs(obj64) / h
        err = abs(fd - g64[q]) / max(abs(fd), floor)
        print(f"  voxel {q}: adjoint(fp64) {g64[q]:.8e} fd {fd:.8e} rel {err:.1e}; "
              f"adjoint(fp32) {g32[q]:.6e}", flush=True)
        assert err <= 1e-4, (q, g64[q], fd)
        assert np.sign(g32[q]) == np.sign(g64[q]) or abs(g64[q]) <= 5e-3 * gmax


@pytest.mark.parametrize("form", [0, 3])
def test_config4_batch_in_the_benchmark_launch(B, form):
    """All 64 instances batched as the benchmark runs them (tiling (4, 5, 2),
    graph chunks of 64, streaming stores chosen by the batch's total size, in
    either step form the benchmark may pick),
    with the pulse moved early so that it reaches every particle within the
    run: the smallest and the largest instance, the first gap dimer and the
    first single sphere equal their single runs bit for bit, and every
    instance stays finite."""
    fields = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz")
    ws = [W.early_pulse(w) for w in W.config4(seed=0, count=64)]
    steps = 400
    print(f"case config4 batch form {form}: {sum(w.cells for w in ws):.3e} cells, {steps} steps", flush=True)
    sims = [B.Sim(w, precision="fp32") for w in ws]
    bt = B.Batch(sims, tiling=(4, 5, 2), form=form)
    bt.run(steps)
    bt.synchronize()
    assert all(s.check_finite() for s in sims)
    q_small = min(range(len(ws)), key=lambda q: ws[q].cells)
    q_large = max(range(len(ws)), key=lambda q: ws[q].cells)
    q_dimer = next(q for q, w in enumerate(ws) if "dimer" in w.name)
    q_sphere = next(q for q, w in enumerate(ws) if "sphere" in w.name)
    for q in sorted({q_small, q_large, q_dimer, q_sphere}):
        print(f"  instance {ws[q].name}", flush=True)
        got = {f: sims[q].field(f) for f in fields}
        spec = sims[q].spectra()
        s = B.Sim(ws[q], precision="fp32")
        s.set_tiling(4, 5, 2)
        s.set_mode(form)
        s.run(steps)
        for f in fields:
            assert np.array_equal(s.field(f), got[f]), (ws[q].name, f)
        for k, v in s.spectra().items():
            assert np.array_equal(v, spec[k]), (ws[q].name, k)
        assert np.abs(got["Jx"]).max() > 0, ws[q].name
        s.close()
    bt.close()
