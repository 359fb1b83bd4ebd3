"""Checks at the benchmark configurations' full sizes, where the oracle is too
slow to run: properties that hold at any size and FP32-vs-FP64 agreement.

* 320^3 sphere (the benchmark workload, autotuned launch configuration):
  FP32 spectra within 1e-4 of the FP64 GPU path; div H invariant in the FP64
  run away from the TF surface and the CPML.
* 640^3 star: the library's and the oracle's voxelisers agree bit for bit;
  FP32 vs FP64 spectra after a short early-pulse run.
* 160^3 design problem: FP32 adjoint gradient vs central differences of the
  FP64 objective on random voxels.
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


def test_star640_masks_and_fp32_vs_fp64(B):
    import torch
    w = W.early_pulse(W.config3(seed=0))
    w.omega = W.spectrum_omegas(40)
    print("case 640^3 star: masks, fp32 vs fp64", flush=True)
    m_lib = B.voxelize(w)
    m_orc = oracle_mask(w)
    assert np.array_equal(m_lib, m_orc)
    del m_orc
    steps = 600
    out = {}
    for prec in ("fp32", "fp64"):
        s = B.Sim(w, precision=prec, mask=m_lib)
        s.run(steps)
        out[prec] = (s.spectra(), s.check_finite())
        s.close()
        torch.cuda.empty_cache()
    assert out["fp32"][1] and out["fp64"][1]
    for k in ("inc", "ext"):
        e = rel_l2(out["fp32"][0][k], out["fp64"][0][k])
        print(f"  {k}: fp32 vs fp64 rel-L2 {e:.3e}", flush=True)
        assert e <= 1e-4


def test_design160_fp32_gradient_vs_fd(B):
    w = W.early_pulse(W.config5(0))
    w.omega = W.spectrum_omegas(9, 2.0, 3.0)  # 2.5 eV is index 4
    m = 4
    steps = 3000
    print(f"case 160^3 design gradient fp32 ({steps} steps, checkpoints every 500) vs fd(fp64)",
          flush=True)
    s32 = B.Sim(w, precision="fp32")
    obj, g = s32.gradient(steps, 500, m)
    s64 = B.Sim(w, precision="fp64")
    rho0 = np.array(w.rho, dtype=np.float32)
    rng = np.random.default_rng(11)
    errs = []
    for _ in range(6):
        q = tuple(int(rng.integers(0, n)) for n in g.shape)
        h = min(1.0 / 64.0, float(rho0[q]) / 2, (1.0 - float(rho0[q])) / 2)
        vals, pts = [], []
        for sgn in (+1, -1):
            r = rho0.copy()
            r[q] = np.float32(rho0[q] + sgn * h)
            pts.append(float(r[q]))
            s64.update_design(r)
            s64.reset()
            s64.run(steps)
            vals.append(s64.spectra()["ext"][m])
        fd = (vals[0] - vals[1]) / (pts[0] - pts[1])
        errs.append(abs(fd - g[q]) / np.abs(g).max())
        print(f"  voxel {q}: adjoint(fp32) {g[q]:.6e} fd(fp64) {fd:.6e}", flush=True)
    assert max(errs) <= 2e-3
