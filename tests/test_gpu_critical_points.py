"""Critical points (bound electrons, Eq. CritPoint; f3, Eq. critpointupdate)
on the HIP path, through the C-ABI, against the FP64 oracle.

FP64: E, H, J, the critical-point polarisations and the spectra agree with the
oracle to rel-L2 <= 1e-10 (rounding only: the oracle keeps the three-level
recursion, the GPU the increment form).  FP32: <= 1e-3 on fields, 1e-4 on
spectra.  A batch that mixes instances with and without poles reproduces the
instances run one by one bit for bit.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

BASE = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_06997_amd import binding
    return binding


def fields_of(w):
    return BASE + tuple(f"PC{p}{c}" for p in range(len(w.cp)) for c in "xyz")


def compare(g, o, w, ftol, stol):
    worst = {}
    names = fields_of(w)
    pairs = {f: (g.field(f), o.get(f)) for f in names}
    for f, (a, b) in pairs.items():
        kin = [h for h in pairs if h[:-1] == f[:-1]]  # same field, any component
        floor = 1e-3 * max(np.linalg.norm(pairs[h][1]) for h in kin)
        den = max(np.linalg.norm(b), floor)
        worst[f] = float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))
        assert np.isfinite(a).all(), f
    sg, so = g.spectra(), o.spectra()
    for k in ("inc", "ext", "abs", "sca"):
        worst[k] = rel_l2(sg[k], so[k])
    say("  rel-L2: " + ", ".join(f"{k} {v:.1e}" for k, v in worst.items()))
    for f in names:
        assert worst[f] <= ftol, (f, worst[f])
    for k in ("inc", "ext", "abs", "sca"):
        assert worst[k] <= stol, (k, worst[k])
    return worst


def oracle_run(w, steps):
    s = orc.OracleSim(oracle_problem(w, threads=8), oracle_mask(w))
    s.run(steps)
    return s


@pytest.mark.parametrize("seed", [0, 3])
def test_fp64_critical_points_vs_oracle(B, seed):
    w = W.with_critical_points(W.early_pulse(W.config1(seed)))
    w.omega = W.spectrum_omegas(24)
    say(f"case fp64 critical points config1 seed {seed}: {len(w.cp)} poles, {w.steps} steps")
    g = B.Sim(w, precision="fp64")
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    assert np.abs(o.get("PC1x")).max() > 0  # the poles respond
    compare(g, o, w, 1e-10, 1e-10)


def test_fp32_critical_points_vs_oracle(B):
    w = W.with_critical_points(W.early_pulse(W.config1(1)))
    w.omega = W.spectrum_omegas(24)
    say("case fp32 critical points config1 seed 1")
    g = B.Sim(w, precision="fp32")
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    compare(g, o, w, 1e-3, 1e-4)


@pytest.mark.parametrize("mode", [0, 2, 3])
def test_critical_points_in_metal_cpml_class(B, mode):
    """A sphere across x tiles 0 and 1 of a 160-wide grid: tile 0 holds the
    low x slab (metal + CPML class), tile 1 no slab (metal class), so both
    critical-point variants run; a ragged tiling; one pole with a positive
    phase."""
    n, dx, r = 160, 0.25e-9, 2.0e-9
    c = np.array([62.3, 23.5, 23.2])
    w = W.sphere_problem("wrap", n, dx, 8, c, r, steps=300)
    w.ny = w.nz = 48
    w = W._boxes(w, c * dx - r, c * dx + r)
    w = W.with_critical_points(W.early_pulse(w), poles=((0.9, 4.5e15, 8.0e14, 0.7),), eps_inf=1.3)
    w.omega = W.spectrum_omegas(20)
    say(f"case critical points across x tiles 160x48x48, tiling (4, 13, 2), step form {mode}")
    g = B.Sim(w, precision="fp64")
    g.set_mode(mode)  # hybrid: the metal class stays two-sweep (no f3 in the fused kernel)
    g.set_tiling(4, 13, 2)
    assert g.tile_classes()[2] > 0 and g.tile_classes()[3] > 0
    g.run(w.steps)
    o = oracle_run(w, w.steps)
    compare(g, o, w, 1e-10, 1e-10)


@pytest.mark.parametrize("form", [0, 3])
def test_batch_with_and_without_poles_bitwise(B, form):
    """Instances of 128^3 - 200^3, the 192^3 gap dimer with critical points.
    In step form 3 that instance keeps its metal tiles in the two sweeps
    while the 200^3 one takes them in one pass, as each would alone."""
    ws = [W.early_pulse(w) for w in W.config4(seed=1, count=3) + W.config4(seed=0, count=4)[3:]]
    ws[1] = W.with_critical_points(ws[1])
    for q, w in enumerate(ws):
        w.omega = W.spectrum_omegas(10 + 2 * q)
        w.flux = q == 1
    steps = 97
    say(f"case batch with critical points, form {form}: sizes {[w.nx for w in ws]}, "
        f"poles {[len(w.cp) for w in ws]}")
    solo = []
    for w in ws:
        s = B.Sim(w, precision="fp32")
        s.set_tiling(2, 8, 0)
        s.set_mode(form)
        s.run(steps)
        solo.append(({f: s.field(f) for f in fields_of(w)}, s.spectra()))
        s.close()
    sims = [B.Sim(w, precision="fp32") for w in ws]
    assert sims[1].tile_classes()[2] > 0 and sims[3].tile_classes()[2] > 0
    bt = B.Batch(sims, tiling=(2, 8, 0), form=form)
    bt.run(steps)
    bt.synchronize()
    for (fields, spec), s in zip(solo, sims):
        for f, v in fields.items():
            assert np.array_equal(s.field(f), v), (s.w.name, f)
        sp = s.spectra()
        for k in spec:
            assert np.array_equal(sp[k], spec[k]), (s.w.name, k)


def test_critical_points_refuse_fused_step(B):
    w = W.with_critical_points(W.config1(0))
    g = B.Sim(w, precision="fp32")
    with pytest.raises(B.GnorError):
        g.set_fused(True)
    g.run(4)
    assert g.check_finite()
