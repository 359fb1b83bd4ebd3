"""Batched launches over many instances (spheres and gap dimers of uneven
grid sizes, per-instance beta and D) reproduce the instances run one by one
bit for bit, and the batch reproduces the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

FIELDS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz")


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_06997_amd import binding
    return binding


def instances(count=5, seed=0):
    ws = [W.early_pulse(w) for w in W.config4(seed=seed, count=count)]
    for q, w in enumerate(ws):
        w.omega = W.spectrum_omegas(12 + 4 * q)  # uneven frequency counts
        w.flux = (q % 2 == 1)
    return ws


@pytest.mark.parametrize("prec,tiling,form", [("fp32", (2, 8, 0), 0), ("fp64", (2, 8, 0), 0),
                                              ("fp32", (2, 3, 2), 0), ("fp32", (4, 4, 1), 0),
                                              ("fp32", (2, 5, 2), 3), ("fp64", (2, 3, 2), 3),
                                              ("fp32", (4, 4, 1), 3), ("fp64", (8, 4, 0), 3)])
def test_batch_equals_individual_runs_bitwise(B, prec, tiling, form):
    """Also with the XCD-aware tile orders 1 and 2, under which the
    instances' block ranges are spaced apart by idle blocks; in the two-sweep
    form and in the form with the tiles without metal in one pass (whose
    TF/SF launch covers every instance's shell)."""
    ws = instances()
    print(f"case batch {prec} tiling {tiling} form {form}: sizes {[w.nx for w in ws]}", flush=True)
    steps = 131  # odd: eager steps around graph chunks
    solo, fused = [], []
    for w in ws:
        s = B.Sim(w, precision=prec)
        s.set_tiling(*tiling)
        s.set_mode(form)  # the batch's step form
        s.run(steps)
        solo.append(({f: s.field(f) for f in FIELDS}, s.spectra()))
        s.close()
        s = B.Sim(w, precision=prec)
        s.set_fused(True)
        s.run(steps)
        fused.append(s.spectra())
        s.close()
    sims = [B.Sim(w, precision=prec) for w in ws]
    bt = B.Batch(sims, tiling=tiling, form=form)
    bt.run(steps)
    bt.synchronize()
    for (fields, spec), s in zip(solo, sims):
        assert s.step == steps
        for f in FIELDS:
            assert np.array_equal(s.field(f), fields[f]), (s.w.name, f)
        sp = s.spectra()
        for k in spec:
            assert np.array_equal(sp[k], spec[k]), (s.w.name, k)
    # the fused one-pass step gives the same spectra up to rounding
    tol = 1e-5 if prec == "fp32" else 1e-12
    for f_spec, s in zip(fused, sims):
        sp = s.spectra()
        for k in ("inc", "ext"):
            assert rel_l2(f_spec[k], sp[k]) <= tol, (s.w.name, k)


def test_batch_with_streamed_stores_bitwise(B):
    """A batch whose field traffic exceeds the Infinity Cache runs the
    streaming-store sweep variants for every instance (the small instance
    alone would not); results are unchanged, bit for bit."""
    ws = []
    for q, (n, r) in enumerate(((200, 5.0e-9), (96, 3.0e-9))):
        c = [(n - 1) / 2.0 + 0.3 * q] * 3
        w = W.early_pulse(W.sphere_problem(f"sphere_{n}", n, 0.25e-9, 8, c, r, steps=220))
        w.omega = W.spectrum_omegas(10)
        ws.append(w)
    steps = 220  # the pulse enters the 200^3 TF box after about 160 steps
    print(f"case streamed batch: sizes {[w.nx for w in ws]}", flush=True)
    solo = []
    for w in ws:
        s = B.Sim(w, precision="fp32")
        s.set_tiling(2, 8, 0)
        s.run(steps)
        solo.append(({f: s.field(f) for f in FIELDS}, s.spectra()))
        s.close()
    sims = [B.Sim(w, precision="fp32") for w in ws]
    bt = B.Batch(sims, tiling=(2, 8, 0))
    bt.run(steps)
    bt.synchronize()
    for (fields, spec), s in zip(solo, sims):
        for f in FIELDS:
            assert np.array_equal(s.field(f), fields[f]), (s.w.name, f)
        for k, v in s.spectra().items():
            assert np.array_equal(v, spec[k]), (s.w.name, k)
    assert np.abs(solo[0][0]["Jx"]).max() > 0


@pytest.mark.parametrize("form", [0, 3])
def test_batch_instance_vs_oracle(B, form):
    """Every instance of an FP64 batch (a 128^3 sphere, a 192^3 gap dimer with
    flux boxes, a 104^3 sphere) against the oracle after 320 steps: the
    incident front, which starts with the pulse at t = 0, crosses the last
    metal plane of the largest instance (plane 129) after about 2 (129 + 3) =
    264 steps, so every particle has responded.  All nine fields and the four
    spectra; and in every instance the metal's current reaches a stated
    fraction of eps0 wp e0 (the current a unit field drives at the plasma
    frequency)."""
    ws = instances(count=3, seed=1)
    steps = 320
    print(f"case batch fp64 form {form} vs oracle, {steps} steps: {[w.name for w in ws]}", flush=True)
    sims = [B.Sim(w, precision="fp64") for w in ws]
    bt = B.Batch(sims, form=form)  # the default batch tiling (XCD-aware order, rotated starts)
    bt.run(steps)
    bt.synchronize()
    eps0 = 8.8541878128e-12
    for w, s in zip(ws, sims):  # every instance, the gap dimer included
        print(f"  instance {w.name}", flush=True)
        m = oracle_mask(w)
        top = int(np.nonzero(m.any(axis=(1, 2)))[0].max())
        assert steps >= 2 * (top + 3) + 40, (w.name, top)
        o = orc.OracleSim(oracle_problem(w, threads=8), m)
        o.run(steps)
        ref = {f: o.get(f) for f in FIELDS}
        for f in FIELDS:
            a, b = s.field(f), ref[f]
            # components that are rounding noise on both sides are measured
            # against 1e-3 of the largest component of the same field
            floor = 1e-3 * max(np.linalg.norm(ref[g]) for g in FIELDS if g[0] == f[0])
            e = np.linalg.norm(a - b) / max(np.linalg.norm(b), floor)
            assert e <= 1e-10, (w.name, f, e)
        sg, so = s.spectra(), o.spectra()
        for k in ("inc", "ext", "abs", "sca"):
            assert rel_l2(sg[k], so[k]) <= 1e-10, (w.name, k)
        if w.flux:
            assert np.abs(so["abs"]).max() > 0 and np.abs(so["sca"]).max() > 0, w.name
        jmax = float(np.abs(ref["Jx"][m & 1 != 0]).max())
        print(f"    max|Jx| in the metal {jmax:.3e} A/m^2 = {jmax / (eps0 * w.wp * w.e0):.3f} eps0 wp e0",
              flush=True)
        assert jmax >= 0.05 * eps0 * w.wp * w.e0, w.name
        o.close()


def test_batch_rejects_mixed_precision_and_foreign_steps(B):
    ws = instances(count=2)
    with pytest.raises(B.GnorError):  # no such batch step form
        B.Batch([B.Sim(ws[0], precision="fp32")], form=1)
    a = B.Sim(ws[0], precision="fp32")
    b = B.Sim(ws[1], precision="fp64")
    with pytest.raises(B.GnorError):
        B.Batch([a, b])
    c = B.Sim(ws[1], precision="fp32")
    bt = B.Batch([a, c])
    bt.run(4)
    bt.synchronize()
    a.run(2)  # stepped outside the batch
    with pytest.raises(B.GnorError):
        bt.run(2)


def test_batch_mixes_substrate_and_background_bitwise(B):
    """Instances that differ in their dielectric surroundings (one resting on
    an eps 2.25 half-space whose plane lies just above its particle, one in
    an n = 1.3 background, one in vacuum) batch together and reproduce their
    single runs bit for bit, once the pulse has crossed the substrate plane."""
    ws = instances(count=3, seed=1)
    top = int(np.nonzero(oracle_mask(ws[0]).any(axis=(1, 2)))[0].max())
    ws[0].eps_sub, ws[0].sub_k = 2.25, top + 1
    ws[1].eps_b = 1.69
    steps = 300
    print(f"case mixed batch: sizes {[w.nx for w in ws]}, substrate plane {ws[0].sub_k}", flush=True)
    solo = []
    for w in ws:
        s = B.Sim(w, precision="fp32")
        s.set_tiling(2, 5, 2)
        s.run(steps)
        solo.append(({f: s.field(f) for f in FIELDS}, s.spectra()))
        s.close()
    sims = [B.Sim(w, precision="fp32") for w in ws]
    bt = B.Batch(sims, tiling=(2, 5, 2))
    bt.run(steps)
    bt.synchronize()
    for (fields, spec), s in zip(solo, sims):
        for f in FIELDS:
            assert np.array_equal(s.field(f), fields[f]), (s.w.name, f)
        for k, v in s.spectra().items():
            assert np.array_equal(v, spec[k]), (s.w.name, k)
    assert np.abs(solo[0][0]["Ex"][ws[0].sub_k + 1:]).max() > 0  # the pulse reached the substrate
    assert np.abs(solo[0][0]["Jx"]).max() > 0
