"""Dielectric substrate on the HIP path, through the C-ABI, against the FP64
oracle: a GNOR sphere resting on a glass-like half-space (eps 2.25) whose
interface crosses the TF box and both monitor boxes.  FP64 fields and spectra
<= 1e-10 rel-L2; FP32 <= 1e-3 on fields, 1e-4 on spectra.  The fused and
hybrid step forms, metal beyond the substrate plane and design gradients are
refused."""
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


def on_substrate(seed):
    """config 1 with the substrate plane right above the top metal plane (the
    pulse travels +z: the light meets the particle, then the substrate)."""
    w = W.early_pulse(W.config1(seed))
    top = int(np.nonzero(oracle_mask(w).any(axis=(1, 2)))[0].max())
    w.eps_sub, w.sub_k = 2.25, top + 1
    assert w.tf_lo[2] < w.sub_k < w.tf_hi[2] and w.sca_lo[2] < w.sub_k < w.sca_hi[2]
    w.omega = W.spectrum_omegas(24)
    return w


def compare(g, o, ftol, stol):
    pairs = {f: (g.field(f), o.get(f)) for f in FIELDS}
    worst = {}
    for f, (a, b) in pairs.items():
        kin = max(np.linalg.norm(pairs[h][1]) for h in FIELDS if h[0] == f[0])
        worst[f] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-3 * kin))
    sg, so = g.spectra(), o.spectra()
    for k in ("inc", "ext", "abs", "sca"):
        worst[k] = rel_l2(sg[k], so[k])
    say("  rel-L2: " + ", ".join(f"{k} {v:.1e}" for k, v in worst.items()))
    for f in FIELDS:
        assert worst[f] <= ftol, (f, worst[f])
    for k in ("inc", "ext", "abs", "sca"):
        assert worst[k] <= stol, (k, worst[k])


@pytest.mark.parametrize("prec,seed,mode", [("fp64", 0, 0), ("fp64", 3, 0), ("fp32", 1, 0),
                                            ("fp64", 0, 3)])
def test_sphere_on_substrate_vs_oracle(B, prec, seed, mode):
    """Step form 3 (plain tiles in one pass) takes the substrate's per-plane
    coefficients in its own kernel."""
    w = on_substrate(seed)
    say(f"case {prec} sphere on substrate, seed {seed}, plane {w.sub_k}, step form {mode}")
    g = B.Sim(w, precision=prec)
    g.set_mode(mode)
    g.run(w.steps)
    o = orc.OracleSim(oracle_problem(w, threads=8), oracle_mask(w))
    o.run(w.steps)
    assert np.abs(o.get("Jx")).max() > 0
    tol = (1e-10, 1e-10) if prec == "fp64" else (1e-3, 1e-4)
    compare(g, o, *tol)


def test_substrate_refusals(B):
    w = on_substrate(0)
    g = B.Sim(w, precision="fp32")
    for mode in (1, 2):
        with pytest.raises(B.GnorError):
            g.set_mode(mode)
    g.run(4)
    assert g.check_finite()
    w.sub_k -= 2  # the top metal planes now lie beyond the substrate plane
    with pytest.raises(B.GnorError):
        B.Sim(w, precision="fp32")
