"""The method's degenerate limits and the interface's largest sizes on the HIP
path, through the C-ABI, against the FP64 oracle (FP64, rel-L2 <= 1e-10).

* beta = D = 0, the local Drude model (eta = 0: no pressure or diffusion
  force), and D = 0, the nonlocal Drude model (eta = beta^2, no Phi_J
  history), Sec. II.
* The largest counts at once: four critical points (Eq. CritPoint, the
  most a material takes) and eight map frequencies (the most a map takes),
  with 256 spectral frequencies and both flux boxes (the spectra have no
  fixed limit); a ninth map frequency is refused.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_mask, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

BASE = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz")
FOUR_POLES = W.CP_SYNTH + ((0.3, 3.0e15, 4.0e14, 0.5), (0.2, 7.0e15, 1.2e15, -0.4))


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_06997_amd import binding
    return binding


def worst_fields(g, o, names):
    """rel-L2 per field; a component that is rounding noise is measured
    against 1e-3 of the largest component of the same field."""
    pairs = {f: (g.field(f), o.get(f)) for f in names}
    out = {}
    for f, (a, b) in pairs.items():
        kin = max(np.linalg.norm(pairs[h][1]) for h in pairs if h[:-1] == f[:-1])
        out[f] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-3 * kin))
    return out


@pytest.mark.parametrize("beta,diff", [(0.0, 0.0), (W.BETA, 0.0)])
def test_local_and_nonlocal_drude_limits_vs_oracle(B, beta, diff):
    w = W.early_pulse(W.config1(4))
    w.beta, w.diff = beta, diff
    w.omega = W.spectrum_omegas(20)
    say(f"case fp64 beta {beta:g} D {diff:g}")
    g = B.Sim(w, precision="fp64")
    g.run(w.steps)
    o = orc.OracleSim(oracle_problem(w, threads=8), oracle_mask(w))
    o.run(w.steps)
    worst = worst_fields(g, o, BASE)
    sg, so = g.spectra(), o.spectra()
    for k in ("inc", "ext", "abs", "sca"):
        worst[k] = rel_l2(sg[k], so[k])
    say("  rel-L2: " + ", ".join(f"{k} {v:.1e}" for k, v in worst.items()))
    assert np.abs(o.get("Jx")).max() > 0
    for k, v in worst.items():
        assert v <= 1e-10, (k, v)


def test_largest_sizes_vs_oracle(B):
    w = W.with_maps(W.with_critical_points(W.early_pulse(W.config1(2)), poles=FOUR_POLES),
                    W.spectrum_omegas(8, 2.0, 5.0))
    w.omega = W.spectrum_omegas(256)
    w.flux = True
    assert len(w.cp) == 4
    say("case fp64: 256 frequencies with flux boxes, 4 critical points, 8 map frequencies")
    g = B.Sim(w, precision="fp64")
    g.run(w.steps)
    o = orc.OracleSim(oracle_problem(w, threads=8), oracle_mask(w))
    o.run(w.steps)
    names = BASE + tuple(f"PC{p}{c}" for p in range(4) for c in "xyz")
    worst = worst_fields(g, o, names)
    sg, so = g.spectra(), o.spectra()
    for k in ("inc", "ext", "abs", "sca"):
        assert len(sg[k]) == 256
        worst[k] = rel_l2(sg[k], so[k])
    gm, om = g.maps(), o.maps()
    scale = max(np.linalg.norm(om[q]) for q in ("Ex", "Ey", "Ez"))
    for k in ("Ex", "Ey", "Ez", "n", "inc"):
        den = scale if k.startswith("E") else np.linalg.norm(om[k])
        worst["map " + k] = float(np.linalg.norm(gm[k] - om[k]) / den)
    say("  rel-L2: " + ", ".join(f"{k} {v:.1e}" for k, v in worst.items()))
    assert np.abs(o.get("PC3x")).max() > 0
    for k, v in worst.items():
        assert v <= 1e-10, (k, v)


def test_ninth_map_frequency_is_refused(B):
    """gnor_set_maps takes at most 8 frequencies (a fifth critical point is
    refused by gnor_set_material, checked on the CPU with the ABI tests)."""
    base = W.early_pulse(W.config1(0))
    with pytest.raises(B.GnorError):
        B.Sim(W.with_maps(base, W.spectrum_omegas(9, 2.0, 5.0)), precision="fp32")


def test_profile_refuses_more_than_4096_steps(B):
    """gnor_profile_kernels takes at most 4096 steps (one set of events per
    step); the simulation stays usable after the refusal."""
    w = W.early_pulse(W.config1(0))
    g = B.Sim(w, precision="fp32")
    with pytest.raises(B.GnorError):
        g.profile(4097)
    assert g.step == 0
    pr = g.profile(8)
    assert pr["h"] > 0 and pr["ej"] > 0 and g.step == 8
    g.run(16)
    assert g.check_finite()
