"""Total-field operation on the GPU against the FP64 oracle: a soft plane
source instead of TF/SF and GNOR metal that runs through the absorbing layers,
where it follows the local Drude model (end of Sec. III).

The grid (72 x 41 x 44, two x tiles with a ragged second one, ragged y) holds a
GNOR film across its whole x-y extent, through the x and y layers, and a
block that reaches through the top z layer to the last interior plane.  FP64:
fields, current, the 1D line and the J-route spectra to rel-L2 <= 1e-10; FP32
to the FP32 bars of the other parity tests.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2005_06997_amd import workloads as W
from tests.helpers import oracle_problem, rel_l2

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


def film_workload(beta=W.BETA, diff=W.DIFF, steps=400):
    w = W.Workload(name="film_total_field_72x41x44", nx=72, ny=41, nz=44, dx=0.5e-9, npml=6,
                   total_field=True, source_k=9, flux=False, norm_k=11,
                   omega=W.spectrum_omegas(12), beta=beta, diff=diff, steps=steps)
    w.t0 = 0.3 * w.tau  # the pulse peaks near step 290
    return w


def film_mask(w):
    m = np.zeros((w.nz, w.ny, w.nx), np.uint8)
    m[22:27, 1:w.ny - 1, 1:w.nx - 1] = 7   # film through the x and y layers
    m[37:w.nz - 1, 12:30, 20:50] = 7        # block through the top z layer
    return m


def compare(g, o, ftol, stol):
    worst = {}
    for f in FIELDS:
        a, b = g.field(f), o.get(f)
        assert np.isfinite(a).all(), f
        floor = 1e-3 * max(np.linalg.norm(o.get(h)) for h in FIELDS if h[0] == f[0])
        worst[f] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor))
    worst["line"] = rel_l2(g.aux()[0], o.aux()[0])
    sg, so = g.spectra(), o.spectra()
    for k in ("inc", "ext"):
        worst[k] = rel_l2(sg[k], so[k])
    say("  rel-L2: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    for f in FIELDS:
        assert worst[f] <= ftol, (f, worst[f])
    for k in ("line", "inc", "ext"):
        assert worst[k] <= stol, (k, worst[k])


@pytest.fixture(scope="module")
def oracle_film():
    w = film_workload()
    s = orc.OracleSim(oracle_problem(w, threads=8), film_mask(w))
    s.run(w.steps)
    # the film is driven hard, also inside the layers
    jx = s.get("Jx")
    assert np.abs(jx[22:27, 1:5, 1:5]).max() > 1e-3 * np.abs(jx).max()
    yield s
    s.close()


@pytest.mark.parametrize("prec,mode", [("fp64", 0), ("fp64", 2), ("fp64", 3), ("fp32", 0), ("fp32", 3)])
def test_film_through_the_layers_matches_the_oracle(B, oracle_film, prec, mode):
    w = film_workload()
    say(f"case total-field film {prec} step form {mode}: 72x41x44, {w.steps} steps")
    g = B.Sim(w, precision=prec, mask=film_mask(w))
    g.set_mode(mode)
    g.run(w.steps)
    tol = (1e-10, 1e-10) if prec == "fp64" else (1e-3, 1e-4)
    compare(g, oracle_film, *tol)
    g.close()


def test_gnor_inside_the_layers_is_local_drude_on_the_gpu(B):
    """The GPU's own rule, independently of the oracle: GNOR metal wholly
    inside the layers evolves bit for bit as local Drude metal."""
    w = film_workload(steps=200)
    m = np.zeros((w.nz, w.ny, w.nx), np.uint8)
    m[16:30, 2:w.ny - 2, 1:w.npml] = 7     # inside the low-x layer
    m[w.nz - 5:w.nz - 1, 10:20, 30:40] = 7  # inside the top z layer
    say("case total-field: GNOR in the layers vs local Drude (fp64)")
    out = []
    for beta, diff in ((W.BETA, W.DIFF), (0.0, 0.0)):
        g = B.Sim(film_workload(beta, diff, 200), precision="fp64", mask=m)
        g.run(200)
        out.append({f: g.field(f) for f in FIELDS})
        g.close()
    assert np.abs(out[1]["Jx"]).max() > 0
    for f in FIELDS:
        assert np.array_equal(out[0][f], out[1][f]), f
