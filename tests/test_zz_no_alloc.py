"""gnor_batch_create_static (the allocation-free batch, tables in the
library's static device buffer) against gnor_batch_create (tables in a
caller buffer), through the C-ABI: two static batches in a row, the second
with fewer instances, each equal bit for bit to the caller-table batch of the
same instances; the first static batch is refused once the second has taken
the buffer over, and a static batch beyond the buffer's capacity is
refused."""
import ctypes as C

import numpy as np
import pytest

from paper_2005_06997_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz")


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_06997_amd import binding
    return binding


def instances(count):
    ws = [W.early_pulse(w) for w in W.config4(seed=2, count=count)]
    for q, w in enumerate(ws):
        w.omega = W.spectrum_omegas(8 + 4 * q)
        w.flux = q % 2 == 0
    return ws


def sims_for(B, ws):
    out = []
    for w in ws:
        s = B.Sim(w, precision="fp32")
        s.set_tiling(2, 5, 2)
        out.append(s)
    return out


def results(sims):
    return [({f: s.field(f) for f in FIELDS}, s.spectra()) for s in sims]


def reference(B, ws, steps):
    sims = sims_for(B, ws)
    bt = B.Batch(sims, tiling=(2, 5, 2))
    bt.run(steps)
    bt.synchronize()
    out = results(sims)
    bt.close()
    return out


def static_batch(B, sims):
    import torch
    L = B.load()
    arr = (C.c_void_p * len(sims))(*[s.h.value for s in sims])
    stream = torch.cuda.Stream(device=sims[0].device)
    h = C.c_void_p()
    st = L.gnor_batch_create_static(len(sims), arr, C.c_void_p(stream.cuda_stream), C.byref(h))
    assert st == 0, st
    return h, stream


def run_static(B, h, nsteps):
    L = B.load()
    st = L.gnor_batch_run(h, int(nsteps))
    if st == 0:
        st = L.gnor_batch_synchronize(h)
    return st


def test_static_batch_equals_caller_table_batch_twice(B):
    steps = 150
    first, second = instances(5), instances(3)
    print(f"case static batch: {[w.nx for w in first]} then {[w.nx for w in second]}, {steps} steps",
          flush=True)
    want1 = reference(B, first, steps)
    want2 = reference(B, second, steps)
    L = B.load()
    sims1 = sims_for(B, first)
    h1, st1 = static_batch(B, sims1)
    assert run_static(B, h1, steps) == 0
    got1 = results(sims1)
    sims2 = sims_for(B, second)
    h2, st2 = static_batch(B, sims2)
    assert run_static(B, h2, steps) == 0
    got2 = results(sims2)
    for want, got, ws in ((want1, got1, first), (want2, got2, second)):
        for (wf, wsp), (gf, gsp), w in zip(want, got, ws):
            for f in FIELDS:
                assert np.array_equal(gf[f], wf[f]), (w.name, f)
            for k in wsp:
                assert np.array_equal(gsp[k], wsp[k]), (w.name, k)
        assert np.abs(got[0][0]["Jx"]).max() > 0
    # the first static batch no longer owns the buffer
    assert run_static(B, h1, 2) == 5
    L.gnor_batch_destroy(h1)
    assert run_static(B, h2, 2) == 0
    L.gnor_batch_destroy(h2)


def test_static_batch_refuses_more_than_its_capacity(B):
    L = B.load()
    w = instances(1)[0]
    s = B.Sim(w, precision="fp32")
    arr = (C.c_void_p * 129)(*([s.h.value] * 129))
    h = C.c_void_p()
    assert L.gnor_batch_create_static(129, arr, C.c_void_p(s.stream.cuda_stream), C.byref(h)) == 6
    assert L.gnor_batch_create_static(1, arr, None, C.byref(h)) == 1
