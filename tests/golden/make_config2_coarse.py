"""Write the FP64 oracle's spectra of the 2x-coarsened sphere workload.

The 320^3 sphere workload (r = 10 nm, dx = 0.1 nm, 20 000 steps) is too large
for the CPU oracle.  Its coarsened copy -- the same particle on a 160^3 grid at
dx = 0.2 nm with an 8-cell CPML, run for 10 000 steps (the same physical
time) -- is not: this script runs it through the oracle alone and writes
inc, ext, abs and sca at the 100 monitor frequencies (1 .. 6 eV) to
``config2_coarse_oracle_spectra.txt`` beside it.  The GPU test of the FP32
path on the same copy compares against that file.

Only ``oracle/`` computes here; the workload module supplies the seeded
problem parameters (no FDTD arithmetic).  Run from the repository root:

    python tests/golden/make_config2_coarse.py [threads]

It takes about 45 minutes on 8 host threads.
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "config2_coarse_oracle_spectra.txt")


def main():
    import numpy as np

    from oracle import oracle as orc
    from paper_2005_06997_amd import workloads as W
    from tests.helpers import oracle_mask, oracle_problem

    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    w = W.config2_coarse("fp64")
    s = orc.OracleSim(oracle_problem(w, threads=threads), oracle_mask(w))
    t0 = time.time()
    done = 0
    while done < w.steps:
        n = min(500, w.steps - done)
        s.run(n)
        done += n
        print(f"{done} / {w.steps} steps, {time.time() - t0:.0f} s", flush=True)
    sp = s.spectra()
    s.close()
    with open(OUT + ".tmp", "w") as fh:
        fh.write("# FP64 oracle spectra of the coarsened sphere workload: a gold-like\n"
                 "# Drude sphere (wp 1.37e16 rad/s, gamma 1.06e14 rad/s, beta 1e6 m/s,\n"
                 "# D 1.9e-4 m^2/s) of radius 10 nm centred in a 160^3 grid at dx = 0.2 nm,\n"
                 "# 8-cell CPML, Courant 0.5, TF/SF modulated-Gaussian pulse (1-6 eV),\n"
                 f"# {w.steps} steps; flux boxes on.  Written by make_config2_coarse.py\n"
                 "# (oracle only).  Columns: omega [rad/s], inc [(V s/m)^2], ext, abs,\n"
                 "# sca [m^2].\n")
        for m in range(len(w.omega)):
            row = (w.omega[m], sp["inc"][m], sp["ext"][m], sp["abs"][m], sp["sca"][m])
            fh.write(" ".join(repr(float(v)) for v in row) + "\n")
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")
    assert np.all(np.isfinite(sp["ext"]))


if __name__ == "__main__":
    main()
