"""Write the FP64 oracle's exact directional derivatives of the design
objective on the 48^3 copy of the adjoint workload.

The adjoint workload is a gold-like dimer on a 160^3 grid at dx = 0.25 nm with
a 60^3 design region and the objective sigma_ext at 2.5 eV after 6000 steps.
Its 48^3 copy (same dx, geometry scaled by 0.3, an 18^3 design region, 6000
steps) fits the CPU oracle.  For three seeded directions v in design space
this script runs the oracle on dual numbers (forward-mode differentiation
through every step of the literal P-form update) and writes the objective and
its exact derivative along v to ``config5_small_oracle_directional.txt``
beside it.  The GPU test projects the library's adjoint gradient onto the
same directions.

Only ``oracle/`` computes here; the workload module supplies the seeded
problem parameters and directions (no FDTD arithmetic).  Run from the
repository root:

    python tests/golden/make_config5_small.py [threads]
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "config5_small_oracle_directional.txt")
SEEDS = (101, 102, 103)
M_TARGET = 4  # 2.5 eV in spectrum_omegas(9, 2.0, 3.0)


def workload():
    from paper_2005_06997_amd import workloads as W
    w = W.config5_small(0)
    w.omega = W.spectrum_omegas(9, 2.0, 3.0)
    return w


def main():
    import numpy as np

    from oracle import oracle as orc
    from paper_2005_06997_amd import workloads as W
    from tests.helpers import oracle_mask_and_weight, oracle_problem

    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    w = workload()
    assert abs(w.omega[M_TARGET] - W.ev_to_rad(2.5)) < 1e-6 * w.omega[M_TARGET]
    mask, weight = oracle_mask_and_weight(w)
    p = oracle_problem(w, threads=threads)
    (x0, y0, z0), (x1, y1, z1) = w.design_lo, w.design_hi
    rows = []
    t0 = time.time()
    for seed in SEEDS:
        v = W.design_direction(np.asarray(w.rho).shape, seed)
        vfull = np.zeros_like(weight)
        vfull[z0:z1, y0:y1, x0:x1] = v
        val, der = orc.directional(p, mask, weight, vfull, w.steps, M_TARGET)
        rows.append((seed, val, der))
        print(f"seed {seed}: L {val!r} dL/dt {der!r} ({time.time() - t0:.0f} s)", flush=True)
    with open(OUT + ".tmp", "w") as fh:
        fh.write("# FP64 oracle, 48^3 copy of the adjoint workload: gold-like dimer (r 1.5 nm,\n"
                 "# gap 0.3 nm) at dx = 0.25 nm, 4-cell CPML, 18^3 design region of seeded\n"
                 f"# densities, {w.steps} steps, objective sigma_ext at 2.5 eV (frequency index\n"
                 f"# {M_TARGET} of 9 between 2 and 3 eV).  Exact derivative along seeded\n"
                 "# directions v (workloads.design_direction) by dual numbers.  Written by\n"
                 "# make_config5_small.py (oracle only).\n"
                 "# Columns: direction seed, objective [m^2], derivative along v [m^2].\n")
        for seed, val, der in rows:
            fh.write(f"{seed} {float(val)!r} {float(der)!r}\n")
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
