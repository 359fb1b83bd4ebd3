"""A short run of one workload, for a profiler to wrap (rocprofv3 kernel
traces and counters of a workload other than bench.py's main one).

    python -m paper_2005_06997_amd.profile_run star [--steps 64] [--form 3] [--tiling ty,kz,order]
    python -m paper_2005_06997_amd.profile_run adjoint [--steps 1000]
    python -m paper_2005_06997_amd.profile_run batch [--steps 64] [--form 3]

star:    the 640^3 star particle (FP32, 100 frequencies, flux boxes): step
         form and tiling autotuned unless given, then --steps steps with the
         tile classes launched one after another (so that a kernel trace times
         each launch alone), the spectra folded at the end.
adjoint: the 160^3 dimer design problem (FP32, 60^3 design region): the
         objective and its adjoint gradient over --steps steps, checkpoints
         every 500.
batch:   the 64 instances of the batched workload (spheres and gap dimers,
         grids 64^3-200^3, FP32, tiling (4, 5, 2)) in step form --form
         (default 3): 64 warm-up steps, then --steps steps.
Prints one JSON line with the wall time.
"""
from __future__ import annotations

import argparse
import json
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=("star", "adjoint", "batch"))
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--form", type=int, default=None, choices=(0, 3))
    ap.add_argument("--tiling", type=str, default=None)
    args = ap.parse_args(argv)

    import torch
    from paper_2005_06997_amd import binding
    from paper_2005_06997_amd import workloads as W

    if args.workload == "star":
        w = W.config3(seed=0)
        s = binding.Sim(w, precision="fp32")
        best = None
        for form in ((0, 3) if args.form is None else (args.form,)):
            s.set_mode(form)
            if args.tiling:
                ty, kz, xcd = (int(v) for v in args.tiling.split(","))
                s.set_tiling(ty, kz, xcd)
                tl = dict(ty=ty, kz=kz, xcd=xcd, ms=0.0)
            else:
                tl = s.autotune(trial_steps=10)
            if best is None or tl["ms"] < best[1]["ms"]:
                best = (form, tl)
        s.set_mode(best[0])
        s.set_tiling(best[1]["ty"], best[1]["kz"], best[1]["xcd"])
        s.set_class_streams(False)
        s.run(8)
        s.synchronize()
        t0 = time.perf_counter()
        s.run(args.steps)
        s.flush_spectra()
        s.synchronize()
        dt = time.perf_counter() - t0
        out = dict(workload="640^3 star, FP32", steps=args.steps, form=best[0],
                   tiling=[best[1]["ty"], best[1]["kz"], best[1]["xcd"]], seconds=round(dt, 4),
                   ms_per_step=round(dt / args.steps * 1e3, 4),
                   gcell_per_s=round(w.cells * args.steps / dt / 1e9, 3))
    elif args.workload == "batch":
        form = 3 if args.form is None else args.form
        sims = [binding.Sim(x, precision="fp32") for x in W.config4(seed=0, count=64)]
        bt = binding.Batch(sims, tiling=(4, 5, 2), form=form)
        bt.run(64)
        bt.synchronize()
        t0 = time.perf_counter()
        bt.run(args.steps)
        bt.synchronize()
        dt = time.perf_counter() - t0
        out = dict(workload="64-instance batch, FP32", steps=args.steps, form=form, seconds=round(dt, 4),
                   ms_per_step=round(dt / args.steps * 1e3, 4),
                   gcell_per_s=round(bt.cells * args.steps / dt / 1e9, 3))
        bt.close()
    else:
        import numpy as np
        w = W.config5(seed=0)
        s = binding.Sim(w, precision="fp32")
        m = int(np.argmin(np.abs(w.omega - W.ev_to_rad(2.5))))  # the objective at 2.5 eV
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obj, grad = s.gradient(args.steps, 500, m)
        dt = time.perf_counter() - t0
        out = dict(workload="160^3 dimer design problem, FP32", steps=args.steps, seconds=round(dt, 4),
                   gcell_steps_per_s=round(w.cells * args.steps / dt / 1e9, 3), objective=obj,
                   grad_norm=float(np.linalg.norm(grad)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
