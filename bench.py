"""Throughput of the GNOR-FDTD step on one MI355X.

A step is one full leapfrog step of the hot path: H update with CPML and
TF/SF, fused E / free-electron-current update (GNOR) with CPML and TF/SF,
auxiliary incident line, FP64 running transforms of the induced current and
the incident field, and the flux-box transforms.  The workload is a
gold-like sphere of radius 10 nm on a 320^3 grid at dx = 0.1 nm (12-cell
CPML), FP32 fields and currents with FP64 spectral accumulators.

Prints one JSON line:  value = Gcell-updates/s (nx ny nz steps / time) of the
FP32 path over exactly --steps steps, the timed region holding every
flux-box fold those steps owe (see run_gpu); roofline = achieved algorithmic
HBM bytes / s of the dominant kernel (in step form 3 the one-pass launch of
the plain tiles with its TF/SF launch, timed alone; in the two-sweep form the
E/J sweep, its classes timed together) from HIP events on the library's
stream; traffic = its measured HBM bytes per launch from the committed
rocprofv3 counter summary when that summary was taken on the current kernel
sources at the timed tiling (else null); the
FP32 path's spectral errors from fixed-length legs (against the FP64 path,
and against the FP64 oracle on the coarsened copy); cpu_baseline = the FP64
CPU oracle on the host cores (all of the GPU's share, and one) on short
samples of the same grid.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "step_kernels_sphere320_fp32.md")
PROFILE_SUMMARY_FP64 = os.path.join(ROOT, "profiles", "step_kernels_sphere320_fp64.md")


def profiled_tiling(summary=PROFILE_SUMMARY, fp64=False):
    """The sweep tiling (ty, kz, order) of the FP32 (or FP64) leg of the run a
    rocprofv3 summary was taken from (its --tiling / --tiling-fp64 option), or
    None."""
    import re
    try:
        text = open(summary).read()
    except OSError:
        return None
    m = re.search(r"--tiling%s (\d+),(\d+),(\d+)" % ("-fp64" if fp64 else ""), text)
    return tuple(int(v) for v in m.groups()) if m else None


def measured_traffic(kernel, summary=PROFILE_SUMMARY, tiling=None, fp64=False):
    """HBM bytes per sweep of `kernel` (sum over its tile-class launches) from
    a rocprofv3 counter summary, or None if the summary is missing, was taken
    on other kernel sources or (tiling given) at another sweep tiling."""
    try:
        from paper_2005_06997_amd.rocprof_summary import source_hash
        text = open(summary).read()
    except (OSError, ImportError):
        return None
    import re
    m = re.search(r"library source hash \(csrc/\*\): `([0-9a-f]+)`", text)
    if not m or m.group(1) != source_hash():
        return None
    if tiling is not None and profiled_tiling(summary, fp64) != tuple(tiling):
        return None
    m = re.search(r"<!-- traffic " + re.escape(kernel) + r" sweep ([0-9.e+]+) -->", text)
    return float(m.group(1)) if m else None


def algorithmic_bytes(w, mask, word):
    """Per-launch algorithmic bytes of the H and E/J kernels.

    H:   read E (3) + H (3), write H (3) per cell; CPML: psi read + write for
         two H components per (cell, axis) inside an absorbing slab.
    E/J: read H (3) + E^n (3), write E^{n+1} (3) per cell; per metal cell
         E^{n-1} (3), J read (3) and write (3), Phi_P and Phi_J read + write
         (4); CPML as for H.
    """
    N = w.nx * w.ny * w.nz
    nm = int(np.count_nonzero(mask))
    n = (w.nx, w.ny, w.nz)
    cd = sum(2 * w.npml * (N // n[a]) for a in range(3))
    h = word * (9 * N + 4 * cd)
    ej = word * (9 * N + 13 * nm + 4 * cd)
    return h, ej, nm, cd


def dominant(form, word, cells, slab_dirs, ejb, prof, prof_serial):
    """The dominant kernel of a step form: its name, algorithmic bytes per
    launch, average launch time (ms) and kernel family.  Form 3: the one-pass
    launch of the plain tiles (class 0, x-slab tiles included, with its TF/SF
    launch), timed alone (serial classes), at 18 field words per cell and 8
    psi words per (cell, axis) in a slab, the per-unit figures of the step.
    Form 0: the E/J sweep, its classes timed together."""
    if form == 3:
        return ("k_fplain (class 0 in one pass, x-slab tiles included, + k_tfsf_fix, timed alone)",
                word * (18 * cells[0] + 8 * slab_dirs[0]), prof_serial["h_cls"][0], "k_fplain")
    return ("k_ej (E/J sweep = one launch per tile class, timed together)", ejb, prof["ej"], "k_ej")


def time_tiling(sim, tiling, steps=256):
    """Best of two timings (ms per step) of `steps` steps at a tiling; the
    state is reset afterwards."""
    sim.set_tiling(*tiling)
    best = None
    for _ in range(2):
        sim.reset()
        sim.run(32)
        sim.synchronize()
        t0 = time.perf_counter()
        sim.run(steps)
        sim.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        best = ms if best is None else min(best, ms)
    sim.reset()
    return best


def run_gpu(w, precision, steps, warmup, tiling=None, serial=False, forms=(0, 3), prefer=None):
    """Pick the step form (two sweeps, or the plain tiles in one pass) and
    the sweep tiling, warm up, then time `steps` full steps.  The timed
    region holds every flux-box fold its steps owe: the warm-up's staged
    samples are folded before it starts, and it ends with the fold of the
    samples its own steps staged since the last window fold (a partial window
    costs the whole accumulator read-modify-write, so short runs are charged
    more per step than long ones).  prefer: the tiling the committed counters
    were taken at (step form 3); when the autotuner picks another, both are
    timed over 256 steps and `prefer` is kept unless the other is more than
    0.5 % faster (the autotuner's short trials do not separate tilings that
    close)."""
    import torch
    from paper_2005_06997_amd import binding

    sim = binding.Sim(w, precision=precision)
    if serial:
        sim.set_class_streams(False)
    best = None
    for form in forms:
        sim.set_mode(form)
        if tiling is None:
            tl = sim.autotune(trial_steps=10)  # timed search over sweep tilings (state reset after)
            tuned = (tl["ty"], tl["kz"], tl["xcd"])
            if form == 3 and prefer is not None and tuple(prefer) != tuned:
                ms_t, ms_p = time_tiling(sim, tuned), time_tiling(sim, prefer)
                if ms_p <= 1.005 * ms_t:
                    tl = dict(ty=prefer[0], kz=prefer[1], xcd=prefer[2], ms=ms_p, cached=False)
                else:
                    tl = dict(tl, ms=ms_t)
        else:
            sim.set_tiling(*tiling)
            sim.reset()
            sim.run(8)
            sim.synchronize()
            t0 = time.perf_counter()
            sim.run(64)
            sim.synchronize()
            tl = dict(ty=tiling[0], kz=tiling[1], xcd=tiling[2], ms=(time.perf_counter() - t0) / 64 * 1e3,
                      cached=False)
            sim.reset()
        if best is None or tl["ms"] < best[1]["ms"]:
            best = (form, tl)
    sim.set_mode(best[0])
    sim.set_tiling(best[1]["ty"], best[1]["kz"], best[1]["xcd"])
    sim.tiling = best[1]
    sim.form = best[0]
    sim.run(warmup)
    sim.flush_spectra()
    sim.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    sim.flush_spectra()
    sim.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return sim, dt


def spectral_errors(a, b):
    out = {}
    for k in ("inc", "ext", "abs", "sca"):
        den = np.linalg.norm(b[k])
        out[k] = float(np.linalg.norm(a[k] - b[k]) / den) if den > 0 else None
    return out


def error_legs(tiling, form):
    """Spectral errors of the FP32 path from runs of fixed length (independent
    of --steps), in the timed step form: FP32 vs FP64 on the 320^3 workload
    with the pulse moved early (2400 steps: the pulse has crossed the
    particle), and FP32 vs the FP64 oracle's spectra of the 2x-coarsened copy
    over its full 10 000 steps (stored in tests/golden by an oracle-only
    script)."""
    import torch
    from paper_2005_06997_amd import binding
    from paper_2005_06997_amd import workloads as W

    w = W.early_pulse(W.config2())
    spec = {}
    for prec in ("fp32", "fp64"):
        s = binding.Sim(w, precision=prec)
        s.set_mode(form)
        s.set_tiling(*tiling)
        s.run(2400)
        spec[prec] = s.spectra()
        s.close()
        torch.cuda.empty_cache()
    out = {"fp32_vs_fp64_spectra_rel_l2": spectral_errors(spec["fp32"], spec["fp64"]),
           "fp32_vs_fp64_leg": "320^3 sphere, pulse peak at 1.2 tau, 2400 steps"}
    path = os.path.join(ROOT, "tests", "golden", "config2_coarse_oracle_spectra.txt")
    if os.path.exists(path):
        rows = np.array([[float(v) for v in line.split()] for line in open(path)
                         if line.strip() and not line.startswith("#")])
        gold = dict(inc=rows[:, 1], ext=rows[:, 2], abs=rows[:, 3], sca=rows[:, 4])
        wc = W.config2_coarse()
        s = binding.Sim(wc, precision="fp32")
        s.set_mode(form)
        t0 = time.perf_counter()
        s.run(wc.steps)
        sp = s.spectra()
        tc = time.perf_counter() - t0
        s.close()
        torch.cuda.empty_cache()
        out["fp32_vs_oracle_coarse_spectra_rel_l2"] = spectral_errors(sp, gold)
        out["fp32_vs_oracle_leg"] = ("160^3 coarsened copy (dx 0.2 nm, 10 000 steps) vs the FP64 "
                                     f"oracle's spectra; GPU run {tc:.2f} s")
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, steps, threads):
    """The FP64 oracle as it stands on `threads` host threads: Gcell-updates/s
    over `steps` steps of the workload (after one untimed step that touches
    every array)."""
    from oracle import oracle as orc
    from tests.helpers import oracle_mask, oracle_problem

    p = oracle_problem(w, threads=threads)
    s = orc.OracleSim(p, oracle_mask(w))
    s.run(1)
    t0 = time.perf_counter()
    s.run(steps)
    dt = time.perf_counter() - t0
    s.close()
    return w.cells * steps / dt / 1e9, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # defaults: whole 256-step flux windows inside the timed region (one fold
    # of the flux-box transforms per 256 steps, as in a full run)
    ap.add_argument("--steps", type=int, default=2048)
    ap.add_argument("--warmup", type=int, default=256)
    ap.add_argument("--profile-steps", type=int, default=256)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle steps of the all-cores CPU sample (the 1-core sample takes 2)")
    ap.add_argument("--no-error-legs", action="store_true",
                    help="skip the fixed-length FP32 error legs")
    ap.add_argument("--adjoint-steps", type=int, default=6000,
                    help="steps of the design-gradient run (forward + adjoint; 0 = skip)")
    ap.add_argument("--cp-steps", type=int, default=512,
                    help="steps of the same sphere with two critical points (0 = skip)")
    ap.add_argument("--maps-steps", type=int, default=512,
                    help="steps of the same sphere with near-field and density maps (0 = skip)")
    ap.add_argument("--substrate-steps", type=int, default=512,
                    help="steps of the same sphere in an n = 1.3 background on an eps 2.25 substrate "
                         "(0 = skip)")
    ap.add_argument("--star-steps", type=int, default=256,
                    help="steps of the 640^3 star particle (FP32, 100 frequencies, flux boxes; 0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=256,
                    help="steps of the 64-instance batched sweep (0 = skip)")
    ap.add_argument("--tiling", type=str, default=None,
                    help="ty,kz,order: fixed sweep tiling of the FP32 legs instead of the autotuner "
                         "(profiling runs)")
    ap.add_argument("--tiling-fp64", type=str, default=None,
                    help="ty,kz,order: the same for the FP64 leg")
    ap.add_argument("--form", type=int, default=None, choices=(0, 3),
                    help="step form (0 two sweeps, 3 plain tiles in one pass) instead of the "
                         "faster of the two")
    ap.add_argument("--serial-classes", action="store_true",
                    help="tile-class launches one after another (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 2 GiB (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU (there is no multi-GPU sharding); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        a = torch.empty(1 << 31, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 31, "launches": 5}))
        return

    from paper_2005_06997_amd import workloads as W

    w = W.config2("fp32")
    tiling = tuple(int(v) for v in args.tiling.split(",")) if args.tiling else None
    forms = (0, 3) if args.form is None else (args.form,)
    sim, dt = run_gpu(w, "fp32", args.steps, args.warmup, tiling, args.serial_classes, forms,
                      prefer=profiled_tiling())
    value = w.cells * args.steps / dt / 1e9
    ms_step = dt / args.steps * 1e3
    prof = sim.profile(args.profile_steps)  # each sweep timed as it runs (classes concurrent)
    classes = sim.tile_classes()
    cells, slab_dirs = sim.tile_class_cells()
    sim.set_class_streams(False)
    prof_serial = sim.profile(max(2, args.profile_steps // 4))  # per-class breakdown
    sim.set_class_streams(not args.serial_classes)
    form = sim.form
    sim.set_fused(True)
    prof_fused = sim.profile(max(2, args.profile_steps // 4))
    sim.set_mode(form)
    hb, ejb, nmetal, ncd = algorithmic_bytes(w, sim.mask, 4)
    dom, dom_bytes, dom_ms, dom_kernel = dominant(form, 4, cells, slab_dirs, ejb, prof, prof_serial)
    dom_traffic = measured_traffic(dom_kernel, tiling=(sim.tiling["ty"], sim.tiling["kz"], sim.tiling["xcd"]))
    ach = dom_bytes / (dom_ms * 1e-3) / 1e9
    out = {
        "metric": "Gcell-updates/s and % HBM roofline, FP32 vs FP64 GNOR-FDTD at stated error",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sphere_r10nm_320^3_dx0.1nm_gnor_fp32_fields_fp64_spectra",
                   "grid": [w.nx, w.ny, w.nz], "npml": w.npml, "metal_cells": nmetal,
                   "nfreq": int(len(w.omega)), "flux_boxes": bool(w.flux)},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": dom_traffic,
                     "bytes_per_launch": dom_bytes, "avg_launch_ms": round(dom_ms, 5)},
        "step_form": form,
        "class_cells": cells, "class_slab_dirs": slab_dirs,
        "kernels_ms": {k: round(prof[k], 5) for k in ("h", "ej", "dft", "flux_acc")},
        "class_ms_serial": {"h": [round(v, 5) for v in prof_serial["h_cls"]],
                            "ej": [round(v, 5) for v in prof_serial["ej_cls"]]},
        "tile_classes": {"plain": classes[0], "cpml": classes[1], "metal": classes[2],
                         "metal_cpml": classes[3]},
        "tiling": {k: sim.tiling[k] for k in ("ty", "kz", "xcd")},
        # (form 3: "h" is the first phase, one-pass class 0 beside the H sweep of the rest)
        "h_roofline_frac": round(hb / (prof["h"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if form == 0 else None,
        "step_roofline_frac": round((hb + ejb) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "fused_step": {"note": "one-pass H+E/J variant for every class (12 instead of 18 field words "
                               "per cell): slower here, see DESIGN.md",
                       "step_ms": round(prof_fused["step"], 5)},
    }
    del sim
    torch.cuda.empty_cache()
    if not args.no_fp64:
        # the same K steps in FP64 (same warm-up and fold accounting)
        tiling64 = tuple(int(v) for v in args.tiling_fp64.split(",")) if args.tiling_fp64 else tiling
        sim64, dt64 = run_gpu(w, "fp64", args.steps, args.warmup, tiling64, args.serial_classes, forms,
                              prefer=profiled_tiling(PROFILE_SUMMARY_FP64, fp64=True))
        v64 = w.cells * args.steps / dt64 / 1e9
        prof64 = sim64.profile(max(2, args.profile_steps // 2))
        sim64.set_class_streams(False)
        prof64s = sim64.profile(max(2, args.profile_steps // 4))
        sim64.set_class_streams(not args.serial_classes)
        _, ejb64, _, _ = algorithmic_bytes(w, sim64.mask, 8)
        c64, d64 = sim64.tile_class_cells()
        name64, b64, ms64, k64 = dominant(sim64.form, 8, c64, d64, ejb64, prof64, prof64s)
        out["fp64"] = {"value": round(v64, 3), "ms_per_step": round(dt64 / args.steps * 1e3, 5),
                       "step_form": sim64.form, "roofline_kernel": name64,
                       "roofline_frac": round(b64 / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "traffic": measured_traffic(k64, PROFILE_SUMMARY_FP64,
                                                   (sim64.tiling["ty"], sim64.tiling["kz"], sim64.tiling["xcd"]),
                                                   fp64=True),
                       "tiling": {k: sim64.tiling[k] for k in ("ty", "kz", "xcd")},
                       "fp32_speedup": round(value / v64, 3)}
        del sim64
        torch.cuda.empty_cache()
    if not args.no_error_legs:
        tl = out["tiling"]
        out.update(error_legs((tl["ty"], tl["kz"], tl["xcd"]), out["step_form"]))
    if args.cp_steps > 0:
        # bound electrons: the same sphere with two critical points (f3); the
        # E/J sweep adds P_CP and its increment (read + write) per pole and
        # component at the metal points
        wc = W.with_critical_points(w)
        tl = out["tiling"]
        simc, dtc = run_gpu(wc, "fp32", args.cp_steps, args.warmup, (tl["ty"], tl["kz"], tl["xcd"]), forms=(out["step_form"],))
        # (the poles live in the E/J launches of the metal classes; "ej_ms"
        # is the E/J sweep as it runs, in form 3 that of classes 1-3)
        profc = simc.profile(max(2, args.profile_steps))
        out["critical_points"] = {
            "workload": "the same sphere with 2 synthetic critical points, eps_inf 1.1, FP32",
            "poles": len(wc.cp), "steps": args.cp_steps,
            "value": round(wc.cells * args.cp_steps / dtc / 1e9, 3), "unit": "Gcell-updates/s",
            "ms_per_step": round(dtc / args.cp_steps * 1e3, 5), "step_form": simc.form,
            "ej_ms": round(profc["ej"], 5)}
        del simc
        torch.cuda.empty_cache()
    if args.maps_steps > 0:
        # near-field and density maps: 4 frequencies on the xz plane through
        # the sphere, every step (8 FP64 accumulators per point and frequency)
        wm = W.with_maps(w, W.spectrum_omegas(4, 2.5, 4.0), every=1, axis=1)
        tl = out["tiling"]
        simm, dtm = run_gpu(wm, "fp32", args.maps_steps, args.warmup, (tl["ty"], tl["kz"], tl["xcd"]), forms=(out["step_form"],))
        mp = simm.maps()
        out["maps"] = {
            "workload": "the same sphere with maps at 4 frequencies on the 320x320 xz plane, every step",
            "steps": args.maps_steps, "value": round(wm.cells * args.maps_steps / dtm / 1e9, 3),
            "unit": "Gcell-updates/s", "ms_per_step": round(dtm / args.maps_steps * 1e3, 5),
            "overhead_ms_per_step": round(dtm / args.maps_steps * 1e3 - ms_step, 5),
            "peak_density_m3s": float(np.abs(mp["n"]).max())}
        del simm
        torch.cuda.empty_cache()
    if args.substrate_steps > 0:
        # the same sphere in an n = 1.3 background, resting on an eps 2.25
        # half-space that starts right above its top metal plane
        from dataclasses import replace
        ws_ = replace(w, eps_b=1.69, eps_sub=2.25,
                      sub_k=int(round((w.spheres[0, 2] + w.spheres[0, 3]) / w.dx)) + 1)
        tl = out["tiling"]
        sims_, dts = run_gpu(ws_, "fp32", args.substrate_steps, args.warmup, (tl["ty"], tl["kz"], tl["xcd"]), forms=(out["step_form"],))
        out["substrate"] = {
            "workload": "the same sphere in an n = 1.3 background on an eps 2.25 substrate (plane "
                        f"{ws_.sub_k}), FP32",
            "steps": args.substrate_steps,
            "value": round(ws_.cells * args.substrate_steps / dts / 1e9, 3), "unit": "Gcell-updates/s",
            "ms_per_step": round(dts / args.substrate_steps * 1e3, 5)}
        del sims_
        torch.cuda.empty_cache()
    if args.star_steps > 0:
        # the star particle: R = 15 nm sphere with six capped cones, 640^3 at
        # 0.2 nm, 12-cell CPML (at the sphere's step form and tiling)
        wst = W.config3(seed=0)
        tl = out["tiling"]
        simst, dtst = run_gpu(wst, "fp32", args.star_steps, args.warmup, (tl["ty"], tl["kz"], tl["xcd"]),
                              forms=(out["step_form"],))
        out["star"] = {
            "workload": "640^3 star particle (sphere R 15 nm + 6 cones), dx 0.2 nm, 12-cell CPML, "
                        "100 frequencies with flux boxes, FP32",
            "steps": args.star_steps,
            "value": round(wst.cells * args.star_steps / dtst / 1e9, 3), "unit": "Gcell-updates/s",
            "ms_per_step": round(dtst / args.star_steps * 1e3, 5), "step_form": simst.form,
            "tiling": {k: simst.tiling[k] for k in ("ty", "kz", "xcd")}}
        simst.close()
        del simst
        torch.cuda.empty_cache()
    if args.batch_steps > 0:
        from paper_2005_06997_amd import binding
        ws = W.config4(seed=0, count=64)
        sims = [binding.Sim(x, precision="fp32") for x in ws]
        # both step forms of the batch (two sweeps; the tiles without metal
        # in one pass), each warmed up and timed; the faster is reported
        bt = binding.Batch(sims, tiling=(4, 5, 2))
        tforms = {}
        for form in (0, 3):
            bt.set_form(form)
            bt.run(64)
            bt.synchronize()
            t0 = time.perf_counter()
            bt.run(args.batch_steps)
            bt.synchronize()
            tforms[form] = time.perf_counter() - t0
        bform = min(tforms, key=tforms.get)
        tb = tforms[bform]
        bt.close()
        # the same instances stepped one at a time in that form (each with
        # its own graph chunks and the batch's tiling), for comparison
        t_one = 0.0
        for s in sims:
            s.set_mode(bform)
            s.run(64)
            s.synchronize()
            t0 = time.perf_counter()
            s.run(64)
            s.synchronize()
            t_one += (time.perf_counter() - t0) / 64
        bbytes = sum(sum(algorithmic_bytes(s.w, s.mask, 4)[:2]) for s in sims)
        out["batch"] = {"workload": "64 spheres / gap dimers, r 1-8 nm, grids 64^3-200^3, FP32, one "
                                    "launch per tile class and phase over all instances",
                        "value": round(bt.cells * args.batch_steps / tb / 1e9, 3),
                        "unit": "Gcell-updates/s", "cells": bt.cells, "steps": args.batch_steps,
                        "ms_per_step": round(tb / args.batch_steps * 1e3, 4),
                        "step_form": bform,
                        "ms_per_step_by_form": {str(f): round(t / args.batch_steps * 1e3, 4)
                                                for f, t in tforms.items()},
                        "one_at_a_time_ms_per_step": round(t_one * 1e3, 4),
                        "step_roofline_frac": round(bbytes / (tb / args.batch_steps) / 1e9 / HBM_PEAK_GBS,
                                                    4)}
        del sims
        torch.cuda.empty_cache()
    if args.adjoint_steps > 0:
        from paper_2005_06997_amd import binding
        wd = W.config5(0)
        m = int(np.argmin(np.abs(wd.omega - W.ev_to_rad(2.5))))
        sd = binding.Sim(wd, precision="fp32")
        t0 = time.perf_counter()
        obj, grad = sd.gradient(args.adjoint_steps, 500, m)
        ta = time.perf_counter() - t0
        out["adjoint"] = {"workload": "dimer r 5 nm, gap 1 nm, 160^3, 60^3 design region, FP32, "
                                      "objective sigma_ext at 2.5 eV, checkpoints every 500 steps",
                          "steps": args.adjoint_steps, "seconds": round(ta, 3),
                          "gcell_steps_per_s": round(wd.cells * args.adjoint_steps / ta / 1e9, 3),
                          "objective_m2": obj, "grad_norm": float(np.linalg.norm(grad))}
        sd.close()
        torch.cuda.empty_cache()
    if not args.no_cpu:
        # all host threads of the GPU's share (at most 16), then one core
        cores = min(16, os.cpu_count() or 1)
        v, secs = cpu_baseline(w, args.cpu_steps, cores)
        v1, secs1 = cpu_baseline(w, 2, 1)
        out["cpu_baseline"] = {"value": round(v, 5), "unit": "Gcell-updates/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{args.cpu_steps} FP64 oracle steps of the same 320^3 problem "
                                         f"on {cores} threads ({secs:.1f} s)",
                               "one_core": {"value": round(v1, 6), "unit": "Gcell-updates/s",
                                            "sample": f"2 steps on 1 thread ({secs1:.1f} s)"},
                               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
