"""Summarise rocprofv3 CSV output of a bench.py run into a short Markdown
report: average duration per kernel (kernel trace) and HBM bytes per dispatch
(FETCH_SIZE and WRITE_SIZE counter runs), the latter scaled by what the same
counters read for a plain device copy of known size.

usage: python -m paper_2005_06997_amd.rocprof_summary [--only=K1,K2,...] TRACE_DIR FETCH_DIR
           WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR COPY_BYTES OUT.md "command 1" ["command 2" ...]

--only keeps the kernels whose name (template arguments dropped) is listed,
e.g. the batched kernels of a run that also steps single simulations.
--type=T keeps the kernels whose first template argument is T (float or
double), e.g. the FP64 sweeps of a run that also steps in FP32.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# kernel families launched once per tile class, the classes of one sweep
# back to back (or concurrently)
SWEEPS = ("k_h", "k_ej", "k_step", "k_fplain", "k_fplain_pml", "k_fplain_metal", "k_h_batch", "k_ej_batch",
          "k_fplain_batch")
# kernels launched with a sweep (inside its fork/join, or just before or
# after its launch on the same stream), counted with that sweep: the sweeps
# each may belong to, the first when the launch before it is none of them
MEMBER_OF = {"k_aux_e_batch": ("k_ej_batch",),
             "k_tfsf_fix": ("k_fplain", "k_fplain_pml", "k_fplain_metal"),
             "k_nodes": ("k_fplain_metal",),
             "k_tfsf_fix_batch": ("k_fplain_batch",),
             "k_nodes_batch": ("k_fplain_batch",)}
# sweeps that run beside another family's launches in one phase of a step:
# such a launch joins that family when the launch before it is one of them
# (the batched H sweep of the metal tiles next to the batched one-pass
# launches), and is a sweep of its own otherwise (the two-sweep form)
BESIDE = {"k_h_batch": ("k_fplain_batch",)}


def family(kernel: str, prev=None) -> str:
    """The sweep family of a launch; prev: the family of the launch before it
    (a member kernel joins it when it may)."""
    base = kernel.split("<")[0]
    if base in BESIDE:
        return prev if prev in BESIDE[base] else base
    parents = MEMBER_OF.get(base)
    if not parents:
        return base
    return prev if prev in parents else parents[0]


def of_type(kernel: str, typ) -> bool:
    """True when typ is None or the kernel's first template argument is typ."""
    if typ is None:
        return True
    if "<" not in kernel:
        return False
    return kernel.split("<", 1)[1].split(",")[0].rstrip(">").strip() == typ


def _csv(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return list(csv.DictReader(open(files[0])))


def short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "")
    n = n.split("(")[0]
    for pre in ("void ", "gnor::"):
        n = n.replace(pre, "")
    return n.strip()


def counters(d):
    out = defaultdict(list)
    for r in _csv(d, "counter_collection.csv"):
        out[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return out


def sweep_spans(trace_dir, typ=None, joined=None):
    """Per sweep family (SWEEPS): number of sweeps and the mean span
    (us) from the first start to the last end of each run of that family's
    class launches, with the dispatches of the whole run in start order.
    joined (a dict, filled if given): member kernel -> the sweeps it joined."""
    rows = _csv(trace_dir, "kernel_trace.csv")
    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(r["Kernel_Name"]))
                for r in rows if of_type(short(r["Kernel_Name"]), typ))
    out = defaultdict(list)
    cur, lo, hi = None, 0, 0
    for st, en, name in ev + [(0, 0, None)]:
        base = None if name is None else family(name, cur)
        if joined is not None and name is not None and (name.split("<")[0] in MEMBER_OF or
                                                         name.split("<")[0] in BESIDE):
            joined.setdefault(name.split("<")[0], set()).add(base)
        if base != cur:
            if cur in SWEEPS:
                out[cur].append((hi - lo) / 1e3)
            cur, lo, hi = base, st, en
        else:
            hi = max(hi, en)
    return {k: (len(v), sum(v) / len(v)) for k, v in out.items()}


def source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def main(argv):
    only, typ = None, None
    while argv and argv[0].startswith("--"):
        opt, _, val = argv[0].partition("=")
        if opt == "--only":
            only = set(val.split(","))
        elif opt == "--type":
            typ = val
        else:
            raise SystemExit(f"unknown option {argv[0]}")
        argv = argv[1:]
    trace, fetch, write, cfetch, cwrite, copy_bytes, out = argv[:7]
    cmds = argv[7:]
    copy_bytes = float(copy_bytes)
    stats = _csv(trace, "kernel_stats.csv")
    if only is not None:
        stats = [r for r in stats if short(r["Name"]).split("<")[0] in only]
    stats = [r for r in stats if of_type(short(r["Name"]), typ)]
    f, w = counters(fetch), counters(write)
    cf, cw = counters(cfetch), counters(cwrite)
    ckey = max(cf, key=lambda k: sum(cf[k]))
    f_scale = copy_bytes / (sum(cf[ckey]) / len(cf[ckey]) * 1024.0)
    w_scale = copy_bytes / (sum(cw[ckey]) / len(cw[ckey]) * 1024.0)
    title = "GNOR-FDTD step kernels" if only is None else "GNOR-FDTD kernels " + ", ".join(sorted(only))
    if typ is not None:
        title += f" ({typ})"
    lines = ["# rocprofv3 summary: " + title, "",
             f"library source hash (csrc/*): `{source_hash()}`", "", "Commands (repository root):", ""]
    lines += [f"    {c}" for c in cmds]
    lines += ["", f"Copy calibration ({copy_bytes / 2**30:.0f} GiB device copy): FETCH_SIZE scale "
                  f"{f_scale:.4f}, WRITE_SIZE scale {w_scale:.4f} (true bytes / counter bytes).", "",
              "| kernel | calls | avg us | FETCH MB/dispatch (scaled) | WRITE MB/dispatch (scaled) |"
              " HBM GB/s |", "|---|---|---|---|---|---|"]
    fam = defaultdict(lambda: [0.0, 0.0, 0.0])  # sweep: avg us, fetch MB, write MB (sum of classes)
    joined = {}
    spans = sweep_spans(trace, typ, joined)
    for r in stats[:16]:
        k = short(r["Name"])
        avg = float(r["AverageNs"])
        fm = sum(f[k]) / len(f[k]) * 1024 * f_scale / 1e6 if k in f else float("nan")
        wm = sum(w[k]) / len(w[k]) * 1024 * w_scale / 1e6 if k in w else float("nan")
        bw = (fm + wm) * 1e6 / (avg * 1e-9) / 1e9 if avg > 0 else float("nan")
        lines.append(f"| {k} | {r['Calls']} | {avg / 1e3:.1f} | {fm:.1f} | {wm:.1f} | {bw:.0f} |")
        # a member kernel counts once with each of its sweeps in the summary
        bases = sorted(joined.get(k.split("<")[0], ())) or [family(k)]
        for base in bases:
            if base in SWEEPS:
                e = fam[base]
                e[0] += avg / 1e3
                e[1] += fm
                e[2] += wm
    lines += ["", "Sweeps (one launch per tile class, the classes of a sweep running concurrently).",
              "Span = first start to last end of a sweep's class launches, averaged over the sweeps;",
              "bytes = per-dispatch counters summed over the classes (each runs once per sweep)",
              "and over the kernels launched inside the sweep (" +
              ", ".join(f"{k} in {' or '.join(v)}" for k, v in MEMBER_OF.items()) + "; " +
              ", ".join(f"{k} in {' or '.join(v)} when it starts inside it" for k, v in BESIDE.items()) +
              "):", "",
              "| sweep | sweeps | avg span us | FETCH MB | WRITE MB | HBM GB/s over the span |",
              "|---|---|---|---|---|---|"]
    for base, (us, fm, wm) in sorted(fam.items()):
        n, span = spans.get(base, (0, float("nan")))
        lines.append(f"| {base} | {n} | {span:.1f} | {fm:.1f} | {wm:.1f} | "
                     f"{(fm + wm) * 1e6 / (span * 1e-6) / 1e9:.0f} |")
        lines.append(f"<!-- traffic {base} sweep {(fm + wm) * 1e6:.0f} -->")
        lines.append(f"<!-- time {base} sweep {span:.2f} -->")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main(sys.argv[1:])
