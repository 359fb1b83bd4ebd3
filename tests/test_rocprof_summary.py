"""Host logic of the rocprofv3 summary (CPU only): sweep spans over concurrent
class launches, kernels counted with the sweep they run inside, the
element-type filter, and the counter scaling by a copy of known size.  The
inputs are small CSV files in rocprofv3's column layout with values chosen
so that every expected figure is worked out by hand below."""
import csv
import os

from paper_2005_06997_amd import rocprof_summary as R


def write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def trace(d, events):
    write_csv(os.path.join(d, "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
              events)


def counters(d, rows):
    write_csv(os.path.join(d, "run_counter_collection.csv"), ["Kernel_Name", "Counter_Value"], rows)


def test_family_and_type_filter():
    assert R.family("k_aux_e_batch<float>") == "k_ej_batch"
    assert R.family("k_h<float, 2, 0, true>") == "k_h"
    # the TF/SF launch joins the one-pass sweep launched before it; the node
    # scalars open the metal class's
    assert R.family("k_tfsf_fix<float>", "k_fplain_metal") == "k_fplain_metal"
    assert R.family("k_tfsf_fix<float>", "k_fplain") == "k_fplain"
    assert R.family("k_tfsf_fix<float>", "k_h") == "k_fplain"
    assert R.family("k_nodes<float>", "k_fplain_pml") == "k_fplain_metal"
    assert R.of_type("k_h<double, 2, 0, true>", "double")
    assert not R.of_type("k_h<float, 2, 0, true>", "double")
    assert R.of_type("k_dft<double>", "double")
    assert not R.of_type("k_flux_acc", "double")
    assert R.of_type("k_flux_acc", None)


def test_sweep_spans_group_concurrent_classes(tmp_path):
    """Two batched H sweeps (classes overlapping in time), each followed by a
    batched E/J sweep whose line kernel starts between its class launches;
    an FP64 launch in between is dropped by the type filter.  Spans: H
    (0..300) and (1000..1250) -> mean 275 ns = 0.275 us; E/J (400..900) and
    (1300..1700) -> 0.45 us, the line kernel counted inside its sweep."""
    d = str(tmp_path / "t")
    ns = "void gnor::(anonymous namespace)::"
    ev = [
        (ns + "k_h_batch<float, 2, 0, true>(...)", 0, 200),
        (ns + "k_h_batch<float, 2, 1, true>(...)", 50, 300),
        (ns + "k_ej_batch<float, 2, 0, false, true>(...)", 400, 800),
        (ns + "k_aux_e_batch<float>(...)", 410, 500),
        (ns + "k_ej_batch<float, 2, 1, false, true>(...)", 420, 900),
        (ns + "k_h<double, 2, 0, true>(...)", 950, 990),
        (ns + "k_h_batch<float, 2, 0, true>(...)", 1000, 1250),
        (ns + "k_ej_batch<float, 2, 0, false, true>(...)", 1300, 1700),
    ]
    trace(d, ev)
    spans = R.sweep_spans(d, "float")
    assert spans["k_h_batch"][0] == 2 and abs(spans["k_h_batch"][1] - 0.275) < 1e-12
    assert spans["k_ej_batch"][0] == 2 and abs(spans["k_ej_batch"][1] - 0.45) < 1e-12
    assert "k_aux_e_batch" not in spans and "k_h" not in spans
    no_filter = R.sweep_spans(d)
    assert no_filter["k_h"][0] == 1  # the FP64 launch forms a sweep of its own


def test_batched_metal_h_sweep_joins_the_one_pass_phase(tmp_path):
    """Form 3 of a batch: the one-pass launches of classes 0-2 (with the node
    scalars before class 2) and the H sweep of the metal tiles beside them,
    then the TF/SF launch, then the metal E/J sweep.  Two steps: each phase
    is one sweep (0..700 and 1000..1700, the TF/SF launch included: 0.7 us),
    the H launch counted inside it; on its own (no one-pass launch before
    it) the H launch is a sweep of its own."""
    assert R.family("k_h_batch<float, 4, 3, true>", "k_fplain_batch") == "k_fplain_batch"
    assert R.family("k_h_batch<float, 4, 3, true>", "k_ej_batch") == "k_h_batch"
    d = str(tmp_path / "t")
    ns = "void gnor::(anonymous namespace)::"
    step = [
        (ns + "k_fplain_batch<float, 4, true, 0>(...)", 0, 600),
        (ns + "k_fplain_batch<float, 4, true, 1>(...)", 10, 650),
        (ns + "k_nodes_batch<float>(...)", 20, 100),
        (ns + "k_h_batch<float, 4, 3, true>(...)", 30, 60),
        (ns + "k_fplain_batch<float, 4, true, 2>(...)", 110, 690),
        (ns + "k_tfsf_fix_batch<float>(...)", 690, 700),
        (ns + "k_aux_batch<float>(...)", 705, 710),
        (ns + "k_ej_batch<float, 4, 3, false, true>(...)", 715, 720),
    ]
    ev = step + [(k, a + 1000, b + 1000) for k, a, b in step]
    trace(d, ev)
    joined = {}
    spans = R.sweep_spans(d, "float", joined)
    assert spans["k_fplain_batch"][0] == 2 and abs(spans["k_fplain_batch"][1] - 0.7) < 1e-12
    assert "k_h_batch" not in spans and joined["k_h_batch"] == {"k_fplain_batch"}
    assert spans["k_ej_batch"][0] == 2
    alone = str(tmp_path / "a")
    trace(alone, [(ns + "k_h_batch<float, 4, 0, true>(...)", 0, 300),
                  (ns + "k_ej_batch<float, 4, 0, false, true>(...)", 400, 800)])
    assert R.sweep_spans(alone, "float")["k_h_batch"][0] == 1


def test_summary_scales_counters_and_sums_classes(tmp_path):
    """A copy of 2 GiB reads FETCH_SIZE 2 GiB / 2 and WRITE_SIZE 2 GiB in
    KiB, so the scales are 2 and 1.  The H sweep's two classes read 100 and
    50 KiB (scaled: 200 and 100 KiB = 0.2048 and 0.1024 MB) and write 10 and
    5 KiB; its span is 1 us, so 0.3072 + 0.01536 MB in 1 us = 322.56 GB/s."""
    base = str(tmp_path)
    tr, fe, wr, cf, cw = (os.path.join(base, n) for n in ("trace", "fetch", "write", "cfetch", "cwrite"))
    k0 = "void gnor::(anonymous namespace)::k_h<float, 2, 0, true>(...)"
    k1 = "void gnor::(anonymous namespace)::k_h<float, 2, 1, true>(...)"
    trace(tr, [(k0, 0, 800), (k1, 100, 1000)])
    write_csv(os.path.join(tr, "run_kernel_stats.csv"), ["Name", "Calls", "AverageNs"],
              [(k0, 1, 800), (k1, 1, 900)])
    counters(fe, [(k0, 100.0), (k1, 50.0)])
    counters(wr, [(k0, 10.0), (k1, 5.0)])
    copy = "void at::native::copy_kernel(...)"
    gib2 = 2.0 * 2 ** 30
    counters(cf, [(copy, gib2 / 2 / 1024)])
    counters(cw, [(copy, gib2 / 1024)])
    out = os.path.join(base, "s.md")
    R.main([tr, fe, wr, cf, cw, str(gib2), out, "cmd"])
    text = open(out).read()
    assert "FETCH_SIZE scale 2.0000, WRITE_SIZE scale 1.0000" in text
    fetch_mb = (100 + 50) * 1024 * 2 / 1e6
    write_mb = (10 + 5) * 1024 / 1e6
    assert f"<!-- traffic k_h sweep {(fetch_mb + write_mb) * 1e6:.0f} -->" in text
    assert "<!-- time k_h sweep 1.00 -->" in text
    assert f"| {(fetch_mb + write_mb) * 1e6 / 1e-6 / 1e9:.0f} |" in text


def test_bench_reads_traffic_only_for_the_current_sources(tmp_path):
    """bench.py takes a sweep's measured bytes from a summary only while the
    summary's source hash matches the kernel sources; otherwise, or without
    a summary, the traffic is reported as null."""
    import bench
    f = tmp_path / "s.md"
    f.write_text(f"library source hash (csrc/*): `{R.source_hash()}`\n"
                 "<!-- traffic k_ej sweep 123456 -->\n<!-- traffic k_h sweep 654321 -->\n")
    assert bench.measured_traffic("k_ej", str(f)) == 123456.0
    assert bench.measured_traffic("k_h", str(f)) == 654321.0
    assert bench.measured_traffic("k_ej_batch", str(f)) is None
    f.write_text("library source hash (csrc/*): `0123456789abcdef`\n<!-- traffic k_ej sweep 123456 -->\n")
    assert bench.measured_traffic("k_ej", str(f)) is None
    assert bench.measured_traffic("k_ej", str(tmp_path / "missing.md")) is None


def test_bench_reads_traffic_only_at_the_profiled_tiling(tmp_path):
    """With a timed tiling given, the traffic is taken only when it is the
    tiling of the profiled run (its --tiling option for FP32, --tiling-fp64
    for FP64); the counters of another tiling give null."""
    import bench
    f = tmp_path / "s.md"
    f.write_text(f"library source hash (csrc/*): `{R.source_hash()}`\n"
                 "    rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --tiling 4,3,2 --tiling-fp64 2,4,2 --form 3\n"
                 "<!-- traffic k_fplain sweep 777 -->\n")
    assert bench.profiled_tiling(str(f)) == (4, 3, 2)
    assert bench.profiled_tiling(str(f), fp64=True) == (2, 4, 2)
    assert bench.measured_traffic("k_fplain", str(f), (4, 3, 2)) == 777.0
    assert bench.measured_traffic("k_fplain", str(f), (2, 3, 2)) is None
    assert bench.measured_traffic("k_fplain", str(f), (2, 4, 2), fp64=True) == 777.0
    assert bench.measured_traffic("k_fplain", str(f), (4, 3, 2), fp64=True) is None
    assert bench.profiled_tiling(str(tmp_path / "missing.md")) is None
