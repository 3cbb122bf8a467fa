"""The rocprofv3 summarizers of bench.py on synthetic CSV runs (CPU only): the marker windows, the
copy calibration of FETCH_SIZE / WRITE_SIZE, the per-class profiled-pass means, the per-shape runs
of the stencil-variant summary and the legs window."""
import csv
import json
import os

import pytest

import bench

MARK = "void at::native::vectorized_elementwise_kernel<4, at::native::bitwise_not_kernel_cuda(int)>"
COPY = "__amd_rocclr_copyBuffer"
F32 = "void sgn::(anonymous namespace)::stencil_staged_kernel<float, HIP_vector_type<float, 2u>, false, false>(P)"
F32D = "void sgn::(anonymous namespace)::stencil_staged_kernel<float, HIP_vector_type<float, 2u>, true, true>(P)"
PACK = "void sgn::(anonymous namespace)::pack_kernel(x)"
LZ = "void sgn::(anonymous namespace)::lz_update_kernel<false>(x)"


def _write_trace(d, seq):
    """seq: (kernel, duration in us); one dispatch after another"""
    os.makedirs(d)
    with open(os.path.join(d, "run_kernel_trace.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Workgroup_Size_X", "LDS_Block_Size", "Grid_Size_X",
                    "Start_Timestamp", "End_Timestamp"])
        t = 1000
        for i, (k, us) in enumerate(seq):
            w.writerow([i + 1, k, 256, 0, 1024, t, t + int(us * 1000)])
            t += int(us * 1000) + 500
    with open(os.path.join(d, "run_kernel_stats.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writerow([F32, 1, 1000, 1000, 100.0])


def _write_counters(d, seq, value):
    """value(kernel, index) -> {counter: value}"""
    os.makedirs(d)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Grid_Size", "Counter_Name",
                    "Counter_Value", "Start_Timestamp", "End_Timestamp"])
        t = 1000
        for i, (k, us) in enumerate(seq):
            for c, v in value(k, i).items():
                w.writerow([i + 1, k, 256, 0, 1024, c, v, t, t + 10])
            t += 20


def _fetch(k, i):
    # a copy of 512 MiB reads 262144 KiB in FETCH_SIZE (half its bytes): factor 2
    return {"FETCH_SIZE": 262144.0 if k == COPY else (100000.0 if k == F32 else 150000.0)}


def _write(k, i):
    return {"WRITE_SIZE": 524288.0 if k == COPY else 60000.0}


def test_headline_summary_windows_and_calibration(tmp_path, monkeypatch):
    # outside the window: an autotuner-like launch of 40 us that must not enter the class means
    seq = [(COPY, 100)] * 3 + [(F32, 40.0), (MARK, 2)] + [(F32, 70.0), (F32D, 90.0)] * 4 + [(MARK, 2), (F32, 40.0)]
    d = str(tmp_path)
    _write_trace(os.path.join(d, "tr"), seq)
    _write_counters(os.path.join(d, "fe"), seq, _fetch)
    _write_counters(os.path.join(d, "wr"), seq, _write)
    out = os.path.join(d, "summary.md")
    monkeypatch.setattr(bench, "source_digest", lambda: "feedface")
    bench.summarize_rocprof(os.path.join(d, "tr"), os.path.join(d, "fe"), os.path.join(d, "wr"), out, "cmd")
    lines = open(out).read().splitlines()
    trace_us = {l.split()[1]: float(l.split()[2]) for l in lines if l.startswith("trace_us ")}
    traffic = {l.split()[1]: float(l.split()[2]) for l in lines if l.startswith("traffic ")}
    assert trace_us == {"stencil_f32": pytest.approx(80.0, abs=0.01)}  # (70 + 90) / 2 inside the window only
    # per class, over the profiled pass's dispatches only: (FETCH x 2 + WRITE) KiB x 1024 of the
    # four plain and four epilogue launches (the two outside the window do not count)
    want = (4 * (100000.0 * 2 + 60000.0) + 4 * (150000.0 * 2 + 60000.0)) / 8 * 1024
    assert traffic["stencil_f32"] == pytest.approx(want, rel=1e-6)
    assert "source_sha256 feedface" in lines
    # and profile_summary reads both back while the sources hash to the recorded value
    monkeypatch.setattr(bench, "PROFILE", out)
    t, us = bench.profile_summary()
    assert us["stencil_f32"] == pytest.approx(80.0, abs=0.01) and t["stencil_f32"] == pytest.approx(want, rel=1e-6)
    monkeypatch.setattr(bench, "source_digest", lambda: "changed")
    assert bench.profile_summary() == ({}, {})


def test_headline_summary_refuses_a_trace_without_markers(tmp_path, monkeypatch):
    seq = [(COPY, 100)] * 3 + [(F32, 70.0)] * 4
    d = str(tmp_path)
    _write_trace(os.path.join(d, "tr"), seq)
    _write_counters(os.path.join(d, "fe"), seq, _fetch)
    _write_counters(os.path.join(d, "wr"), seq, _write)
    with pytest.raises(SystemExit):
        bench.summarize_rocprof(os.path.join(d, "tr"), os.path.join(d, "fe"), os.path.join(d, "wr"),
                                os.path.join(d, "s.md"), "cmd")


def test_stencil_variant_runs_are_labelled_in_order(tmp_path):
    # two shapes with the same kernel name and block size: told apart by the non-stencil kernels
    # between their runs of 3 + 20 dispatches
    seq = [(COPY, 100)] * 2 + [(MARK, 2), (PACK, 3)] + [(F32, 60.0)] * 23 + [(PACK, 3)] + [(F32, 50.0)] * 23 + [(MARK, 2)]
    d = str(tmp_path)
    _write_trace(os.path.join(d, "tr"), seq)
    names = bench.COUNTER_SET.split()
    _write_counters(os.path.join(d, "pmc"), seq, lambda k, i: {c: float(i) for c in names})
    _write_counters(os.path.join(d, "fe"), seq, _fetch)
    _write_counters(os.path.join(d, "wr"), seq, _write)
    vj = os.path.join(d, "v.json")
    open(vj, "w").write(json.dumps({"stencil_variants": [
        {"prec": "f32", "kernel": "staged", "block_sites": 576, "t_slices": 2, "us": 60.0},
        {"prec": "f32", "kernel": "staged", "block_sites": 576, "t_slices": 1, "us": 50.0}]}) + "\n")
    out = os.path.join(d, "c.md")
    bench.summarize_counters(os.path.join(d, "tr"), os.path.join(d, "pmc"), os.path.join(d, "fe"),
                             os.path.join(d, "wr"), vj, out, "cmd")
    rows = [l for l in open(out).read().splitlines() if l.startswith("| f32 |")]
    assert len(rows) == 2
    assert "| 576 x 2 |" in rows[0] and "| 60.0 |" in rows[0]
    assert "| 576 x 1 |" in rows[1] and "| 50.0 |" in rows[1]
    # counters: the mean over the last 20 of the 23 dispatches of each run (dispatch indices 7..26, 31..50)
    assert f"| {sum(range(7, 27)) / 20:.3g} |" in rows[0]
    assert f"| {sum(range(31, 51)) / 20:.3g} |" in rows[1]


def test_legs_summary_uses_the_second_marker_pair(tmp_path):
    seq = ([(COPY, 100)] * 2 + [(MARK, 2), (LZ, 50.0), (MARK, 2), (MARK, 2)] + [(LZ, 180.0)] * 10 + [(MARK, 2)]
           + [(LZ, 60.0)] * 5)
    d = str(tmp_path)
    _write_trace(os.path.join(d, "tr"), seq)
    # an lz update reading 6 and writing 2 FP64 vectors of 24^3 x 48 (121.5 MiB each)
    vec_kib = 12 * 24 ** 3 * 48 * 16 / 1024
    _write_counters(os.path.join(d, "fe"), seq, lambda k, i: {"FETCH_SIZE": 262144.0 if k == COPY else 3 * vec_kib})
    _write_counters(os.path.join(d, "wr"), seq, lambda k, i: {"WRITE_SIZE": 524288.0 if k == COPY else 2 * vec_kib})
    out = os.path.join(d, "legs.md")
    bench.summarize_legs(os.path.join(d, "tr"), os.path.join(d, "fe"), os.path.join(d, "wr"), out, "cmd")
    text = open(out).read()
    assert "over 10 dispatches" in text  # only the second pair's window
    assert "| lz_update_kernel<false> | 10 | 1.80 | 180.0 | 100.0 |" in text
    assert "| 6.00 | 2.00 |" in text


def test_stored_site_bytes_of_the_byte_model():
    # two spinors and four two-row links per site; a temporal-gauge lattice skips the time link off
    # its last slice in the staged kernels only
    assert bench.stored_site_bytes("f64", 6, False, 48) == 2 * 192 + 4 * 6 * 16
    assert bench.stored_site_bytes("f32", 6, False, 48) == 384
    assert bench.stored_site_bytes("h16", 6, False, 48) == 288
    assert bench.stored_site_bytes("f32", 6, True, 48) == pytest.approx(192 + (3 + 1 / 48) * 48)
    assert bench.stored_site_bytes("f32", 6, True, 48, staged=False) == 384
    assert bench.stored_site_bytes("f64", 9, True, 24) == pytest.approx(384 + (3 + 1 / 24) * 144)
