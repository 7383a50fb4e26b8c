"""Host logic of the measurement record: the rocprofv3 summaries kept in profiles/
and the HBM traffic figure bench.py reports (no GPU needed)."""

import csv
import json

import pytest

import bench
from paper_2208_12569_amd import profiling

TRACER = "void fq::(anonymous namespace)::trace_kernel<float, float, 1, true, false, 0, false>(fq::TraceJob const*)"
COPY = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctor_add<float>>"


def _counter_csv(path, counter, rows):
    """rows: (dispatch id, kernel name, [values of the counter's instances])"""
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, name, vals in rows:
            for v in vals:
                w.writerow([d, name, counter, v])
                w.writerow([d, name, "OTHER", 1e9])  # other counters are ignored


def test_traffic_is_scaled_by_the_calibration_copy(tmp_path):
    gib_kib = profiling.COPY_BYTES / 1024.0
    # the copy reads twice its size on FETCH_SIZE and its size on WRITE_SIZE; the
    # tracer's instances (one row per block of the chip) add up per dispatch
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    _counter_csv(f, "FETCH_SIZE", [(1, TRACER, [100.0, 300.0]), (2, TRACER, [600.0]),
                                   (3, COPY, [gib_kib, gib_kib])])
    _counter_csv(w, "WRITE_SIZE", [(1, TRACER, [50.0]), (2, TRACER, [70.0]), (3, COPY, [gib_kib])])
    t = profiling.traffic(str(f), str(w))
    assert t["launches"] == 2
    assert t["fetch_calibration"] == pytest.approx(0.5)
    assert t["write_calibration"] == pytest.approx(1.0)
    assert t["fetch_bytes_per_launch"] == pytest.approx((400.0 + 600.0) / 2 * 1024.0 * 0.5)
    assert t["write_bytes_per_launch"] == pytest.approx((50.0 + 70.0) / 2 * 1024.0)
    assert t["traffic_bytes_per_launch"] == pytest.approx(t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"])
    assert t["kernel_source_sha"] == profiling.kernel_source_sha()


def test_traffic_needs_the_calibration_copy_and_the_kernel(tmp_path):
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    _counter_csv(f, "FETCH_SIZE", [(1, TRACER, [1.0])])
    _counter_csv(w, "WRITE_SIZE", [(1, TRACER, [1.0])])
    with pytest.raises(ValueError, match="calibration copy"):
        profiling.traffic(str(f), str(w))
    _counter_csv(f, "FETCH_SIZE", [(1, COPY, [1.0])])
    _counter_csv(w, "WRITE_SIZE", [(1, COPY, [1.0])])
    with pytest.raises(ValueError, match="not found"):
        profiling.traffic(str(f), str(w))


def test_stats_table_is_ordered_by_total_time(tmp_path):
    p = tmp_path / "s.csv"
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs", "Percentage"])
        w.writerow(["fq::(anonymous namespace)::stencil_kernel(fq::MapJob)", 2, 2e5, 1e5, 9e4, 1.1e5, 5.0])
        w.writerow([TRACER, 2, 8e6, 4e6, 3.9e6, 4.1e6, 90.0])
        w.writerow(["fill", 4, 2e4, 5e3, 4e3, 6e3, 0.5])
    md = profiling.stats_md(str(p), "rocprofv3 --kernel-trace --stats -- python3 bench.py")
    lines = md.splitlines()
    assert lines[0] == "Command: `rocprofv3 --kernel-trace --stats -- python3 bench.py`"
    rows = [l for l in lines if l.startswith("| ") and not l.startswith("| kernel")]
    assert rows[0].startswith("| trace_kernel<float, float, 1, true, false, 0, false>")
    assert "| 8.000 | 4000.0 |" in rows[0]
    assert rows[1].startswith("| stencil_kernel |")
    assert rows[2].startswith("| fill |")


def test_bench_reports_traffic_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    rec = {"c2/f32x": {"kernel_source_sha": profiling.kernel_source_sha(),
                       "traffic_bytes_per_launch": 6.2e9}}
    (tmp_path / "profiles" / "trace_kernel_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile("c2", "f32x") == pytest.approx(6.2e9)
    assert bench.traffic_from_profile("c2", "f64") is None
    rec["c2/f32x"]["kernel_source_sha"] = "0" * 16
    (tmp_path / "profiles" / "trace_kernel_traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profile("c2", "f32x") is None



def _multi_counter_csv(path, dispatches):
    """dispatches: (dispatch id, kernel name, {counter: [instance values]})"""
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, name, cs in dispatches:
            for c, vals in cs.items():
                for v in vals:
                    w.writerow([d, name, c, v])


def test_valu_mix_derives_busy_lanes_and_per_step_counts(tmp_path):
    """Two launches of the tracer (instances summed per dispatch, launches averaged):
    1.0e9 VALU instructions per launch on 1024 SIMDs for 2 ms at 4 cycles each is
    1e9 * 4 / (1024 * 2e-3 * 2.4e9) = 81.4% busy; 1e9 * 64 / 5e7 trial steps = 1280
    per lane trial step; 48 lanes per instruction; 'other' is VALU minus the listed
    classes."""
    a = tmp_path / "a.csv"
    b = tmp_path / "b.csv"
    ca = {c: [0.0] for c in profiling.VALU_A}
    ca.update({"SQ_INSTS_VALU": [4e8, 6e8], "SQ_ACTIVE_INST_VALU": [1e9], "SQ_THREAD_CYCLES_VALU": [48e9],
               "SQ_INSTS_VALU_FMA_F32": [3e8], "SQ_INSTS_VALU_MUL_F32": [1e8], "SQ_INSTS_VALU_ADD_F32": [1e8]})
    cb = {c: [0.0] for c in profiling.VALU_B}
    cb.update({"SQ_INSTS_VALU_INT32": [1e8], "SQ_INSTS_VMEM_RD": [2.5e7]})
    _multi_counter_csv(a, [(1, TRACER, ca), (2, TRACER, ca), (3, COPY, {"SQ_INSTS_VALU": [5.0]})])
    _multi_counter_csv(b, [(1, TRACER, cb), (2, TRACER, cb)])
    md = profiling.valu_md(str(a), str(b), "cmd a", "cmd b", 2.0, 5e7, 1e8)
    assert "= 48.0 of 64" in md
    assert "2.4 GHz) = 81%" in md
    assert "trial steps = 1280" in md
    assert "bit operations): 4e+08, 40%" in md
    assert "| SQ_INSTS_VALU_FMA_F32 | 3.0000e+08 | 30.0% |" in md
    assert "per wave-level cell fetch: 16.0" in md
