"""Host logic of the measurement (no GPU): the rocprofv3 summaries of
paper_0705_4371_amd/profiling.py on synthetic CSV files, and bench.py's rule
that the HBM traffic is reported only while the recorded kernel source hash
matches the sources."""
import csv
import json
import os
import types

import pytest

from paper_0705_4371_amd import profiling


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_stats_markdown_converts_ns_to_us(tmp_path):
    _write_csv(str(tmp_path / "run" / "x_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"],
               [["k_a(int)", 10, 4000000, 400000.0, 75.5, 390000, 410000],
                ["k_b|bar", 3, 30000, 10000.0, 24.5, 9000, 11000]])
    md = profiling.stats_markdown(str(tmp_path), command="cmd --flag", title="T")
    assert md.startswith("# T")
    assert "    cmd --flag" in md
    assert "| `k_a(int)` | 10 | 400.0 | 390.0 | 410.0 | 75.50% |" in md
    assert "k_b\\|bar" in md   # a pipe in a kernel name does not break the table


def _counter_rows(kernel, counter, values):
    return [[kernel, counter, v] for v in values]


def test_pmc_summary_scales_by_the_copy(tmp_path):
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # the step kernel: FETCH_SIZE reads half of what it moves (as the copy does)
    _write_csv(str(tmp_path / "f" / "a_counter_collection.csv"), hdr,
               _counter_rows("k_step<x>", "FETCH_SIZE", [1000.0, 512.0, 512.0]) +
               _counter_rows("other", "FETCH_SIZE", [7.0]))
    _write_csv(str(tmp_path / "w" / "a_counter_collection.csv"), hdr,
               _counter_rows("k_step<x>", "WRITE_SIZE", [3000.0, 1024.0, 1024.0]))
    _write_csv(str(tmp_path / "cf" / "c_counter_collection.csv"), hdr,
               _counter_rows("copyBuffer", "FETCH_SIZE", [512.0]))
    _write_csv(str(tmp_path / "cw" / "c_counter_collection.csv"), hdr,
               _counter_rows("copyBuffer", "WRITE_SIZE", [1024.0]))
    a = types.SimpleNamespace(
        kernel="k_step", kernel_match="k_step<", fetch=str(tmp_path / "f"), write=str(tmp_path / "w"),
        copy_fetch=str(tmp_path / "cf"), copy_write=str(tmp_path / "cw"), copy_kernel="copyBuffer",
        copy_bytes=1024.0 * 1024.0, copy_what="1 MiB copy", algorithmic_bytes=2.0 * 1024 * 1024,
        workload="w", skip_first=1, command=["c1"])
    s = profiling.pmc_summary(a)
    assert s["fetch_size_kib_per_dispatch"] == 512.0 and s["write_size_kib_per_dispatch"] == 1024.0
    assert s["dispatches_averaged"] == 2
    assert s["copy_calibration"]["fetch_factor"] == 2.0 and s["copy_calibration"]["write_factor"] == 1.0
    assert s["hbm_read_bytes_per_launch"] == 1024 * 1024 and s["hbm_write_bytes_per_launch"] == 1024 * 1024
    assert s["ratio_to_algorithmic"] == 1.0
    assert s["kernel_source_hash"] == profiling.kernel_source_hash()


def test_counter_without_dispatches_raises(tmp_path):
    _write_csv(str(tmp_path / "f" / "a_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
               _counter_rows("other", "FETCH_SIZE", [1.0]))
    with pytest.raises(ValueError):
        profiling.counter_per_dispatch(str(tmp_path / "f"), "k_step", "FETCH_SIZE")


def test_kernel_source_hash_covers_the_step_sources():
    h = profiling.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    for name in profiling.STEP_SOURCES:
        assert os.path.exists(os.path.join(profiling.ROOT, "paper_0705_4371_amd", "csrc", name)), name


def test_bench_reports_traffic_only_for_the_current_kernel(tmp_path, monkeypatch):
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(str(tmp_path / "profiles"))
    path = str(tmp_path / "profiles" / "k_step_wl_fp32_pmc.json")
    assert bench.traffic_from_profile("wl", "fp32", 1) is None          # no summary
    with open(path, "w") as fh:
        json.dump({"kernel_source_hash": profiling.kernel_source_hash(), "hbm_bytes_per_launch": 123}, fh)
    assert bench.traffic_from_profile("wl", "fp32", 1) == 123
    with open(path, "w") as fh:
        json.dump({"kernel_source_hash": "0" * 16, "hbm_bytes_per_launch": 123}, fh)
    assert bench.traffic_from_profile("wl", "fp32", 1) is None          # kernel changed since


def test_valu_summary_per_wavefront_with_kernel_patterns(tmp_path):
    """Instruction counts per 64 sites: the median over a kernel's dispatches
    with at least half its largest count (the smaller dispatches are another
    workload), counters split over two runs, named kernel patterns, and the
    HBM counters in KiB when a run counted them."""
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    vals = {"SQ_INSTS_VALU": 1000.0, "SQ_INSTS_VALU_TRANS_F32": 40.0, "SQ_INSTS_VALU_TRANS_F64": 10.0,
            "SQ_INSTS_MFMA": 0.0}
    rows1 = []
    for d, scale in ((1, 1.0), (2, 1.02), (3, 0.98), (4, 0.1)):     # dispatch 4: a smaller solve
        rows1 += [[d, "void k_x<0>(A)", c, v * scale] for c, v in vals.items()]
    rows2 = []
    for d in (1, 2, 3):
        rows2 += [[d, "void k_x<0>(A)", "SQ_INSTS_VALU_FMA_F64", 200.0], [d, "void k_x<0>(A)", "SQ_INSTS_VALU_ADD_F64", 64.0],
                  [d, "void k_x<0>(A)", "SQ_INSTS_VALU_MUL_F64", 56.0], [d, "void k_x<0>(A)", "FETCH_SIZE", 512.0]]
    _write_csv(str(tmp_path / "r1" / "p_counter_collection.csv"), hdr, rows1)
    _write_csv(str(tmp_path / "r2" / "p_counter_collection.csv"), hdr, rows2)
    a = types.SimpleNamespace(dirs=[str(tmp_path / "r1"), str(tmp_path / "r2")], sites=640, workload="w",
                              command=["c"], kernel=["x=k_x<0>("])
    out = profiling.valu_summary(a)
    k = out["kernels"]["x"]
    assert k["dispatches"] == 3
    assert k["valu"] == 100.0 and k["transcendental"] == 5.0 and k["fp64"] == 32.0 and k["mfma"] == 0.0
    assert k["fetch_size_kib"] == 512.0 and "write_size_kib" not in k
    assert out["fstar_source_hash"] == profiling.fstar_source_hash()
    assert out["step_source_hash"] == profiling.kernel_source_hash()
