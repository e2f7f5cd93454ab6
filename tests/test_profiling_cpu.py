"""The rocprofv3 summarisers in paper_2407_19048_amd/profiling.py on small
synthetic result files: kernel-time table, counter table, VALU-issue table
and the HBM traffic record (copy-probe calibration, variant and grid
selection, source-hash invalidation)."""

import csv
import json
import os

import pytest

from paper_2407_19048_amd import profiling

COUNTER_FIELDS = ["Correlation_Id", "Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value",
                  "Start_Timestamp", "End_Timestamp"]


def _write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=COUNTER_FIELDS)
        w.writeheader()
        for i, r in enumerate(rows):
            w.writerow(dict({"Correlation_Id": i, "Dispatch_Id": r.get("disp", i)}, **{
                "Grid_Size": r["grid"], "Kernel_Name": r["name"], "Counter_Name": r["counter"],
                "Counter_Value": r["value"], "Start_Timestamp": r.get("t0", 0), "End_Timestamp": r.get("t1", 0)}))


def test_short_names():
    assert profiling.short_name("void (anonymous namespace)::k_welch<float, double, 4096, 0, 3>"
                                "((anonymous namespace)::WelchArgs)") == "k_welch<float, double, 4096, 0, 3>"
    assert profiling.short_name("(anonymous namespace)::k_sample_params((anonymous namespace)::SampleArgs)") \
        == "k_sample_params"
    assert profiling.short_name("k_plain") == "k_plain"


def test_trace_table_groups_by_grid(tmp_path):
    p = tmp_path / "t.csv"
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z",
                    "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z"])
        for t0, t1 in ((0, 1000000), (0, 3000000), (0, 2000000)):
            w.writerow(["void k_a<1>(Args)", t0, t1, 512, 1, 1, 256, 1, 1])
        w.writerow(["void k_a<1>(Args)", 0, 9000000, 1024, 1, 1, 256, 1, 1])
        w.writerow(["void k_b(Args)", 0, 5000000, 64, 1, 1, 64, 1, 1])
        w.writerow(["void k_c<float, 4>(Args)", 0, 7000000, 64, 1, 1, 64, 1, 1])
        w.writerow(["void k_c<float, 1>(Args)", 0, 7000000, 64, 1, 1, 64, 1, 1])
    t = profiling.trace_table(str(p), "k_a", "T", "cmd")
    lines = [l for l in t.splitlines() if l.startswith("| `")]
    assert lines[0] == "| `k_a<1>` | 1024 | 256 | 1 | 9.0000 ms | 9.0000 ms | 9.000 ms |"
    assert lines[1] == "| `k_a<1>` | 512 | 256 | 3 | 2.0000 ms | 2.0000 ms | 6.000 ms |"
    assert len(lines) == 2
    t = profiling.trace_table(str(p), "k_a@512|7;k_b", "T", "cmd")
    assert [l.split("|")[1:3] for l in t.splitlines() if l.startswith("| `")] == [
        [" `k_a<1>` ", " 512 "], [" `k_b` ", " 64 "]]
    # substrings with commas select template arguments
    t = profiling.trace_table(str(p), "k_c<float, 4", "T", "cmd")
    assert [l.split("|")[1].strip() for l in t.splitlines() if l.startswith("| `")] == ["`k_c<float, 4>`"]


def test_stats_table_sorted_by_total(tmp_path):
    p = tmp_path / "s.csv"
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs"])
        w.writerow(["k_small", 10, 1000000, 100000])
        w.writerow(["k_big", 4, 4000000, 1000000])
    t = profiling.stats_table(str(p), "T", "cmd")
    lines = [l for l in t.splitlines() if l.startswith("| `")]
    assert lines[0].startswith("| `k_big`") and "1.0000 ms" in lines[0] and "80.00 %" in lines[0]
    assert lines[1].startswith("| `k_small`") and "20.00 %" in lines[1]


def test_valu_table_derived_columns(tmp_path):
    d = str(tmp_path / "valu")
    name, grid = "k_welch<float, double, 4096, 0, 3>", 1572864
    rows = []
    # two dispatches of 1 ms each: 1024 SIMDs x 1e-3 s x 2.4e9 / 4 = 614.4e6
    # instructions would be 100 % issue; 307.2e6 is 50 %
    for disp, (t0, t1) in enumerate([(0, 1000000), (5000000, 6000000)]):
        for c, v in (("SQ_INSTS_VALU", 307.2e6), ("SQ_WAVES", 1000), ("SQ_LDS_BANK_CONFLICT", 10),
                     ("SQ_LDS_IDX_ACTIVE", 100), ("SQ_WAIT_ANY", 25), ("SQ_WAVE_CYCLES", 100)):
            rows.append(dict(disp=disp, grid=grid, name=name, counter=c, value=v, t0=t0, t1=t1))
    rows.append(dict(grid=64, name="other_kernel", counter="SQ_INSTS_VALU", value=1, t0=0, t1=1))
    _write_counters(d, rows)
    t = profiling.valu_table(d, "k_welch", "V", "cmd")
    line = [l for l in t.splitlines() if l.startswith("| `k_welch")][0]
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert cells[1] == str(grid) and cells[2] == "2" and cells[3] == "1000"
    assert cells[4] == "307200" and cells[5] == "1.0000 ms"
    assert cells[6] == "50.0 %" and cells[7] == "10.0 %" and cells[8] == "25.0 %"
    assert "other_kernel" not in t
    with pytest.raises(ValueError):
        profiling.valu_table(d, "absent", "V", "cmd")


def test_traffic_record_scaled_by_copy_probe(tmp_path, monkeypatch):
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    copy_bytes = 1 << 30
    kern, grid = "k_welch<float, double, 4096, 0, 3>", 1572864
    # counters read half the true bytes on the copy: scale 2
    _write_counters(fd, [
        dict(grid=1 << 28, name="copy_kernel", counter="FETCH_SIZE", value=copy_bytes / 1024 / 2),
        dict(grid=1 << 20, name="copy_kernel", counter="FETCH_SIZE", value=1.0),
        dict(grid=grid, name=kern, counter="FETCH_SIZE", value=1000.0),
        dict(grid=grid, name=kern, counter="FETCH_SIZE", value=3000.0),
        dict(grid=grid, name="k_welch<float, double, 4096, 0, 2>", counter="FETCH_SIZE", value=9e9),
        dict(grid=7, name=kern, counter="FETCH_SIZE", value=9e9)])
    _write_counters(wd, [
        dict(grid=1 << 28, name="copy_kernel", counter="WRITE_SIZE", value=copy_bytes / 1024),
        dict(grid=grid, name=kern, counter="WRITE_SIZE", value=50.0)])
    monkeypatch.setattr(profiling, "ROOT", str(tmp_path))
    rec = profiling.summarise(fd, wd, "k_welch", kern, grid, "wl", 1.0, "cmd")
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == 2000 * 1024 * 2
    assert rec["write_bytes_per_launch"] == 50 * 1024
    assert rec["hbm_bytes_per_launch"] == 2000 * 1024 * 2 + 50 * 1024
    assert rec["dispatches"] == [2, 1]
    with open(profiling.traffic_path("k_welch", "wl")) as fh:
        assert json.load(fh)["hbm_bytes_per_launch"] == rec["hbm_bytes_per_launch"]
    # the stored record counts only while the kernel sources are unchanged
    assert profiling.measured_traffic("k_welch", "wl") == rec["hbm_bytes_per_launch"]
    monkeypatch.setattr(profiling, "kernel_source_hash", lambda kernel=None: "changed")
    assert profiling.measured_traffic("k_welch", "wl") is None


def test_source_hash_covers_the_kernels_translation_unit():
    # the plain kernels' record depends on their translation unit only
    assert "paper_2407_19048_amd/csrc/gwgen.hip" in profiling.KERNEL_SOURCES["k_welch"]
    assert not any("gw_long" in f for f in profiling.KERNEL_SOURCES["k_window"])
    assert profiling.kernel_source_hash("k_welch") == profiling.kernel_source_hash("k_window")
    assert profiling.kernel_source_hash("k_other") != profiling.kernel_source_hash("k_welch")
