"""Host logic of the rocprofv3 summaries: copy-kernel scaling of the HBM counters and the
source-hash guard on stored traffic figures."""
import csv
import os

from paper_2005_05371_amd import profiling


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Agent_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (name, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Agent_Id": 1, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": val})


def test_traffic_scaled_by_copy_kernel(tmp_path):
    mib = 64
    # the counters read 80% of the true bytes for the copy and the kernel alike
    copy_kib = 0.8 * mib * 1024
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE",
                    [("at::native::vectorized_elementwise_kernel<16, bitwise_not_kernel_cuda>", copy_kib)] * 3 + [("amf_stage_kernel<x>", 0.8 * 2000.0)] * 4)
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE",
                    [("at::native::vectorized_elementwise_kernel<16, bitwise_not_kernel_cuda>", copy_kib)] * 3 + [("amf_stage_kernel<x>", 0.8 * 10000.0)] * 4)
    rec = profiling.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "amf_stage_kernel", mib)
    assert abs(rec["fetch_bytes"] - 2000 * 1024) <= 1
    assert abs(rec["write_bytes"] - 10000 * 1024) <= 1
    assert rec["copy_scale"] == [1.25, 1.25]
    assert rec["dispatches"] == [4, 4]


def test_record_roundtrip_and_hash_guard(tmp_path):
    path = str(tmp_path / "t.md")
    rec = {"fetch_bytes": 1, "write_bytes": 2, "copy_scale": [1.0, 1.0], "raw_kib": [0, 0],
           "copy_raw_kib": [0, 0], "dispatches": [1, 1]}
    profiling.write_record(path, "k", "w", rec, "cmd")
    profiling.write_record(path, "k", "w", dict(rec, fetch_bytes=5), "cmd")  # replaces the first
    got = profiling.measured_traffic("k", "w", path)
    assert got["fetch_bytes"] == 5 and got["source_sha256"] == profiling.kernel_source_hash()
    assert profiling.measured_traffic("k", "other", path) is None
    text = open(path).read().replace(profiling.kernel_source_hash(), "0" * 16)
    open(path, "w").write(text)
    assert profiling.measured_traffic("k", "w", path) is None  # sources changed: no figure


def test_record_replaces_its_command_line(tmp_path):
    path = str(tmp_path / "t.md")
    rec = {"fetch_bytes": 1, "write_bytes": 2, "copy_scale": [1.0, 1.0], "raw_kib": [0, 0],
           "copy_raw_kib": [0, 0], "dispatches": [1, 1]}
    profiling.write_record(path, "k", "w", rec, "first")
    profiling.write_record(path, "k", "w", rec, "second")
    text = open(path).read()
    assert "first" not in text and text.count("<!-- command for k / w:") == 1


def test_valu_record_medians_and_guard(tmp_path):
    d = str(tmp_path / "v")
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Agent_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, v in enumerate([1000.0, 1200.0, 1100.0]):  # three dispatches
            for c, x in (("SQ_WAVES", 10.0), ("SQ_INSTS_VALU", v), ("SQ_INSTS_SALU", v / 2),
                         ("SQ_INSTS_LDS", 7.0)):
                w.writerow({"Dispatch_Id": i, "Agent_Id": 1, "Kernel_Name": "amf_stage_kernel<x>",
                            "Counter_Name": c, "Counter_Value": x})
            w.writerow({"Dispatch_Id": 100 + i, "Agent_Id": 1, "Kernel_Name": "other",
                        "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 9e9})
    rec = profiling.valu(d, "amf_stage_kernel")
    assert rec == {"waves": 10, "valu_insts": 1100, "salu_insts": 550, "lds_insts": 7, "dispatches": 3}
    path = str(tmp_path / "v.md")
    profiling.write_record(path, "k", "w", rec, "cmd", kind="valu")
    assert profiling.measured_valu("k", "w", path)["valu_insts"] == 1100
    assert profiling.measured_traffic("k", "w", path) is None  # kinds do not mix


def test_code_text_ignores_comments_and_layout():
    a = 'int f(int x) { // twice\n  return 2 * x; /* no\n overflow */ }\nconst char *s = "a // b";'
    b = 'int f(int x) {\n\n    return 2 * x;   }\nconst char *s = "a // b";'
    assert profiling.code_text(a) == profiling.code_text(b)
    # a code change, and a change inside a string literal, show
    assert profiling.code_text(a) != profiling.code_text(a.replace("2 * x", "3 * x"))
    assert profiling.code_text(a) != profiling.code_text(a.replace('"a // b"', '"a // c"'))
    assert profiling.code_text("char c = '\\''; // q") == "char c = '\\'';"


def test_counters_table_groups_by_kernel_and_grid(tmp_path):
    d = tmp_path / "c"
    os.makedirs(d)
    fields = ["Dispatch_Id", "Agent_Id", "Grid_Size", "Kernel_Name", "Workgroup_Size", "Counter_Name",
              "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows = []
    # three dispatches of 8 workgroups, one of 2, one of another kernel; VALU split over two
    # rows of a dispatch (summed), waves per dispatch = 4 x workgroups
    for disp, (name, groups, valu, t) in enumerate([("k<a>", 8, 3200.0, 10000), ("k<a>", 8, 3520.0, 12000),
                                                    ("k<a>", 8, 3840.0, 11000), ("k<a>", 2, 400.0, 3000),
                                                    ("other", 8, 1.0, 1000)]):
        base = {"Dispatch_Id": disp, "Agent_Id": 1, "Grid_Size": 256 * groups, "Kernel_Name": name,
                "Workgroup_Size": 256, "Start_Timestamp": 0, "End_Timestamp": t}
        rows.append(dict(base, Counter_Name="SQ_WAVES", Counter_Value=4 * groups))
        rows.append(dict(base, Counter_Name="SQ_INSTS_VALU", Counter_Value=valu / 2))
        rows.append(dict(base, Counter_Name="SQ_INSTS_VALU", Counter_Value=valu / 2))
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)
    lines = profiling.counters_table(str(d), "k<").splitlines()
    assert lines[0] == "| kernel | workgroups | dispatches | median us | SQ_INSTS_VALU / wave | SQ_WAVES |"
    assert lines[2] == "| `k<a>` | 8 | 3 | 11.0 | 110 | 32.00 |"  # 3520 / 32 waves
    assert lines[3] == "| `k<a>` | 2 | 1 | 3.0 | 50.00 | 8.00 |"
    assert len(lines) == 4


def test_grid_table_splits_launch_sizes(tmp_path):
    d = tmp_path / "t"
    os.makedirs(d)
    fields = ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Workgroup_Size_X",
              "Workgroup_Size_Y", "Workgroup_Size_Z", "Start_Timestamp", "End_Timestamp"]
    rows = [("k", (2560, 1, 1), 5000), ("k", (2560, 1, 1), 7000), ("k", (2560, 1, 1), 6000),
            ("k", (256, 4, 2), 1000), ("other", (64, 1, 1), 500)]
    with open(d / "x_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for name, (gx, gy, gz), ns in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size_X": gx, "Grid_Size_Y": gy, "Grid_Size_Z": gz,
                        "Workgroup_Size_X": 256, "Workgroup_Size_Y": 1, "Workgroup_Size_Z": 1,
                        "Start_Timestamp": 100, "End_Timestamp": 100 + ns})
    lines = profiling.grid_table(str(d), "k").splitlines()
    assert lines[2] == "| `k` | 10 | 3 | 6.0 | 5.0 | 7.0 |"
    assert lines[3] == "| `k` | 8 | 1 | 1.0 | 1.0 | 1.0 |"  # 1 x 4 x 2 workgroups
    assert len(lines) == 4
