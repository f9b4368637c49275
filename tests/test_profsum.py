"""Host logic of the profile summariser on synthetic rocprofv3 CSV files:
byte counters are scaled by what the same counter reads for the 1 GiB copy,
per-dispatch means, occupancy from wave cycles, and the file names and
commands of a split-decomposition summary."""
import csv
import json
import os

from paper_2506_00263_amd import profsum


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _counter_rows(kernel, values, copy_values):
    rows = []
    for did, v in enumerate(values, start=1):
        for name, val in v.items():
            rows.append([kernel, did, name, val])
    for name, val in copy_values.items():
        rows.append(["__amd_rocclr_copyBuffer", 99, name, val])
    return rows


def _fake_run(d, sched="async"):
    kern = profsum.KERNELS[sched][0]
    hdr = ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"]
    # the copy reads half and writes all of 1 GiB in KiB: scales x2 and x1
    _write(os.path.join(d, f"fetch_{sched}", "run_counter_collection.csv"), hdr,
           _counter_rows(f"void mcx::{kern}<1>(...)", [{"FETCH_SIZE": 100.0}, {"FETCH_SIZE": 300.0}],
                         {"FETCH_SIZE": 524288.0}))
    _write(os.path.join(d, f"write_{sched}", "run_counter_collection.csv"), hdr,
           _counter_rows(f"void mcx::{kern}<1>(...)",
                         [{"WRITE_SIZE": 1000.0, "TCC_HIT_sum": 1.0, "TCC_MISS_sum": 3.0}] * 2,
                         {"WRITE_SIZE": 1048576.0}))
    sq1 = {"SQ_WAVES": 1.0, "SQ_BUSY_CYCLES": 1.0, "SQ_WAVE_CYCLES": 2560.0, "SQ_INSTS_VALU": 10.0,
           "SQ_ACTIVE_INST_VALU": 10.0, "SQ_THREAD_CYCLES_VALU": 320.0, "SQ_WAIT_INST_ANY": 1.0,
           "SQ_WAIT_ANY": 640.0, "GRBM_GUI_ACTIVE": 8.0 * 10.0}
    _write(os.path.join(d, f"sq1_{sched}", "run_counter_collection.csv"), hdr,
           _counter_rows(f"void mcx::{kern}<1>(...)", [sq1], {}))
    _write(os.path.join(d, f"trace_{sched}", "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"],
           [[f"void mcx::{kern}<1>(...)", 4, 4000.0, 1000.0, 900.0, 1100.0]])


def test_scaled_bytes_and_occupancy(tmp_path):
    d = str(tmp_path / "prof")
    out = str(tmp_path / "out")
    _fake_run(d)
    t = profsum.summarise(d, out, "lattice_1e6")
    a = t["async_kernel"]
    assert a["read_scale"] == 2.0 and a["write_scale"] == 1.0
    assert a["read"] == 200.0 * 1024 * 2.0          # mean of 100 and 300 KiB, scaled
    assert a["write"] == 1000.0 * 1024
    assert a["bytes_per_launch"] == a["read"] + a["write"]
    assert a["source_hash"] == profsum.build.source_hash()
    text = open(os.path.join(out, "async_kernel_lattice_1e6.md")).read()
    assert "| average duration | 1.0 us |" in text
    assert "| L2 hit rate | 0.250 |" in text
    # 4 wave cycles per cycle per CU ... : 4 * 2560 / (80 / 8) / 256 = 4.00 waves per CU
    assert "| mean resident waves per CU (4 WAVE_CYCLES / GUI_ACTIVE per XCD / 256 CUs) | 4.00 of 32 |" in text
    assert "| active lanes per VALU instruction (THREAD_CYCLES_VALU / 64 ACTIVE_INST_VALU) | 0.500 |" in text
    assert json.load(open(os.path.join(out, "traffic.json")))["async_kernel"]["write"] == 1000.0 * 1024
    assert "--decomp" not in text


def test_split_summary_names(tmp_path):
    d = str(tmp_path / "prof")
    out = str(tmp_path / "out")
    _fake_run(d, "stack")
    profsum.summarise(d, out, "lattice_1e6_split", "split")
    assert sorted(os.listdir(out)) == ["stack_round_lattice_1e6_split.md", "traffic_split.json"]
    text = open(os.path.join(out, "stack_round_lattice_1e6_split.md")).read()
    assert "python3 bench.py --sched stack --decomp split --steps 5" in text
    assert "profsum <dir> profiles --decomp split" in text
