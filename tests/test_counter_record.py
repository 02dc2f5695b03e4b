"""Host logic of the roofline's counter record (CPU): bench.py --counter-record on synthetic rocprofv3
CSVs — the headline record averages the last launches of the ray march per counter, a counter
collected in several passes is averaged rather than added, and FETCH_SIZE / WRITE_SIZE are scaled
by what the same counters read for the 1 GiB device copy of the same run."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
MARCH = "void raypc::(anonymous namespace)::raymarch_kernel<4, 5, false, false, false, false>(raypc::RenderArgs)"
BATCH = "void raypc::(anonymous namespace)::raymarch_batch_kernel<4, 5, false>(raypc::RenderArgs const*, raypc::BatchRanges)"
COPY = "__amd_rocclr_copyBuffer"


def write_pass(path, launches):
    """launches: [(dispatch id, kernel name, {counter: [values per dimension]})]"""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, name, counters in launches:
            for c, vals in counters.items():
                for v in vals:
                    w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v})


def test_headline_record(tmp_path):
    root = tmp_path / "head"
    # pass 1: an autotuner launch (ignored: only the last 2 launches of the ray march count), two
    # frames, the copy; SQ_INSTS_LDS is summed over its per-XCD dimension values
    write_pass(str(root / "p1" / "p1_counter_collection.csv"), [
        (1, MARCH, {"SQ_INSTS_VALU": [999.0], "SQ_INSTS_LDS": [999.0]}),
        (2, MARCH, {"SQ_INSTS_VALU": [100.0], "SQ_INSTS_LDS": [10.0, 10.0]}),
        (3, MARCH, {"SQ_INSTS_VALU": [300.0], "SQ_INSTS_LDS": [30.0, 10.0]}),
        (4, COPY, {"SQ_INSTS_VALU": [5.0]}),
    ])
    # pass 2 collects SQ_INSTS_LDS too: the record averages it with pass 1 (same launch ids)
    write_pass(str(root / "p2" / "p2_counter_collection.csv"), [
        (2, MARCH, {"SQ_INSTS_LDS": [20.0], "GRBM_GUI_ACTIVE": [8 * 1000.0]}),
        (3, MARCH, {"SQ_INSTS_LDS": [40.0], "GRBM_GUI_ACTIVE": [8 * 1000.0]}),
    ])
    write_pass(str(root / "p4" / "p4_counter_collection.csv"), [
        (2, MARCH, {"FETCH_SIZE": [1000.0]}), (3, MARCH, {"FETCH_SIZE": [3000.0]}),
        (9, COPY, {"FETCH_SIZE": [524288.0]}),
    ])
    write_pass(str(root / "p5" / "p5_counter_collection.csv"), [
        (2, MARCH, {"WRITE_SIZE": [10.0]}), (3, MARCH, {"WRITE_SIZE": [30.0]}),
        (9, COPY, {"WRITE_SIZE": [1048576.0]}),
    ])
    out = tmp_path / "rec.json"
    bench.counter_record("headline", str(root), 2, str(out))
    rec = json.load(open(out))
    c = rec["counters_per_launch"]
    assert c["SQ_INSTS_VALU"] == pytest.approx(200.0)
    assert c["SQ_INSTS_LDS"] == pytest.approx((20 + 40 + 20 + 40) / 4)
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["traffic_bytes_per_launch"] == pytest.approx((2000.0 * 2.0 + 20.0) * 1024.0)
    # VALU busy: instructions x 4 cycles over 1024 SIMDs x the cycles per XCD
    assert rec["valu"]["busy_frac"] == pytest.approx(200.0 * 4 / (1024 * 1000.0))
    # the record names the sources it was measured on, by hash
    assert rec["source_files"] == bench.HEADLINE_SOURCES and len(rec["source_sha256"]) == 64


def test_serving_record_sums_the_replay(tmp_path):
    root = tmp_path / "serve"
    write_pass(str(root / "FETCH_SIZE" / "run_counter_collection.csv"), [
        (1, BATCH, {"FETCH_SIZE": [100.0]}), (2, "void raypc::skip_kernel(raypc::SkipArgs)", {"FETCH_SIZE": [50.0]}),
        (3, BATCH, {"FETCH_SIZE": [200.0]}), (4, COPY, {"FETCH_SIZE": [262144.0]}),
    ])
    write_pass(str(root / "WRITE_SIZE" / "run_counter_collection.csv"), [
        (1, BATCH, {"WRITE_SIZE": [7.0]}), (3, BATCH, {"WRITE_SIZE": [3.0]}), (4, COPY, {"WRITE_SIZE": [1048576.0]}),
    ])
    out = tmp_path / "rec.json"
    bench.counter_record("serving", str(root), 2, str(out))
    rec = json.load(open(out))
    assert rec["fetch_size_kib_total"] == pytest.approx(350.0)
    assert rec["write_size_kib_total"] == pytest.approx(10.0)
    assert rec["traffic_bytes_per_launch"] == pytest.approx((350.0 * 4.0 + 10.0) * 1024.0)
