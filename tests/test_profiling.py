"""The counter summary: per-launch means of the run kernel's FETCH_SIZE and
WRITE_SIZE, scaled by the calibration copy (synthetic counter files)."""

import csv

import pytest

from paper_2602_23434_amd import profiling

FIELDS = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Grid_Size": 256, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": val})


COPY = "void at::native::elementwise_kernel<128, 4, direct_copy_kernel_cuda lambda>(int)"
RUNK = "void pl::k_runs<1, 2, 3, 0, 2, 1, 1>(pl::ItemDesc const*, int, int, unsigned int*, int*, unsigned int, int)"


def test_traffic_scaling(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    # the copy moves 256 MiB each way; the counters see a quarter of it
    _write(f, "FETCH_SIZE", [(COPY, 65536.0), ("pl::k_hist(int)", 5.0), (RUNK, 1000.0), (RUNK, 3000.0)])
    _write(w, "WRITE_SIZE", [(COPY, 32768.0), (RUNK, 500.0), (RUNK, 500.0)])
    t = profiling.traffic(str(f), str(w), "cmd")
    assert t["kernel"] == "pl::k_runs<1, 2, 3, 0, 2, 1, 1>"
    assert t["fetch_factor"] == pytest.approx(4.0) and t["write_factor"] == pytest.approx(8.0)
    assert t["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 4)
    assert t["write_bytes_per_launch"] == pytest.approx(500.0 * 1024 * 8)
    assert t["bytes_per_launch"] == pytest.approx(t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"])
    assert t["launches"] == 2 and t["src_digest"] == profiling.src_digest()
    assert t["config"] == profiling.workload_config()


def test_traffic_needs_the_copy(tmp_path):
    f = tmp_path / "f.csv"
    _write(f, "FETCH_SIZE", [(RUNK, 1000.0)])
    with pytest.raises(RuntimeError):
        profiling.traffic(str(f), str(f), "cmd")


def test_instruction_ceilings(tmp_path):
    f = tmp_path / "sq.csv"
    with open(f, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for name, val in (("SQ_WAVES", 2048), ("SQ_INSTS_VALU", 3.0e8), ("SQ_INSTS_LDS", 4.0e7),
                          ("SQ_LDS_BANK_CONFLICT", 1.0e8)):
            w.writerow({"Dispatch_Id": 1, "Grid_Size": 256, "Kernel_Name": RUNK, "Counter_Name": name,
                        "Counter_Value": val})
            w.writerow({"Dispatch_Id": 2, "Grid_Size": 256, "Kernel_Name": COPY, "Counter_Name": name,
                        "Counter_Value": 1.0})
    t = profiling.instructions(str(f), "cmd")
    assert t["valu_wave_insts"] == 3.0e8 and t["lds_wave_insts"] == 4.0e7
    # 3e8 wave instructions x 4 cycles over 1024 SIMDs at 2.4 GHz
    assert t["valu_floor_ms"] == pytest.approx(3.0e8 * 4 / (1024 * 2.4e9) * 1e3)
    assert t["lds_conflict_ms_per_cu"] == pytest.approx(1.0e8 / 256 / 2.4e9 * 1e3)


def _write_many(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, counter, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Grid_Size": 256, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": val})


def test_lds_occupancy_and_bandwidth(tmp_path):
    a, b, ag = tmp_path / "a.csv", tmp_path / "b.csv", tmp_path / "agent.csv"
    # 4 CUs on 2 XCDs; the launch lasts 1000 clocks (GRBM_GUI_ACTIVE summed over the XCDs)
    _write_many(a, [(RUNK, "SQ_LDS_IDX_ACTIVE", 2000.0), (RUNK, "SQ_LDS_BANK_CONFLICT", 500.0),
                    (RUNK, "GRBM_GUI_ACTIVE", 2000.0), (COPY, "SQ_LDS_IDX_ACTIVE", 7.0)])
    _write_many(b, [(RUNK, "SQ_INSTS_LDS_LOAD_BANDWIDTH", 3000.0), (RUNK, "SQ_INSTS_LDS_STORE_BANDWIDTH", 200.0),
                    (RUNK, "SQ_INSTS_LDS_ATOMIC_BANDWIDTH", 800.0), (RUNK, "GRBM_GUI_ACTIVE", 2000.0)])
    with open(ag, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Agent_Type", "Cu_Count", "Num_Xcc"])
        w.writeheader()
        w.writerow({"Agent_Type": "CPU", "Cu_Count": 16, "Num_Xcc": 1})
        w.writerow({"Agent_Type": "GPU", "Cu_Count": 4, "Num_Xcc": 2})
    t = profiling.lds(str(a), str(b), str(ag), "cmd")
    assert t["cu_count"] == 4 and t["xcc_count"] == 2 and t["launch_clocks"] == 1000.0
    assert t["lds_util"] == pytest.approx(2000.0 / (1000.0 * 4))
    assert t["bank_conflict_share_of_active"] == pytest.approx(0.25)
    assert t["lds_bytes"] == pytest.approx(4000.0 * 64)
    # 4 CUs x 128 bytes per clock x 1000 clocks
    assert t["lds_bw_frac"] == pytest.approx(4000.0 * 64 / (128 * 4 * 1000.0))
    assert t["src_digest"] == profiling.src_digest()
