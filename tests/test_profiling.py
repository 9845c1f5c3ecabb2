"""Host logic of the profile summaries: calibrated traffic from FETCH_SIZE / WRITE_SIZE and the
request-size byte count, on hand-written counter CSV files (no GPU, no profiler)."""
import csv
import os

import pytest

from paper_2501_07465_amd import profiling

FIELDS = ["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size", "Workgroup_Size", "VGPR_Count",
          "LDS_Block_Size"]


def _write(dirpath, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v, "Grid_Size": 1,
                        "Workgroup_Size": 1, "VGPR_Count": 1, "LDS_Block_Size": 0})


def test_traffic_scales_by_the_soa_copy(tmp_path):
    mib = 256.0
    kib = mib * 1024
    calib = [("at::MulFunctor<float>", kib / 2), ("pic::k_measure_soa_copy(...)", kib / 2)]
    _write(tmp_path / "f", [(k, "FETCH_SIZE", v) for k, v in calib * 3] + [("pic::k_particles<3>", "FETCH_SIZE", 1000.0)] * 4)
    _write(tmp_path / "w", [(k, "WRITE_SIZE", kib) for k, _ in calib * 3] + [("pic::k_particles<3>", "WRITE_SIZE", 300.0)] * 4)
    r = profiling.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_particles", mib)
    assert r["dispatches"] == 4
    assert r["soa_fetch_factor"] == pytest.approx(2.0) and r["soa_write_factor"] == pytest.approx(1.0)
    assert r["fetch_bytes"] == pytest.approx(2000.0 * 1024) and r["write_bytes"] == pytest.approx(300.0 * 1024)
    assert r["traffic_bytes"] == pytest.approx(2300.0 * 1024)


def test_traffic_refuses_disagreeing_calibration_dispatches(tmp_path):
    kib = 256.0 * 1024
    rows = [("at::MulFunctor<float>", kib / 2), ("at::MulFunctor<float>", kib / 4),
            ("pic::k_measure_soa_copy(...)", kib / 2)]
    _write(tmp_path / "f", [(k, "FETCH_SIZE", v) for k, v in rows] + [("pic::k_fields<3>", "FETCH_SIZE", 1.0)])
    _write(tmp_path / "w", [(k, "WRITE_SIZE", kib) for k, _ in rows] + [("pic::k_fields<3>", "WRITE_SIZE", 1.0)])
    with pytest.raises(ValueError):
        profiling.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_fields", 256.0)


def test_request_bytes_price_each_size(tmp_path):
    rd = []
    for k, n32, n64, n128 in (("pic::k_measure_soa_copy(...)", 0, 0, 2 ** 21), ("pic::k_fields<3>", 10, 20, 30)):
        rd += [(k, "TCC_EA0_RDREQ_sum", n32 + n64 + n128), (k, "TCC_EA0_RDREQ_32B_sum", n32),
               (k, "TCC_EA0_RDREQ_64B_sum", n64), (k, "TCC_EA0_RDREQ_128B_sum", n128)]
    wr = [("pic::k_measure_soa_copy(...)", "TCC_EA0_WRREQ_sum", 2 ** 22), ("pic::k_measure_soa_copy(...)", "TCC_EA0_WRREQ_64B_sum", 2 ** 22),
          ("pic::k_fields<3>", "TCC_EA0_WRREQ_sum", 7), ("pic::k_fields<3>", "TCC_EA0_WRREQ_64B_sum", 3)]
    _write(tmp_path / "rd", rd)
    _write(tmp_path / "wr", wr)
    r = profiling.request_bytes(str(tmp_path / "rd"), str(tmp_path / "wr"), ["k_measure_soa_copy", "k_fields"])
    # 2^21 requests of 128 B read and 2^22 of 64 B written: a 256 MiB copy, no factor
    assert r["k_measure_soa_copy"]["read_bytes"] == 256 * 2 ** 20
    assert r["k_measure_soa_copy"]["write_bytes"] == 256 * 2 ** 20
    f = r["k_fields"]
    assert f["read_bytes"] == 32 * 10 + 64 * 20 + 128 * 30
    assert f["write_bytes"] == 32 * 4 + 64 * 3
    assert f["share_128B"] == pytest.approx(0.5) and f["sized_fraction"] == pytest.approx(1.0)
