"""Host-side checks of the rocprofv3 summary helpers and of the bench line's
traffic gating (no GPU)."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1408_4675_amd import profiling as P  # noqa: E402


@pytest.mark.parametrize("name,cls", [
    ("void kw::kw_ypass<kw::EngFixed<8>, true, 512>(kw::YArgs)", "ypass_inv"),
    ("void kw::kw_ypass<kw::EngFixed<16>, false, 1024>(kw::YArgs)", "ypass_fwd"),
    # the fixed engine's second template argument is its set of radices
    ("void kw::kw_ypass<kw::EngFixed<16, 65536ull>, false, 512>(kw::YArgs)", "ypass_fwd"),
    ("void kw::kw_ypass<kw::EngFixed<8, 256ull>, true, 1024>(kw::YArgs)", "ypass_inv"),
    ("void kw::kw_ypass<kw::EngFixed<16, 0ull>, true, 512>(kw::YArgs)", "ypass_inv"),
    ("void kw::kw_zfused<kw::EngFixed<16, 65536ull>, 1, 512, false>(kw::ZArgs)", "zfused_div"),
    ("void kw::kw_xden3<kw::EngFixed<12, 80ull>, true>(kw::XArgs)", "xden"),
    ("void kw::kw_zfused<kw::EngFixed<16>, 0, 512>(kw::ZArgs)", "zfused_grad"),
    ("void kw::kw_zfused<kw::EngGeneric<16>, 1, 512>(kw::ZArgs)", "zfused_div"),
    ("void kw::kw_zfused<kw::EngFixed<8>, 5, 1024>(kw::ZArgs)", "zfused_abs"),
    ("void kw::kw_xden<kw::EngFixed<8>, true, true>(kw::XArgs)", "xden"),
    ("void kw::kw_xden3<kw::EngGeneric<16>, true>(kw::XArgs)", "xden"),
    ("void kw::kw_xeos<kw::EngFixed<4>, false, true>(kw::XArgs)", "xeos"),
    ("__amd_rocclr_copyBuffer", "copy"),
    ("some_other_kernel", None),
])
def test_kernel_class(name, cls):
    assert P.kernel_class(name) == cls


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_trace_floor_keeps_long_dispatches(tmp_path):
    head = ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    name = "void kw::kw_xden<kw::EngFixed<8>, true, true>(kw::XArgs)"
    rows = [["KERNEL_DISPATCH", name, 0, 200_000],            # 200 us: a small-grid launch
            ["KERNEL_DISPATCH", name, 0, 13_000_000],         # 13 ms
            ["KERNEL_DISPATCH", name, 0, 12_000_000]]         # 12 ms
    _write(tmp_path / "ks_kernel_trace.csv", head, rows)
    out = P.read_kernel_trace(str(tmp_path), 1000.0)
    assert len(out) == 1 and out[0]["calls"] == 2
    assert out[0]["avg_ns"] == pytest.approx(12.5e6)
    md = P.stats_markdown(str(tmp_path), "t", "cmd", min_us=1000.0)
    assert "| xden | 2 | 12500.00 |" in md


def test_traffic_scaled_by_copy_calibration(tmp_path):
    head = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    copy = "__amd_rocclr_copyBuffer"
    xv = "void kw::kw_xvel<kw::EngFixed<8>, 0>(kw::XArgs)"
    for d in ("cf", "cw", "pf", "pw"):
        os.makedirs(tmp_path / d)
    # the 1 MiB copy reads 512 KiB-units and writes 1024 (the device's scales: 2048 and 1024 B)
    _write(tmp_path / "cf" / "x_counter_collection.csv", head, [[1, copy, "FETCH_SIZE", 512]])
    _write(tmp_path / "cw" / "x_counter_collection.csv", head, [[1, copy, "WRITE_SIZE", 1024]])
    _write(tmp_path / "pf" / "x_counter_collection.csv", head,
           [[1, xv, "FETCH_SIZE", 100], [2, xv, "FETCH_SIZE", 300]])
    _write(tmp_path / "pw" / "x_counter_collection.csv", head, [[1, xv, "WRITE_SIZE", 50], [2, xv, "WRITE_SIZE", 50]])
    t = P.traffic_table(str(tmp_path / "pf"), str(tmp_path / "pw"), str(tmp_path / "cf"),
                        str(tmp_path / "cw"), 1.0)
    k = t["kernels"]["xvel"]
    assert t["fetch_scale_bytes_per_kib"] == pytest.approx(2048.0)
    assert t["write_scale_bytes_per_kib"] == pytest.approx(1024.0)
    assert k["fetch_bytes_per_launch"] == pytest.approx(200 * 2048.0)
    assert k["write_bytes_per_launch"] == pytest.approx(50 * 1024.0)
    assert k["dispatches"] == 2


def test_bench_traffic_only_for_the_profiled_grid():
    import bench
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    with open(path) as fh:
        d = json.load(fh)
    current = d.get("source_hash") == P.kernel_source_hash()
    npts = d.get("points")
    assert npts == 256 ** 3
    # a grid without a table of its own never gets another grid's bytes
    assert bench.measured_traffic("xden", 512 ** 3) is None
    got = bench.measured_traffic("xden", npts)
    if current:
        assert got == pytest.approx(d["kernels"]["xden"]["hbm_bytes_per_launch"])
    else:
        assert got is None
    # the 1024^3 table serves the 1024^3 grid only, with its own figures
    with open(os.path.join(ROOT, "profiles", "pmc_traffic_water_bowl_1024.json")) as fh:
        d2 = json.load(fh)
    assert d2.get("points") == 1024 ** 3
    got2 = bench.measured_traffic("xden", 1024 ** 3)
    if d2.get("source_hash") == P.kernel_source_hash():
        assert got2 == pytest.approx(d2["kernels"]["xden"]["hbm_bytes_per_launch"])
        assert got2 != pytest.approx(d["kernels"]["xden"]["hbm_bytes_per_launch"])
    else:
        assert got2 is None
