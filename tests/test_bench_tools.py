"""Host-side measurement tooling of bench.py: the counter bytes per launch that go into
the roofline's `traffic` field (CPU only, on synthetic counter files)."""
import csv
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_tools_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _counters(folder, counter, rows):
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_scales_by_the_copy_probe_and_tells_kernels_apart(bench, tmp_path):
    copy_kib = (128 << 22) // 1024  # the copy probe moves 512 MiB each way
    _counters(tmp_path / "cf", "FETCH_SIZE", [("copy_kernel", copy_kib / 2)])  # FETCH reads half
    _counters(tmp_path / "cw", "WRITE_SIZE", [("copy_kernel", copy_kib)])
    plain = "void rd::combine_cols<16, 2, false>(float const*, long)"
    miss = "void rd::combine_cols<16, 2, true>(float const*, long)"
    _counters(tmp_path / "f", "FETCH_SIZE", [(plain, 100.0), (plain, 300.0), (miss, 50.0),
                                             ("rd::spline_rows(float const*)", 10.0),
                                             ("rd::spline_cols(float const*)", 20.0)])
    _counters(tmp_path / "w", "WRITE_SIZE", [(plain, 7.0), (plain, 9.0), (miss, 4.0),
                                             ("rd::spline_rows(float const*)", 1.0),
                                             ("rd::spline_cols(float const*)", 2.0)])
    rec = bench.traffic_from(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                             workload=1, kernels=["combine", "combine_missing", "shift_spline", "calibrate"])
    k = rec["kernels"]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    # the mean over dispatches, KiB -> bytes, scaled
    assert k["combine"]["fetch_bytes"] == round(200.0 * 1024 * 2) and k["combine"]["write_bytes"] == 8 * 1024
    assert k["combine"]["dispatches"] == 2
    assert k["combine_missing"]["fetch_bytes"] == round(50.0 * 1024 * 2)
    # a call of two kernels: their sum
    assert k["shift_spline"]["bytes"] == round((10 + 20) * 1024 * 2 + (1 + 2) * 1024)
    assert "calibrate" not in k  # no counter rows: nothing recorded
    assert all(len(v["source_sha256"]) == 64 for v in k.values())
