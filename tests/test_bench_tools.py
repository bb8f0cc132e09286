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


def test_cpu_baseline_and_parity_of_the_many_stack_leg(bench, orc):
    """The CPU leg on two small stacks whose 'GPU results' are the oracle's own chain (one
    with its offsets moved by one float ulp): parity within tolerance with identical integer
    offsets, the ulp move counted; the extrapolated time covers every stack of the workload
    and grows with the search's FMA count."""
    import numpy as np
    import synth
    specs = [synth.small_spec(5, 96, 96, n_stars=12, shift_bound=3.0, seed=(91, 0)),
             synth.small_spec(6, 128, 128, n_stars=20, shift_bound=3.0, seed=(91, 1))]
    sample, all_offs = [], []
    for i, sp in enumerate(specs):
        st = synth.make_stack(sp)
        o = orc.reduce_stack(st.raw, st.dark, st.flat, sp.radius)
        offs = o["offsets"].copy()
        offs["sx"][0] = offs["sy"][0] = 0.0
        if i == 1:
            offs["sx"][2] = np.nextafter(np.float32(offs["sx"][2]), np.float32(np.inf))
        out = orc.shift(o["cal"], np.stack([offs["sx"], offs["sy"]], 1).astype(np.float32), o["rect"])
        img = orc.combine(out)[0].astype(np.float32)
        sample.append(dict(index=i, spec=sp, raw=st.raw, dark=st.dark, flat=st.flat, img=img, rect=o["rect"],
                           offs=offs, n_rej=o["n_rej"]))
        all_offs.append(offs)
    workload = specs + [specs[1]] * 3
    base, par = bench.cpu_baseline_many(sample, all_offs, workload, one_thread_sides=(96, 128))
    assert base["kind"] == "oracle" and base["unit"] == "Mpix/s" and base["value"] > 0
    assert base["value_1_thread"] > 0 and base["cores"] >= 1
    assert par["identical_integer_offsets"] == 1.0 and par["rects_identical"]
    assert par["frames_with_subpixel_offset_difference"] == 1
    assert par["frames_searched"] == 4 + 5 and par["frames_all_stacks"] == 4 + 5 * 4
    assert par["within_tolerance"] and par["rel_err"]["max"] <= 2e-6
    assert par["pixels_checked"] + par["threshold_band_pixels"] == sum(s["img"].size for s in sample)


def test_counter_rows_read_the_sqlite_output(bench, tmp_path):
    """rocprofv3 writes its counters to an SQLite database by default: the same rows as CSV."""
    import sqlite3
    d = tmp_path / "pmc" / "host"
    d.mkdir(parents=True)
    db = sqlite3.connect(str(d / "m_results.db"))
    db.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
               "value real)")
    db.executemany("insert into counters_collection values (?, ?, ?, ?)",
                   [(2, "rd::batch_cal(rd::BatchArgs, int)", "FETCH_SIZE", 30.0),
                    (1, "rd::batch_cal(rd::BatchArgs, int)", "FETCH_SIZE", 10.0),
                    (3, "rd::batch_cal(rd::BatchArgs, int)", "WRITE_SIZE", 99.0)])
    db.commit()
    db.close()
    rows = bench._counter_rows(str(tmp_path / "pmc"), "FETCH_SIZE")
    assert rows == [("rd::batch_cal(rd::BatchArgs, int)", 10.0), ("rd::batch_cal(rd::BatchArgs, int)", 30.0)]
