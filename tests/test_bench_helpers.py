"""Host-side checks of bench.py's contract helpers (no GPU): the multi-GPU
refusal, the calibrated byte counts of the traffic summary, and that a traffic
figure is reported only for the kernel sources it was measured on."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for d, name, value in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


def test_traffic_summary_is_calibrated_by_the_copy(tmp_path, monkeypatch):
    # the copy (last dispatch) moves CALIB_BYTES; FETCH_SIZE reports half of it
    calib_kib = bench.CALIB_BYTES / 1024
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    # counters are summed over the instances of one dispatch
    _counter_csv(fetch, "FETCH_SIZE", [(1, "vup::k_propagate_runs(vup::SweepArgs)", 1000.0),
                                       (1, "vup::k_propagate_runs(vup::SweepArgs)", 1000.0),
                                       (2, "vup::(anonymous namespace)::k_mt_main(vup::(anonymous namespace)::MTArgs)", 500.0),
                                       (3, "__amd_rocclr_copyBuffer", calib_kib / 2)])
    _counter_csv(write, "WRITE_SIZE", [(1, "vup::k_propagate_runs(vup::SweepArgs)", 300.0),
                                       (2, "vup::(anonymous namespace)::k_mt_main(vup::(anonymous namespace)::MTArgs)", 7.0),
                                       (3, "__amd_rocclr_copyBuffer", calib_kib)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "paper_1908_11246_amd" / "csrc")
    for name in ("k_sweep.hip", "k_mtiles.hip", "k_grid.hip", "vup_device.hpp",
                 "vup_internal.hpp", "k_fields.hip", "vup_fields.hpp"):
        (tmp_path / "paper_1908_11246_amd" / "csrc" / name).write_text("// " + name)
    bench.summarize_traffic(str(fetch), str(write))
    rec = json.loads((tmp_path / "profiles" / "traffic_grid1024.json").read_text())
    assert rec["fetch_size_calibration"]["scale"] == pytest.approx(2.0)
    assert rec["write_size_calibration"]["scale"] == pytest.approx(1.0)
    p = rec["kernels"]["propagate"]
    assert p["fetch_bytes"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert p["write_bytes"] == pytest.approx(300.0 * 1024)
    assert bench.traffic_bytes("moments") == pytest.approx(500.0 * 1024 * 2.0 + 7.0 * 1024)
    # a change of a kernel source voids the figures of the kernels built from it
    assert bench.traffic_bytes("propagate") is not None
    (tmp_path / "paper_1908_11246_amd" / "csrc" / "k_sweep.hip").write_text("// changed")
    assert bench.traffic_bytes("moments") is not None
    assert bench.traffic_bytes("propagate") is None
    (tmp_path / "paper_1908_11246_amd" / "csrc" / "vup_internal.hpp").write_text("// changed")
    assert bench.traffic_bytes("moments") is None


def test_runs_in_windows_counts_bin_changes():
    """The run count behind the bench's LDS rates: per window row, one run plus
    one per change of bin inside the window, summed over rows and windows
    (brute force from the bins), with empty windows counting 0."""
    import numpy as np
    rng = np.random.default_rng(5)
    rows, n, pitch = 37, 53, 56
    bins = np.cumsum(rng.integers(0, 2, size=(rows, n)), axis=1) // 2  # runs of 1-4 cells
    runidx = np.zeros((rows, pitch), dtype=np.int16)
    runidx[:, :n] = np.concatenate([np.zeros((rows, 1), np.int64),
                                    np.cumsum(bins[:, 1:] != bins[:, :-1], axis=1)], axis=1)
    win = np.zeros((40, 2, 2), dtype=np.int32)
    for k in range(40):
        r = np.sort(rng.integers(0, rows, 2))
        c = np.sort(rng.integers(0, n, 2))
        win[k] = [r, c]
    win[3] = [[5, 4], [0, 10]]  # empty
    brute = 0
    for k in range(40):
        (r0, r1), (c0, c1) = win[k]
        for r in range(r0, r1 + 1):
            if c1 >= c0:
                brute += 1 + int((bins[r, c0 + 1:c1 + 1] != bins[r, c0:c1]).sum())
    assert bench.runs_in_windows(runidx.reshape(-1), rows, pitch, win) == brute
