"""Host logic of bench.py's profiler summaries (CPU): kernel names to
(kernel, weight format), the pairing of update launches with the delivery
launch after them, the event-timed window, and the counter calibration."""
import csv
import json
import os

import pytest

import bench


def test_kernel_group_names():
    g = bench._kernel_group
    assert g("void dpsnn::k_deliver<int, 0, false, true>(dpsnn::StepArgs, dpsnn::StepOff)") == \
        ("k_deliver", "f32")
    assert g("dpsnn::k_deliver<long, 2, false, false>(x)") == ("k_deliver", "i8")
    assert g("dpsnn::k_step<int, 1, 2>(x)") == ("k_step", "f16")
    assert g("dpsnn::k_persist<long, 2, 2, 2>(x)") == ("k_persist", "i8")
    assert g("dpsnn::k_neuron<int, 2, 1>(x)") == ("k_neuron", None)
    assert g("dpsnn::k_gen<0>(x)") is None
    assert g("__amd_rocclr_copyBuffer") is None


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_ALL)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_rocprof_windows_and_scales(tmp_path, monkeypatch):
    """Two weight formats timed one after the other: each format's window
    is its own last N dispatches, update launches take the format of the
    delivery launch after them, dispatch ids order the rows (the CSV is
    shuffled), and the copy calibration scales the counters."""
    names = {"f32": ("dpsnn::k_neuron<int, 2, 1>(a)", "dpsnn::k_deliver<int, 0, false, true>(a)"),
             "f16": ("dpsnn::k_neuron<int, 2, 2>(a)", "dpsnn::k_deliver<int, 1, false, true>(a)")}
    trace, fetch, write = [], [], []
    did = 0
    for fmt, base in (("f32", 100), ("f16", 200)):
        for k in range(6):       # 6 steps; the window below is the last 4
            for kern, dur in ((0, base + k), (1, 2 * base + k)):
                did += 1
                trace.append([did, names[fmt][kern], 1000 * did, 1000 * did + dur * 1000])
                fetch.append([did, names[fmt][kern], "FETCH_SIZE", 10.0 * (kern + 1) + k])
                write.append([did, names[fmt][kern], "WRITE_SIZE", 5.0 * (kern + 1)])
    trace.reverse()
    d = str(tmp_path)
    _write(f"{d}/kt/x_kernel_trace.csv",
           ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _write(f"{d}/fe/x_counter_collection.csv", hdr, fetch[::-1])
    _write(f"{d}/wr/x_counter_collection.csv", hdr, write)
    _write(f"{d}/cf/x_counter_collection.csv", hdr, [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE",
                                                      256 * 1024 / 2]])
    _write(f"{d}/cw/x_counter_collection.csv", hdr, [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE",
                                                      256 * 1024]])
    monkeypatch.setattr(bench, "PROFILES", d)
    bench.summarize_rocprof(f"{d}/kt", f"{d}/fe", f"{d}/wr", f"{d}/cf", f"{d}/cw", "wl", 4)
    for fmt, base in (("f32", 100), ("f16", 200)):
        rec = json.load(open(os.path.join(d, f"k_deliver_k_neuron_wl_{fmt}_traffic.json")))
        assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == 1.0
        kn, kd = rec["kernels"]["k_neuron"], rec["kernels"]["k_deliver"]
        # steps 2..5 of the format: durations base + k and 2 base + k
        assert kn["mean_duration_us"] == pytest.approx(base + 3.5)
        assert kd["mean_duration_us"] == pytest.approx(2 * base + 3.5)
        assert kn["trace_dispatches"] == kd["counter_dispatches"] == 4
        # FETCH 10 (kern + 1) + k KiB, doubled by the calibration; WRITE 5 (kern + 1)
        assert kn["fetch_bytes"] == pytest.approx(2 * (10 + 3.5) * 1024)
        assert kd["write_bytes"] == pytest.approx(10 * 1024)
        assert kd["bytes_per_launch"] == pytest.approx(2 * (20 + 3.5) * 1024 + 10 * 1024)


def test_onset_speeds_planted_plane_wave():
    """A plane wave planted in rate bins: Up states of 300 ms that start at
    t0 + x / v at module column x (two 5 ms bins per module), four events
    2 s apart, 24x24 modules, background noise.  The onset estimate gives
    back v, and every event reaches every module."""
    import numpy as np
    w = h = 24
    v = 100.0                                    # inter-module distances per second
    bins = 1800
    counts = np.zeros((bins, w * h, 3), np.int32)
    rng = np.random.default_rng(3)
    counts[:, :, 1] = rng.integers(0, 3, size=(bins, w * h))
    for ev in range(4):
        t0 = 1.0 + 2.0 * ev
        for y in range(h):
            for x in range(w):
                b0 = int(round((t0 + x / v) / 5e-3))
                counts[b0:b0 + 60, y * w + x, 1] += 40
    events, full, speeds = bench.onset_speeds(counts, w, h, 5.0)
    assert events == 4 and full == 4
    assert np.allclose(speeds, v, rtol=0.02)


def test_onset_speeds_diagonal_wave_scales_by_sqrt2():
    """A wave front moving along the diagonal with the delay 1 / v per
    module in x and in y (one bin): |grad T| = sqrt(2) / v, the speed
    v / sqrt(2)."""
    import numpy as np
    w = h = 24
    v = 200.0
    bins = 1000
    counts = np.zeros((bins, w * h, 3), np.int32)
    for ev in range(2):
        t0 = 0.5 + 2.0 * ev
        for y in range(h):
            for x in range(w):
                b0 = int(round((t0 + (x + y) / v) / 5e-3))
                counts[b0:b0 + 60, y * w + x, 0] += 30
    counts[:, :, 2] += 1
    events, full, speeds = bench.onset_speeds(counts, w, h, 5.0)
    assert events == 2 and full == 2
    assert np.allclose(speeds, v / np.sqrt(2), rtol=0.02)
