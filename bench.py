"""Benchmark: synaptic events per second on one MI355X.

Default workload (the configuration the metric is quoted on): a 24x24 grid
of modules of 1250 LIF-SFA neurons (720k neurons, 0.72G synapses,
out-degree 1000, half local, Eq. 1 remote connectivity with lambda = 1 on a
torus, delays 1-20 steps of 0.1 ms), FP32 efficacies, int32 fixed-point
input slots; one slow-wave (SWA) and one asynchronous-wake (AW) network
advance side by side.  One benchmark step = 1 s of biological time (10 000
steps of dt) of both networks.  Inputs are synthetic and seeded; the
networks are built (connectivity generated on the device) before the timed
region.

Other workloads: --workload sweep64 (64 networks of 4x4 to 16x16 modules in one
batched handle, FP16 efficacies), --workload grid96 (96x96 modules, 11.52M
neurons, int8 efficacies, int64 slots), --workload fbi24 (24x24 modules of
the foreground / background / inhibitory populations of Sec. 2.2 with the
Table S1 states, open boundaries).

Prints one JSON line.
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def bytes_per_neuron_step(p) -> float:
    """Algorithmic bytes of the neuron update: V read+write, c read+write
    (excitatory only), refractory counter read+write, input slot read+clear."""
    acc = 4 if p["acc_bits"] == 32 else 8
    exc = 4 + 4 + 4 + 4 + 1 + 1 + 2 * acc
    inh = 4 + 4 + 1 + 1 + 2 * acc
    if p.get("n_pops", 0):
        n = p["n_pops"]
        f = sum(p["pop_size"][q] for q in range(n) if p["pop_exc"][q]) / p["K"]
    else:
        f = p["frac_exc"]
    return f * exc + (1 - f) * inh


def bytes_per_event(p) -> float:
    """Algorithmic bytes of one synaptic event: target index, stored
    efficacy, read-modify-write of the target's input slot; with plasticity
    the events of excitatory sources also read and write the synapse's
    activation step and signal and read the target's last spike step."""
    acc = 4 if p["acc_bits"] == 32 else 8
    wb = {"f32": 4, "f16": 2, "i8": 1}[p["weight_dtype"]]
    b = 4 + wb + 2 * acc
    if p.get("plastic", 0):
        b += p["frac_exc"] * (4 + 4 + 4 + 4 + 4)
    return b


KERNEL_SRC = os.path.join(ROOT, "paper_1902_08410_amd", "csrc", "kernels.hip")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "k_deliver_k_neuron_grid24_traffic.json")


def kernels_sha256() -> str:
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def recorded_traffic():
    """Per-launch HBM bytes of the kernels from the committed counter runs,
    or None if the kernel source changed since they were taken."""
    try:
        rec = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    return rec if rec.get("kernels_sha256") == kernels_sha256() else None


def summarize_rocprof(kt_dir, fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, out_json):
    """Fold rocprofv3 CSV output (kernel trace/stats and FETCH_SIZE / WRITE_SIZE
    passes of this benchmark, plus the same counters for a 256 MiB copy) into
    per-launch figures: medians over the last 2000 dispatches of each kernel."""
    import csv
    import glob
    import statistics

    def one(d, pat):
        f = glob.glob(os.path.join(d, pat))
        return list(csv.DictReader(open(f[0]))) if f else []

    known_kib = 256 * 1024
    cf = [float(r["Counter_Value"]) for r in one(cal_fetch_dir, "*counter_collection.csv")
          if "copyBuffer" in r["Kernel_Name"]]
    cw = [float(r["Counter_Value"]) for r in one(cal_write_dir, "*counter_collection.csv")
          if "copyBuffer" in r["Kernel_Name"]]
    f_fetch = known_kib / statistics.mean(cf)
    f_write = known_kib / statistics.mean(cw)
    rec = {"kernels_sha256": kernels_sha256(), "fetch_scale": f_fetch, "write_scale": f_write,
           "kernels": {}}
    fe = one(fetch_dir, "*counter_collection.csv")
    wr = one(write_dir, "*counter_collection.csv")
    tr = one(kt_dir, "*kernel_trace.csv")
    for name in ("k_neuron", "k_deliver", "k_step"):
        a = [float(r["Counter_Value"]) for r in fe if name in r["Kernel_Name"]][-2000:]
        b = [float(r["Counter_Value"]) for r in wr if name in r["Kernel_Name"]][-2000:]
        d = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in tr
             if name in r["Kernel_Name"]][-4000:]
        if not a or not b:
            continue
        fetch_b = statistics.median(a) * 1024 * f_fetch
        write_b = statistics.median(b) * 1024 * f_write
        rec["kernels"][name] = {"fetch_bytes": fetch_b, "write_bytes": write_b,
                                "bytes_per_launch": fetch_b + write_b,
                                "median_duration_us": statistics.median(d) / 1e3 if d else None,
                                "dispatches": len(a)}
    json.dump(rec, open(out_json, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def cpu_baseline(params, gpu_net, dpsnn, steps: int, budget_s: float):
    """The oracle (single thread) re-running a post-transient window of the
    same workload from the GPU's state: events/s of the CPU implementation."""
    import numpy as np
    import oracle
    V, c, r = dpsnn.dpsnn_read_state(gpu_net)
    slots = dpsnn.dpsnn_read_slots(gpu_net)
    t = gpu_net.stats()["t"]
    orc = oracle.Oracle(params, gpu_net.seed, store_rows=False)
    orc.set_state(V.astype(np.float64), c.astype(np.float64), r.astype(np.int32))
    orc.set_ring(slots)
    orc.set_time(t)
    done = 0
    t0 = time.perf_counter()
    while done < steps and time.perf_counter() - t0 < budget_s:
        orc.step(1)
        done += 1
    el = time.perf_counter() - t0
    n_sp = len(orc.spikes()[0])
    return {"value": n_sp * params["K_out"] / el, "unit": "synaptic events/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{done} steps ({done * 0.1:.1f} ms biological) of the 24x24 SWA "
                       f"network from the GPU state at step {t}; {n_sp} spikes, "
                       f"{el:.1f} s; rows regenerated from Philox per spike"),
            "cpu": platform.processor() or platform.machine()}


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload(name, dpsnn, workloads, total_bins):
    """Handles of the workload: {label: (handle, params of its first net)}."""
    if name == "grid24":
        regs = {"swa": workloads.grid(24, 24, "swa"), "aw": workloads.grid(24, 24, "aw")}
    elif name == "fbi24":
        regs = {"sw": workloads.fbi(24, 24, "sw"), "aw88": workloads.fbi(24, 24, "aw88")}
    elif name == "grid96":
        regs = {"swa": workloads.grid96("swa"), "aw": workloads.grid96("aw")}
    elif name == "stdp24":
        regs = {"swa": workloads.grid(24, 24, "swa", **workloads.stdp()),
                "aw": workloads.grid(24, 24, "aw", **workloads.stdp())}
    else:
        regs = None
    nets = {}
    if regs is not None:
        for label, p in regs.items():
            p.update(spike_log_cap=0, rate_bins_cap=total_bins)
            nets[label] = (dpsnn.dpsnn_build(p, 1), p)
            progress(f"built {label}: {nets[label][0].stats()['build_ms']:.0f} ms")
    else:
        plist, seeds = workloads.sweep()
        for p in plist:
            p.update(spike_log_cap=0, rate_bins_cap=total_bins)
        nets["sweep"] = (dpsnn.dpsnn_build_batch(plist, seeds), plist[0])
        progress(f"built sweep of {len(plist)}: {nets['sweep'][0].stats()['build_ms']:.0f} ms")
    return nets


DESCRIPTIONS = {
    "grid24": ("24x24 modules x 1250 LIF-SFA neurons (720k neurons, 0.72G synapses), lambda 1, "
           "SWA + AW networks, FP32 efficacies, int32 fixed-point slots"),
    "sweep64": ("batched sweep: 64 networks of 4x4..16x16 modules (9.5M neurons, 9.5G synapses), "
           "g_c log-uniform 0.002-0.02, lambda 1 or 2, FP16 efficacies, int32 slots, "
           "one handle"),
    "grid96": ("96x96 modules x 1250 neurons (11.52M neurons, 11.52G synapses), lambda 2, "
           "SWA + AW networks, int8 efficacies with per-module scale, int64 fixed-point "
           "slots (Q = 32)"),
    "stdp24": ("24x24 modules x 1250 LIF-SFA neurons (720k neurons, 0.72G synapses), lambda 1, "
               "SWA + AW networks, FP32 efficacies, int32 slots, STDP on the synapses of "
               "excitatory sources (20 ms windows, 1 s filter and update period)"),
    "fbi24": ("24x24 modules x (250 F + 750 B + 250 I) neurons (720k neurons, 0.81G "
            "synapses, 1125 per neuron), Table S1 SW and AW 8.8 Hz states, Eq. 1 from "
            "d = 0 with lambda 0.5, open boundaries, FP32 efficacies, int32 slots"),
}
DTYPES = {"grid24": "f32", "sweep64": "f16", "grid96": "i8", "fbi24": "f32", "stdp24": "f32"}


def wave_bench(dpsnn, workloads, torch):
    """Slow-wave analysis of the 24x24 F/B/I network in the SW state
    (lambda = 0.5): 1 s of transient drained, then 3 s (600 bins of 5 ms)
    analysed in place; one JSON line with the best of five timed calls."""
    import ctypes as C
    import numpy as np
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        p = dict(workloads.fbi(24, 24, "sw", lam=0.5), rate_bins_cap=4096)
        net = dpsnn.dpsnn_build(p, 1)
        dpsnn.dpsnn_step(net, 10000)
        dpsnn.dpsnn_read_rates(net)
        dpsnn.dpsnn_step(net, 30000)
        r = dpsnn.dpsnn_waves(net, noise_var=0.5, seed=1, min_modules=50)
        progress("analysis warm")
        wp = dpsnn.DpsnnWaveParams(dpsnn.ABI_VERSION, 0, 0, 0.5, 1, 2, 2, 50, 0)
        res = dpsnn.DpsnnWaveResult()
        nt, nw = max(1, r["n_transitions"]), max(1, r["n_waves"])
        bufs = [np.zeros(nt, np.int32), np.zeros(nt), np.zeros(nt, np.int32),
                np.zeros(nw), np.zeros(nw), np.zeros(nw, np.int32)]
        ptr = [b.ctypes.data_as(C.c_void_p) for b in bufs]
        times = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc = dpsnn.lib().dpsnn_waves(net.h, C.byref(wp), C.byref(res), ptr[0], ptr[1],
                                         ptr[2], nt, ptr[3], ptr[4], ptr[5], nw)
            times.append(time.perf_counter() - t0)
            if rc != 0:
                raise dpsnn.DpsnnError("dpsnn_waves", rc)
        net.close()
    M, P = 576, 3
    print(json.dumps({
        "metric": "slow-wave analysis time (Sec. 2.3, Eq. 4), one call",
        "value": min(times) * 1e3, "unit": "ms", "higher_is_better": False,
        "n_gpus": 1, "data": "synthetic",
        "config": {"workload": "24x24 F/B/I network, SW state, lambda 0.5; 600 bins of 5 ms "
                               "(3 s after 1 s of transient), noise variance 0.5, "
                               "min_down = min_up = 2, min_modules = 50",
                   "count_bytes": int(r["n_bins"]) * M * P * 4},
        "transitions": int(res.n_transitions), "waves": int(res.n_waves),
        "mean_speed_imd_per_s": float(res.mean_speed),
        "all_calls_ms": [t * 1e3 for t in times]}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["grid24", "sweep64", "grid96", "fbi24", "stdp24"],
                    default="grid24")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 10 for grid24, fbi24 and stdp24, 2 for sweep64 and grid96)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dt-steps", type=int, default=None,
                    help="dt steps per bench step (default 10000 = 1 s; 2000 for sweep64 and grid96)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--calibrate", action="store_true",
                    help="only copy 256 MiB device-to-device three times (counter calibration)")
    ap.add_argument("--summarize-rocprof", nargs=6, metavar=("KT", "FETCH", "WRITE",
                    "CAL_FETCH", "CAL_WRITE", "OUT_JSON"),
                    help="fold rocprofv3 CSV directories into per-launch traffic figures")
    ap.add_argument("--profile-steps", type=int, default=2000,
                    help="steps timed per kernel with events for the roofline")
    ap.add_argument("--variants", type=int, default=1,
                    help="grid24: also time FP16 and int8 efficacies")
    ap.add_argument("--waves", action="store_true",
                    help="time the slow-wave analysis (Sec. 2.3, Eq. 4) of 3 s of the 24x24 "
                         "F/B/I SW network instead of the step")
    args = ap.parse_args()
    if args.summarize_rocprof:
        summarize_rocprof(*args.summarize_rocprof)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (there is no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    wl = args.workload
    small = wl in ("grid24", "fbi24", "stdp24")
    steps = args.steps if args.steps is not None else (10 if small else 2)
    S = args.dt_steps if args.dt_steps is not None else (10000 if small else 2000)
    if not small:
        args.profile_steps = min(args.profile_steps, 200)

    import torch
    from paper_1902_08410_amd import dpsnn, workloads

    if not os.path.exists(dpsnn.LIBPATH):
        from paper_1902_08410_amd import build as libbuild
        libbuild.build()
    torch.cuda.set_device(0)
    if args.calibrate:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": a.numel() * 4, "copies": 3}), flush=True)
        return
    if args.waves:
        wave_bench(dpsnn, workloads, torch)
        return
    stream = torch.cuda.Stream()        # default priority; graphs need a non-default stream
    # rate bins: warm-up and timed steps, the autotuner's two passes over
    # at most 11 candidates, the per-kernel timing steps
    tune_steps = 22 * min(1000, S // 2) if args.autotune else 0
    total_bins = ((args.warmup + steps) * S + tune_steps + args.profile_steps) // 50 + 100
    sched = {}
    variants = {}
    with torch.cuda.stream(stream):
        nets = build_workload(wl, dpsnn, workloads, total_bins)
        K_OUT = next(iter(nets.values()))[1]["K_out"]  # same for every handle
        for _ in range(args.warmup):
            for h, _ in nets.values():
                dpsnn.dpsnn_step(h, S)
        for name, (h, _) in nets.items():
            sched[name] = (dpsnn.dpsnn_autotune(h, min(1000, S // 2)) if args.autotune
                           else h.stats()["schedule"])
        torch.cuda.synchronize()
        progress("warmup done")
        sp0 = {k: h.stats()["n_spikes"] for k, (h, _) in nets.items()}
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for k in range(steps):
            for h, _ in nets.values():
                dpsnn.dpsnn_step(h, S)
            progress(f"enqueued timed step {k + 1}")
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev0.elapsed_time(ev1)
        sp1 = {k: h.stats()["n_spikes"] for k, (h, _) in nets.items()}
        progress("timed region done")
        # per-kernel times over further real steps (events around each kernel)
        prof = {}
        for name, (h, _) in nets.items():
            if args.profile_steps <= 0:
                continue
            dpsnn.dpsnn_set_schedule(h, dpsnn.SCHED_SPLIT)
            s_a = h.stats()["n_spikes"]
            upd_ms, del_ms = dpsnn.dpsnn_profile_steps(h, args.profile_steps)
            prof[name] = (upd_ms, del_ms, (h.stats()["n_spikes"] - s_a) * K_OUT)
        progress("kernel timing done")
        if wl == "grid24" and args.variants:
            for wd in ("f16", "i8"):
                for reg in ("swa", "aw"):
                    q = dict(nets[reg][1], weight_dtype=wd)
                    vn = dpsnn.dpsnn_build(q, 1)
                    dpsnn.dpsnn_step(vn, S)
                    torch.cuda.synchronize()
                    v0 = vn.stats()["n_spikes"]
                    ta = time.perf_counter()
                    dpsnn.dpsnn_step(vn, 2 * S)
                    torch.cuda.synchronize()
                    tb = time.perf_counter()
                    ev = (vn.stats()["n_spikes"] - v0) * K_OUT
                    variants[f"{wd}_{reg}"] = {"events_per_s": ev / (tb - ta),
                                               "rate_hz": ev / K_OUT / vn.N / (2 * S * 1e-4)}
                    vn.close()
                    progress(f"variant {wd} {reg} done")

    spikes = {k: sp1[k] - sp0[k] for k in nets}
    events = sum(spikes.values()) * K_OUT
    value = events / wall
    n_steps_all = steps * S * len(nets)
    p0 = next(iter(nets.values()))[1]
    Bn, Be = bytes_per_neuron_step(p0), bytes_per_event(p0)
    neurons = {k: h.stats()["n_neurons"] for k, (h, _) in nets.items()}
    sim_s = steps * S * 0.1e-3
    rates = {k: spikes[k] / neurons[k] / sim_s for k in nets}
    n_prof = max(1, args.profile_steps * len(prof))
    del_ms = sum(v[1] for v in prof.values())
    upd_ms = sum(v[0] for v in prof.values())
    prof_events = sum(v[2] for v in prof.values())
    del_us = del_ms * 1e3 / n_prof
    upd_us = upd_ms * 1e3 / n_prof
    ev_per_launch = prof_events / n_prof
    alg_del = ev_per_launch * Be
    achieved = alg_del / (del_us * 1e-6) / 1e9 if del_us > 0 else None
    n_mean = sum(neurons.values()) / len(neurons)
    # whole-step bound: every neuron-step and every event of the timed window
    # at its algorithmic bytes, over the wall time of the window
    step_bytes = sum(neurons[k] * steps * S * bytes_per_neuron_step(nets[k][1])
                     + spikes[k] * K_OUT * bytes_per_event(nets[k][1]) for k in nets)
    step_gbs = step_bytes / wall / 1e9
    traffic = None
    rec = recorded_traffic() if wl == "grid24" else None
    if rec and "k_deliver" in rec["kernels"]:
        traffic = rec["kernels"]["k_deliver"]["bytes_per_launch"]
    cpu = None
    if wl == "grid24" and not args.no_cpu_baseline:
        cpu = cpu_baseline(nets["swa"][1], nets["swa"][0], dpsnn, 400, args.cpu_budget)

    out = {
        "metric": "synaptic events/sec on 1 MI355X (SWA & AW), FP16/int8 vs FP32 weights",
        "value": value,
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[wl],
        "data": "synthetic",
        "config": {
            "workload": DESCRIPTIONS[wl],
            "bench_step": f"{S} steps of dt = 0.1 ms ({S * 1e-4:g} s biological) of every network",
            "neurons": neurons,
            "handles": list(nets),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic,
            "kernel": "k_deliver (spike delivery: one inbox reservation per target-tile run, "
                      "plus the inbox routers)",
            "bytes_per_event": Be,
            "events_per_launch": ev_per_launch,
            "algorithmic_bytes_per_launch": alg_del,
            "avg_launch_us": del_us,
            "events_per_s_in_kernel": ev_per_launch / (del_us * 1e-6) if del_us > 0 else None,
            "update_kernel": {"kernel": "k_neuron (update, with the queued-input gather)",
                              "avg_launch_us": upd_us,
                              "algorithmic_bytes_per_launch": n_mean * Bn,
                              "achieved_GB_s": n_mean * Bn / (upd_us * 1e-6) / 1e9
                              if upd_us else None,
                              "bytes_per_neuron_step": Bn},
            "step_us": gpu_ms * 1e3 / (n_steps_all / max(1, len(nets))) / max(1, len(nets)),
            "whole_step": {"algorithmic_bytes": step_bytes,
                           "achieved_GB_s": step_gbs,
                           "frac": step_gbs / HBM_PEAK_GBS,
                           "bound_events_per_s": value / (step_gbs / HBM_PEAK_GBS)},
        },
        "cpu_baseline": cpu,
        "per_handle": {k: {"spikes": spikes[k], "rate_hz": rates[k],
                           "events_per_s": spikes[k] * K_OUT / wall,
                           "build_ms": nets[k][0].stats()["build_ms"],
                           "schedule": "split" if sched[k] == 1 else "fused",
                           "deliver_blocks": nets[k][0].stats()["deliver_blocks"],
                           "spike_lists": "appended" if nets[k][0].stats()["spike_lists"]
                           else "per tile"}
                       for k in nets},
        "gpu_ms_timed": gpu_ms,
        "weight_variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
