"""Benchmark: synaptic events per second on one MI355X.

Workload (the configuration the metric is quoted on): a 24x24 grid of
modules of 1250 LIF-SFA neurons (720k neurons, 0.72G synapses, out-degree
1000, half local, Eq. 1 remote connectivity with lambda = 1 on a torus,
delays 1-20 steps of 0.1 ms), FP32 efficacies, int32 fixed-point input
slots; one slow-wave (SWA) and one asynchronous-wake (AW) network advance
side by side.  One benchmark step = 1 s of biological time (10 000 steps
of dt) of both networks.  Inputs are synthetic and seeded; the networks are
built (connectivity generated on the device) before the timed region.

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
K_OUT = 1000


def bytes_per_neuron_step(p) -> float:
    """Algorithmic bytes of the neuron update: V read+write, c read+write
    (excitatory only), refractory counter read+write, input slot read+clear."""
    acc = 4 if p["acc_bits"] == 32 else 8
    exc = 4 + 4 + 4 + 4 + 1 + 1 + 2 * acc
    inh = 4 + 4 + 1 + 1 + 2 * acc
    return p["frac_exc"] * exc + (1 - p["frac_exc"]) * inh


def bytes_per_event(p) -> float:
    """Algorithmic bytes of one synaptic event: target index, stored
    efficacy, read-modify-write of the target's input slot."""
    acc = 4 if p["acc_bits"] == 32 else 8
    wb = {"f32": 4, "f16": 2, "i8": 1}[p["weight_dtype"]]
    return 4 + wb + 2 * acc


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
    return {"value": n_sp * K_OUT / el, "unit": "synaptic events/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{done} steps ({done * 0.1:.1f} ms biological) of the 24x24 SWA "
                       f"network from the GPU state at step {t}; {n_sp} spikes, "
                       f"{el:.1f} s; rows regenerated from Philox per spike"),
            "cpu": platform.processor() or platform.machine()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps of 1 s biological")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dt-steps", type=int, default=10000, help="dt steps per bench step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--autotune", type=int, default=1)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1902_08410_amd import dpsnn, workloads

    if not os.path.exists(dpsnn.LIBPATH):
        from paper_1902_08410_amd import build as libbuild
        libbuild.build()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()        # default priority; graphs need a non-default stream
    S = args.dt_steps
    total_bins = (args.warmup + args.steps) * S // 50 + 200   # + autotune probes
    regimes = {"swa": workloads.grid(24, 24, "swa"), "aw": workloads.grid(24, 24, "aw")}
    nets = {}
    build_ms = {}
    sched = {}
    with torch.cuda.stream(stream):
        for name, p in regimes.items():
            p.update(spike_log_cap=0, rate_bins_cap=total_bins)
            nets[name] = dpsnn.dpsnn_build(p, 1)
            build_ms[name] = nets[name].stats()["build_ms"]
        for _ in range(args.warmup):
            for net in nets.values():
                dpsnn.dpsnn_step(net, S)
        for name, net in nets.items():
            sched[name] = dpsnn.dpsnn_autotune(net, 1000) if args.autotune else \
                net.stats()["reserved"]
        torch.cuda.synchronize()
        sp0 = {k: n.stats()["n_spikes"] for k, n in nets.items()}
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            for net in nets.values():
                dpsnn.dpsnn_step(net, S)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev0.elapsed_time(ev1)

    sp1 = {k: n.stats()["n_spikes"] for k, n in nets.items()}
    spikes = {k: sp1[k] - sp0[k] for k in nets}
    events = sum(spikes.values()) * K_OUT
    value = events / wall
    n_launch = args.steps * S * len(nets)   # steps of dt (one launch sequence each)
    N = nets["swa"].N
    p0 = regimes["swa"]
    Bn, Be = bytes_per_neuron_step(p0), bytes_per_event(p0)
    ev_per_launch = events / n_launch
    alg_bytes = N * Bn + ev_per_launch * Be
    launch_ms = gpu_ms / n_launch
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    sim_s = args.steps * S * 0.1e-3
    rates = {k: spikes[k] / N / sim_s for k in nets}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(regimes["swa"], nets["swa"], dpsnn, 400, args.cpu_budget)

    out = {
        "metric": "synaptic events/sec on 1 MI355X (SWA & AW), FP16/int8 vs FP32 weights",
        "value": value,
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("24x24 modules x 1250 LIF-SFA neurons (720k neurons, 0.72G "
                         "synapses), lambda 1, SWA + AW networks, FP32 efficacies, "
                         "int32 fixed-point slots"),
            "bench_step": f"{S} steps of dt = 0.1 ms (1 s biological) of each network",
            "neurons_per_network": N,
            "networks": list(nets),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "one step of dt (k_neuron + k_deliver, or fused k_step)",
            "bytes_per_neuron_step": Bn,
            "bytes_per_event": Be,
            "avg_launch_us": launch_ms * 1e3,
            "events_per_launch": ev_per_launch,
        },
        "cpu_baseline": cpu,
        "per_regime": {k: {"spikes": spikes[k], "rate_hz": rates[k],
                           "events_per_s": spikes[k] * K_OUT / wall,
                           "build_ms": build_ms[k]} for k in nets},
        "gpu_ms_timed": gpu_ms,
        "schedule": {k: ("split" if v == 1 else "fused") for k, v in sched.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
