"""Benchmark: synaptic events per second on one MI355X.

Default workload (the configuration the metric is quoted on): a 48x48 grid
of modules of 1250 LIF-SFA neurons (2.88M neurons, 2.88G synapses,
out-degree 1000, half local, Eq. 1 remote connectivity with lambda = 1 on a
torus, delays 1-20 steps of 0.1 ms), int32 fixed-point input slots; one
slow-wave (SWA) and one asynchronous-wake (AW) network advance side by side,
with binary32 efficacies (the headline value), then with binary16 and with
int8 efficacies (per source population scale), each weight format timed
with the same protocol (warm-up, autotune, HIP-graph replay, event-timed
kernels).  One benchmark step = 4000 steps of dt (0.4 s of biological time)
of both networks.  Inputs are synthetic and seeded; the networks are built
(connectivity generated on the device) before the timed region.

Other workloads: --workload grid24 (24x24 modules, FP32), sweep64 (64
networks of 4x4 to 16x16 modules in one batched handle, FP16 efficacies),
grid96 (96x96 modules, 11.52M neurons, int8 efficacies, int64 slots), fbi24
(24x24 modules of the foreground / background / inhibitory populations of
Sec. 2.2 with the Table S1 states, open boundaries), stdp24 (24x24 with
plasticity).  --lambda sets the decay length of the grid workloads.

Prints one JSON line.
"""
import argparse
import json
import os
import platform
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
PROFILES = os.path.join(ROOT, "profiles")
EXT_TRAINS = 400  # external Poisson trains per neuron of the paper's model (Table S1)


def traffic_json(workload: str, wdt: str) -> str:
    return os.path.join(PROFILES, f"k_deliver_k_neuron_{workload}_{wdt}_traffic.json")


def kernels_sha256() -> str:
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def recorded_traffic(workload: str, wdt: str):
    """Per-launch HBM bytes of the kernels from the committed counter runs of
    this workload and weight format, or None if the kernel source changed
    since they were taken."""
    try:
        rec = json.load(open(traffic_json(workload, wdt)))
    except (OSError, ValueError):
        return None
    return rec if rec.get("kernels_sha256") == kernels_sha256() else None


WDT_NAMES = {0: "f32", 1: "f16", 2: "i8"}


def _kernel_group(name: str):
    """(kernel, weight format) of a traced step-kernel instantiation, e.g.
    'dpsnn::k_deliver<int, 0, false>(...)' -> ('k_deliver', 'f32'); None for
    other kernels.  k_deliver and k_step take the weight format as their
    second template argument; k_neuron takes the entry format instead, so
    its group is assigned from the k_deliver launches around it."""
    base = name.split("(")[0].replace("void ", "")
    for k in ("k_deliver", "k_neuron", "k_step", "k_persist"):
        if base.startswith(f"dpsnn::{k}<"):
            args = base[len(f"dpsnn::{k}<"):].rstrip(">").split(",")
            if k == "k_neuron":
                return k, None
            return k, WDT_NAMES.get(int(args[1])) if len(args) > 1 else None
    return None


def summarize_rocprof(kt_dir, fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, workload,
                      window):
    """Fold rocprofv3 CSV output (a kernel trace of the benchmark command,
    FETCH_SIZE / WRITE_SIZE passes, and the same counters for a 256 MiB copy)
    into per-launch figures of each weight format's kernels over the window
    the benchmark times them in: the last `window` dispatches of each kernel
    of that format (the event-timed steps; one dispatch per step and batched
    handle).  Writes k_deliver_k_neuron_<workload>_<format>_traffic.json
    under profiles/ for every format present."""
    import csv
    import glob
    import statistics

    def one(d, pat):
        f = glob.glob(os.path.join(d, "**", pat), recursive=True)
        return list(csv.DictReader(open(f[0]))) if f else []

    def by_group(rows, value):
        """{(kernel, format): [values in dispatch order]}; a k_neuron launch
        takes the format of the next k_deliver / k_step launch."""
        out, pend = {}, []
        for r in rows:
            g = _kernel_group(r["Kernel_Name"])
            if g is None:
                continue
            if g[0] == "k_neuron":
                pend.append(value(r))
                continue
            out.setdefault(g, []).append(value(r))
            if pend:
                out.setdefault(("k_neuron", g[1]), []).extend(pend)
                pend = []
        return out

    window = int(window)
    known_kib = 256 * 1024
    cf = [float(r["Counter_Value"]) for r in one(cal_fetch_dir, "*counter_collection.csv")
          if "copyBuffer" in r["Kernel_Name"]]
    cw = [float(r["Counter_Value"]) for r in one(cal_write_dir, "*counter_collection.csv")
          if "copyBuffer" in r["Kernel_Name"]]
    f_fetch = known_kib / statistics.mean(cf)
    f_write = known_kib / statistics.mean(cw)
    def ordered(rows):
        return sorted(rows, key=lambda r: int(r.get("Dispatch_Id") or 0))

    cval = lambda r: float(r["Counter_Value"])
    fe = by_group(ordered(one(fetch_dir, "*counter_collection.csv")), cval)
    wr = by_group(ordered(one(write_dir, "*counter_collection.csv")), cval)
    tr = by_group(ordered(one(kt_dir, "*kernel_trace.csv")),
                  lambda r: int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    recs = {}
    for (k, wdt), a in fe.items():
        b = wr.get((k, wdt), [])
        d = tr.get((k, wdt), [])[-window:]
        a = a[-window:]
        b = b[-window:]
        if not a or not b or wdt is None:
            continue
        rec = recs.setdefault(wdt, {"kernels_sha256": kernels_sha256(), "workload": workload,
                                    "fetch_scale": f_fetch, "write_scale": f_write,
                                    "window_dispatches": window, "kernels": {}})
        fetch_b = statistics.mean(a) * 1024 * f_fetch
        write_b = statistics.mean(b) * 1024 * f_write
        rec["kernels"][k] = {
            "fetch_bytes": fetch_b, "write_bytes": write_b, "bytes_per_launch": fetch_b + write_b,
            "median_bytes_per_launch": (statistics.median(a) * f_fetch +
                                        statistics.median(b) * f_write) * 1024,
            "mean_duration_us": statistics.mean(d) / 1e3 if d else None,
            "median_duration_us": statistics.median(d) / 1e3 if d else None,
            "trace_dispatches": len(d), "counter_dispatches": len(a)}
    for wdt, rec in recs.items():
        json.dump(rec, open(traffic_json(workload, wdt), "w"), indent=1)
    print(json.dumps(recs, indent=1))


def summarize_counters(dirs, out_json):
    """Medians per kernel of every counter of rocprofv3 --pmc passes (one
    directory per pass) over the last 2000 dispatches of each kernel."""
    import csv
    import glob
    import statistics
    rows = []
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += sorted(csv.DictReader(open(f)), key=lambda r: int(r.get("Dispatch_Id") or 0))
    out = {"kernels_sha256": kernels_sha256(), "kernels": {}}
    for name in ("k_neuron", "k_deliver", "k_step", "k_persist"):
        sel = [r for r in rows if name in r["Kernel_Name"]]
        if not sel:
            continue
        by = {}
        for r in sel:
            by.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        out["kernels"][name] = {c: statistics.median(v[-2000:]) for c, v in sorted(by.items())}
    json.dump(out, open(out_json, "w"), indent=1)
    print(json.dumps(out, indent=1))


def host_cpu():
    """CPU model and the number of host threads this process may use."""
    model = platform.processor() or platform.machine()
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return model, nproc


def cpu_baseline(params, seed, gpu_net, k, dpsnn, workloads, label: str, steps: int,
                 budget_s: float):
    """The oracle, single-threaded, (1) re-running a post-transient window of
    network k of the benchmark handle from the GPU's state (rows regenerated
    from Philox per spike), bounded by budget_s; (2) the whole 2x2
    correctness network (5000 neurons, 2 s).  Events/s of the plain CPU
    implementation: a reported baseline, not the target.  The handle is only
    read (its queued inputs are moved into the slots), so no step kernel runs
    after the timed and profiled steps."""
    import numpy as np
    import oracle
    info = dpsnn.dpsnn_net_info(gpu_net, k)
    b, n = info["base"], info["n_neurons"]
    V, c, r = dpsnn.dpsnn_read_state(gpu_net)
    slots = dpsnn.dpsnn_read_slots(gpu_net)
    t = gpu_net.stats()["t"]
    orc = oracle.Oracle(params, seed, store_rows=False)
    orc.set_state(V[b:b + n].astype(np.float64), c[b:b + n].astype(np.float64),
                  r[b:b + n].astype(np.int32))
    orc.set_ring(np.ascontiguousarray(slots[:, b:b + n]))
    orc.set_time(t)
    del V, c, r, slots
    done = 0
    t0 = time.perf_counter()
    while done < steps and time.perf_counter() - t0 < budget_s:
        orc.step(1)
        done += 1
    el = time.perf_counter() - t0
    n_sp = len(orc.spikes()[0])
    orc.close()
    p1 = workloads.swa()
    o1 = oracle.Oracle(p1, 1, store_rows=True)
    t1 = time.perf_counter()
    o1.step(20000)
    el1 = time.perf_counter() - t1
    n1 = len(o1.spikes()[0])
    o1.close()
    model, nproc = host_cpu()
    return {"value": n_sp * params["K_out"] / el, "unit": "synaptic events/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{done} steps ({done * 0.1:.1f} ms biological) of the {label} "
                       f"network from the GPU state at step {t}; {n_sp} spikes, {el:.1f} s; "
                       "rows regenerated from Philox per spike; single thread"),
            "c1_2x2_2s": {"value": n1 * p1["K_out"] / el1, "spikes": n1, "seconds": el1,
                          "sample": "the whole 2x2 network (5000 neurons) for 2 s "
                                    "(20000 steps), stored rows, single thread"},
            "cpu_model": model, "nproc": nproc}


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload_groups(name, workloads, lam, weights):
    """Groups of networks timed together: {group: {label: params}}.  grid48
    has one group per weight format (each an SWA and an AW network)."""
    if name == "grid48":
        return {wd: {"swa": workloads.grid(48, 48, "swa", weight_dtype=wd, **{"lambda": lam}),
                     "aw": workloads.grid(48, 48, "aw", weight_dtype=wd, **{"lambda": lam})}
                for wd in weights}
    if name == "grid24":
        return {"f32": {"swa": workloads.grid(24, 24, "swa", **{"lambda": lam}),
                        "aw": workloads.grid(24, 24, "aw", **{"lambda": lam})}}
    if name == "fbi24":
        return {"f32": {"sw": workloads.fbi(24, 24, "sw"), "aw88": workloads.fbi(24, 24, "aw88")}}
    if name == "fbi48":
        return {wd: {"swv": workloads.fbi(48, 48, "swv", weight_dtype=wd, lam=lam),
                     "aw88": workloads.fbi(48, 48, "aw88", weight_dtype=wd, lam=lam)}
                for wd in weights}
    if name == "grid96":
        return {"i8": {"swa": workloads.grid96("swa"), "aw": workloads.grid96("aw")}}
    if name == "stdp24":
        return {"f32": {"swa": workloads.grid(24, 24, "swa", **workloads.stdp()),
                        "aw": workloads.grid(24, 24, "aw", **workloads.stdp())}}
    return {"f16": {"sweep": None}}


DESCRIPTIONS = {
    "grid48": ("48x48 modules x 1250 LIF-SFA neurons (2.88M neurons, 2.88G synapses), lambda "
               "{lam:g}, SWA + AW networks, FP32 efficacies (headline) and FP16 / int8 "
               "(per source population scale) efficacies timed alike, int32 fixed-point slots"),
    "grid24": ("24x24 modules x 1250 LIF-SFA neurons (720k neurons, 0.72G synapses), lambda "
               "{lam:g}, SWA + AW networks, FP32 efficacies, int32 fixed-point slots"),
    "sweep64": ("batched sweep: 64 networks of 4x4..16x16 modules (9.5M neurons, 9.5G synapses), "
                "g_c log-uniform 0.002-0.02, lambda 1 or 2, FP16 efficacies, int32 slots, "
                "one handle"),
    "grid96": ("96x96 modules x 1250 neurons (11.52M neurons, 11.52G synapses), lambda 2, "
               "SWA + AW networks, int8 efficacies with per-module scale, int64 fixed-point "
               "slots (Q = 32)"),
    "stdp24": ("24x24 modules x 1250 LIF-SFA neurons (720k neurons, 0.72G synapses), lambda 1, "
               "SWA + AW networks, FP32 efficacies, int32 slots, STDP on the synapses of "
               "excitatory sources (20 ms windows, 1 s filter and update period)"),
    "fbi48": ("48x48 modules x (250 F + 750 B + 250 I) neurons (2.88M neurons, 3.24G "
              "synapses, 1125 per neuron), the slow-wave state (swv: Up states of 0.35 s "
              "travelling across the grid at 0.35 Hz) and Table S1's AW 8.8 Hz state, Eq. 1 "
              "from d = 0 with lambda {lam:g}, open boundaries, FP32 (headline), FP16 and "
              "int8 efficacies timed alike, int32 slots"),
    "fbi24": ("24x24 modules x (250 F + 750 B + 250 I) neurons (720k neurons, 0.81G "
              "synapses, 1125 per neuron), Table S1 SW and AW 8.8 Hz states, Eq. 1 from "
              "d = 0 with lambda 0.5, open boundaries, FP32 efficacies, int32 slots"),
}


def build_group(name, group, dpsnn, workloads, total_bins, batched):
    """Handles of one group: {handle label: (handle, [params], [network labels])}.
    batched: the group's networks share one handle (one set of launches per
    step for all of them); else one handle per network."""
    nets = {}
    if name == "sweep64":
        plist, seeds = workloads.sweep()
        for p in plist:
            p.update(spike_log_cap=0, rate_bins_cap=total_bins)
        h = dpsnn.dpsnn_build_batch(plist, seeds)
        nets["sweep"] = (h, plist, [f"net{k}" for k in range(len(plist))])
        progress(f"built sweep of {len(plist)}: {h.stats()['build_ms']:.0f} ms")
        return nets
    for p in group.values():
        p.update(spike_log_cap=0, rate_bins_cap=total_bins)
    if batched and len(group) > 1:
        labels, plist = list(group), list(group.values())
        h = dpsnn.dpsnn_build_batch(plist, [1] * len(plist))
        nets["+".join(labels)] = (h, plist, labels)
        progress(f"built {'+'.join(labels)} ({plist[0]['weight_dtype']}) in one handle: "
                 f"{h.stats()['build_ms']:.0f} ms")
        return nets
    for label, p in group.items():
        h = dpsnn.dpsnn_build(p, 1)
        nets[label] = (h, [p], [label])
        progress(f"built {label} ({p['weight_dtype']}): {h.stats()['build_ms']:.0f} ms")
    return nets


def _net_spikes(dpsnn, h, n_nets):
    """Spikes of each network of a handle since its rate bins were last
    drained (the completed 5 ms bins)."""
    return [int(dpsnn.dpsnn_read_rates_net(h, k).sum()) for k in range(n_nets)]


def time_group(nets, dpsnn, torch, stream, args, steps, S):
    """The timing protocol, the same for every group: warm-up bench steps,
    autotune, the timed bench steps (graph replay on a non-default stream,
    bracketed by synchronisation and HIP events), then further real steps
    with HIP events around each kernel for the roofline."""
    sched = {}
    if args.graph_steps is not None:
        for h, _, _ in nets.values():
            dpsnn.dpsnn_set_graph_steps(h, args.graph_steps)
    for _ in range(args.warmup):
        for h, _, _ in nets.values():
            dpsnn.dpsnn_step(h, S)
    for name, (h, _, _) in nets.items():
        if not args.autotune and args.delivery:
            # a fixed launch configuration (as an autotuned run chose it),
            # for profiler passes that cannot run the autotuner
            sc, b, li = args.delivery.split(":")
            dpsnn.dpsnn_set_schedule(h, {"split": dpsnn.SCHED_SPLIT, "fused": dpsnn.SCHED_FUSED}[sc])
            dpsnn.dpsnn_set_delivery(h, int(b), int(li))
        sched[name] = (dpsnn.dpsnn_autotune(h, min(1000, S // 2)) if args.autotune
                       else h.stats()["schedule"])
    torch.cuda.synchronize()
    sp0 = {k: h.stats()["n_spikes"] for k, (h, _, _) in nets.items()}
    for h, pl, _ in nets.values():   # rate bins before the window
        _net_spikes(dpsnn, h, len(pl))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(steps):
        for h, _, _ in nets.values():
            dpsnn.dpsnn_step(h, S)
        progress(f"enqueued timed step {k + 1}")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    sp1 = {k: h.stats()["n_spikes"] for k, (h, _, _) in nets.items()}
    per_net = {k: _net_spikes(dpsnn, h, len(pl)) for k, (h, pl, _) in nets.items()}
    prof = {}
    bracket = event_bracket_us(torch, stream) if args.profile_steps > 0 else None
    for name, (h, pl, _) in nets.items():
        if args.profile_steps <= 0:
            continue
        dpsnn.dpsnn_set_schedule(h, dpsnn.SCHED_SPLIT)
        k_out = pl[0]["K_out"]
        s_a = h.stats()["n_spikes"]
        upd_ms, del_ms = dpsnn.dpsnn_profile_steps(h, args.profile_steps)
        prof[name] = (upd_ms, del_ms, (h.stats()["n_spikes"] - s_a) * k_out)
    return {"sched": sched, "spikes": {k: sp1[k] - sp0[k] for k in nets}, "per_net": per_net,
            "wall": wall, "gpu_ms": gpu_ms, "prof": prof, "bracket_us": bracket}


def event_bracket_us(torch, stream, n: int = 200) -> float:
    """What a pair of HIP events around one launch adds to the launch's own
    duration: the median interval of event pairs around a one-element
    kernel on the same stream (its dispatch and completion, plus the tiny
    kernel itself)."""
    import statistics
    x = torch.zeros(1, device="cuda")
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(n)]
    with torch.cuda.stream(stream):
        # a busy GPU while the pairs are enqueued, so that the intervals hold
        # no host-side submission gaps (as in the per-kernel timing steps,
        # whose launches queue up behind long kernels)
        torch.cuda._sleep(50_000_000)
        for a, b in pairs:
            a.record(stream)
            x.add_(1.0)
            b.record(stream)
    torch.cuda.synchronize()
    return statistics.median(a.elapsed_time(b) for a, b in pairs) * 1e3


def group_record(workload, wdt, nets, res, steps, S, args):
    """Throughput, rates and rooflines of one timed group."""
    from paper_1902_08410_amd import dpsnn
    K_OUT = next(iter(nets.values()))[1][0]["K_out"]
    spikes, wall, prof = res["spikes"], res["wall"], res["prof"]
    events = sum(spikes.values()) * K_OUT
    p0 = next(iter(nets.values()))[1][0]
    Bn, Be = bytes_per_neuron_step(p0), bytes_per_event(p0)
    stream_b = 4 + {"f32": 4, "f16": 2, "i8": 1}[p0["weight_dtype"]]
    sim_s = steps * S * 0.1e-3
    n_prof = max(1, args.profile_steps * len(prof))
    del_us = sum(v[1] for v in prof.values()) * 1e3 / n_prof
    upd_us = sum(v[0] for v in prof.values()) * 1e3 / n_prof
    ev_per_launch = sum(v[2] for v in prof.values()) / n_prof
    alg_del = ev_per_launch * Be
    achieved = alg_del / (del_us * 1e-6) / 1e9 if del_us > 0 else None
    handle_neurons = {k: h.stats()["n_neurons"] for k, (h, _, _) in nets.items()}
    n_mean = sum(handle_neurons.values()) / len(handle_neurons)
    # whole-step bound: every neuron-step and every event of the timed window
    # at its algorithmic bytes, over the wall time of the window
    step_bytes = 0.0
    per_net = {}
    for k, (h, pl, labels) in nets.items():
        for j, (p, lab) in enumerate(zip(pl, labels)):
            n = dpsnn.dpsnn_net_info(h, j)["n_neurons"]
            sp = res["per_net"][k][j]
            step_bytes += n * steps * S * bytes_per_neuron_step(p) + sp * K_OUT * bytes_per_event(p)
            if len(pl) <= 8:
                per_net[lab] = {"spikes": sp, "rate_hz": sp / n / sim_s,
                                "events_per_s": sp * K_OUT / wall}
    step_gbs = step_bytes / wall / 1e9
    rec = recorded_traffic(workload, wdt)
    rk = rec["kernels"] if rec else {}
    traffic = rk["k_deliver"]["bytes_per_launch"] if "k_deliver" in rk else None
    # the committed kernel trace of this command: mean duration over the same window
    trace_us = rk["k_deliver"].get("mean_duration_us") if "k_deliver" in rk else None
    value = events / wall
    return {
        "events_per_s": value,
        "ms_per_step": wall * 1e3 / steps,
        "paper_equivalent_events_per_s": sum(spikes.values()) * (K_OUT + EXT_TRAINS) / wall,
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
            "event_bracket_us": res["bracket_us"],
            "profile_avg_launch_us": trace_us,
            "events_per_s_in_kernel": ev_per_launch / (del_us * 1e-6) if del_us > 0 else None,
            # the synapse stream alone (target word and stored efficacy per event)
            "synapse_stream": {"bytes_per_event": stream_b,
                               "achieved_GB_s": ev_per_launch * stream_b / (del_us * 1e-6) / 1e9
                               if del_us > 0 else None},
            "update_kernel": {"kernel": "k_neuron (update, with the queued-input gather)",
                              "avg_launch_us": upd_us,
                              "algorithmic_bytes_per_launch": n_mean * Bn,
                              "achieved_GB_s": n_mean * Bn / (upd_us * 1e-6) / 1e9
                              if upd_us else None,
                              "bytes_per_neuron_step": Bn,
                              "traffic": rk["k_neuron"]["bytes_per_launch"]
                              if "k_neuron" in rk else None,
                              "profile_avg_launch_us": rk["k_neuron"].get("mean_duration_us")
                              if "k_neuron" in rk else None},
            "step_us": res["gpu_ms"] * 1e3 / (steps * S * len(nets)),
            "whole_step": {"algorithmic_bytes": step_bytes,
                           "achieved_GB_s": step_gbs,
                           "frac": step_gbs / HBM_PEAK_GBS,
                           "bound_events_per_s": value / (step_gbs / HBM_PEAK_GBS)},
        },
        "per_network": per_net,
        "handles": {k: {"networks": labels,
                        "neurons": h.stats()["n_neurons"],
                        "build_ms": h.stats()["build_ms"],
                        "bytes_per_synapse": h.stats()["bytes_total"] /
                        max(1, h.stats()["n_synapses"]),
                        "schedule": {0: "fused", 1: "split", 2: "persistent"}[res["sched"][k]],
                        "deliver_blocks": h.stats()["deliver_blocks"],
                        "spike_lists": {0: "per tile", 1: "appended",
                                        2: "appended, merged reservations"}[
                            h.stats()["spike_lists"]],
                        # the same launches without the autotuner: --autotune 0 --delivery
                        "delivery": "{}:{}:{}".format(
                            {0: "fused", 1: "split", 2: "split"}[res["sched"][k]],
                            h.stats()["deliver_blocks"], h.stats()["spike_lists"])}
                    for k, (h, _, labels) in nets.items()},
        "gpu_ms_timed": res["gpu_ms"],
    }


def _module_onsets(mua, hold=10):
    """Up onsets of each module, in bins: the MUA smoothed over 3 bins
    crossing upward the midpoint of its 10th and 90th percentiles and staying
    above it for `hold` bins, the crossing placed by linear interpolation."""
    import numpy as np
    out = []
    for m in range(mua.shape[1]):
        x = np.convolve(mua[:, m], np.ones(3) / 3, mode="same")
        lo, hi = np.percentile(x, [10, 90])
        th = 0.5 * (lo + hi)
        above = x > th
        on, b = [], 1
        while b < len(x) - hold:
            if above[b] and not above[b - 1] and above[b:b + hold].all():
                on.append(b - 1 + (th - x[b - 1]) / (x[b] - x[b - 1]))
                b += hold
            else:
                b += 1
        out.append(np.array(on))
    return out


def onset_speeds(counts, w, h, bin_ms, window_bins=40, full=0.868):
    """Second estimate of the wave speed from the rate bins alone: the Up
    onsets of the grid total define the events; each module's onset nearest
    to an event (within window_bins) gives its passage time T; an event that
    reaches at least `full` of the modules gives the median over interior
    modules of 1/|grad T| (central differences, inter-module distances per
    second).  Returns (events, full events, median speed per full event)."""
    import numpy as np
    mua = counts.sum(axis=2).astype(np.float64)
    per = _module_onsets(mua)
    events = _module_onsets(mua.sum(axis=1)[:, None])[0]
    speeds, n_full = [], 0
    for g in events:
        T = np.full(w * h, np.nan)
        for m, o in enumerate(per):
            if len(o):
                k = int(np.argmin(np.abs(o - g)))
                if abs(o[k] - g) < window_bins:
                    T[m] = o[k]
        if np.count_nonzero(~np.isnan(T)) < full * w * h:
            continue
        n_full += 1
        Tg = T.reshape(h, w) * bin_ms * 1e-3
        gx = 0.5 * (Tg[1:-1, 2:] - Tg[1:-1, :-2])
        gy = 0.5 * (Tg[2:, 1:-1] - Tg[:-2, 1:-1])
        gn = np.hypot(gx, gy)
        v = 1.0 / gn[np.isfinite(gn) & (gn > 0)]
        if len(v):
            speeds.append(float(np.median(v)))
    return len(events), n_full, speeds


def wave_speed(dpsnn, workloads, torch):
    """Speed of the slow waves of the F/B/I swv state against the decay
    length lambda of Eq. 1 (Sec. 3.3.2): 24x24 modules, 1 s of transient
    drained, then 20 s analysed in place by dpsnn_waves (Eq. 4 averaged over
    the modules of each wave, waves of at least 50 modules, dwell 4 bins),
    without added noise and with the noise of variance 0.5, and from the
    modules' own onsets (onset_speeds).  One JSON line."""
    import numpy as np
    lams, seeds = (0.4, 0.5, 0.6, 0.7), (1, 2, 3, 4)
    rows = []
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for lam in lams:
            for seed in seeds:
                p = dict(workloads.fbi(24, 24, "swv", lam=lam), rate_bins_cap=4200)
                net = dpsnn.dpsnn_build(p, seed)
                dpsnn.dpsnn_step(net, 10000)
                dpsnn.dpsnn_read_rates(net)
                dpsnn.dpsnn_step(net, 200000)
                row = {"lambda": lam, "seed": seed}
                for nv in (0.0, 0.5):
                    r = dpsnn.dpsnn_waves(net, noise_var=nv, seed=1, min_down=4, min_up=4,
                                          min_modules=50)
                    row[f"eq4_noise{nv:g}"] = {
                        "transitions": int(r["n_transitions"]),
                        "waves": int((r["speed"] > 0).sum()) if r["n_waves"] else 0,
                        "mean_speed": round(float(r["mean_speed"]), 1)}
                counts = dpsnn.dpsnn_read_rates(net)
                net.close()
                ev, full, sp = onset_speeds(counts, 24, 24, 5.0)
                row["onsets"] = {"events": ev, "full_events": full,
                                 "median_speed": round(float(np.median(sp)), 1) if sp else None}
                rows.append(row)
                progress(f"lambda {lam} seed {seed}: Eq. 4 {row['eq4_noise0']['mean_speed']} "
                         f"imd/s, onsets {row['onsets']['median_speed']} imd/s")

    def mean_of(key, sub):
        out = {}
        for lam in lams:
            v = [r[key][sub] for r in rows if r["lambda"] == lam and r[key][sub] is not None]
            out[f"{lam:g}"] = round(float(np.mean(v)), 1) if v else None
        return out
    print(json.dumps({"metric": "slow-wave speed against lambda (Sec. 3.3.2, Eq. 4)",
                      "unit": "inter-module distances per second", "n_gpus": 1,
                      "data": "synthetic",
                      "config": {"workload": "24x24 modules x (250 F + 750 B + 250 I) neurons, "
                                             "swv state, lambda 0.4-0.7, seeds 1-4, 20 s "
                                             "after 1 s of transient, FP32 efficacies"},
                      "eq4_noise0": mean_of("eq4_noise0", "mean_speed"),
                      "eq4_noise0.5": mean_of("eq4_noise0.5", "mean_speed"),
                      "onsets": mean_of("onsets", "median_speed"), "runs": rows}), flush=True)


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
    ap.add_argument("--workload", choices=["grid48", "grid24", "sweep64", "grid96", "fbi24",
                                           "fbi48", "stdp24"], default="grid48")
    ap.add_argument("--lambda", dest="lam", type=float, default=None,
                    help="decay length of Eq. 1 for grid48, grid24 (default 1) and fbi48 "
                         "(default 0.5)")
    ap.add_argument("--weights", default="f32,f16,i8",
                    help="grid48: weight formats timed, the first one is the headline")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 10; 2 for sweep64 and grid96)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dt-steps", type=int, default=None,
                    help="dt steps per bench step (default 4000 for grid48, 10000 for the "
                         "24x24 workloads, 2000 for sweep64 and grid96)")
    ap.add_argument("--separate", action="store_true",
                    help="one handle per network (default: the SWA and AW networks of a "
                         "group in one batched handle)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--graph-steps", type=int, default=None,
                    help="steps per captured HIP graph (0: direct launches, as profiler "
                         "counter passes need); default: the library's")
    ap.add_argument("--delivery", default=None, metavar="SCHED:BLOCKS:LISTS",
                    help="with --autotune 0: schedule (split or fused), delivery blocks "
                         "and spike-list kind of every handle, e.g. split:1024:2")
    ap.add_argument("--calibrate", action="store_true",
                    help="only copy 256 MiB device-to-device three times (counter calibration)")
    ap.add_argument("--summarize-rocprof", nargs=7, metavar=("KT", "FETCH", "WRITE", "CAL_FETCH",
                                                           "CAL_WRITE", "WORKLOAD", "WINDOW"),
                    help="fold rocprofv3 output into profiles/*_traffic.json")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="medians per kernel of --pmc passes: DIR... OUT_JSON")
    ap.add_argument("--profile-steps", type=int, default=2000,
                    help="steps timed per kernel with events for the roofline")
    ap.add_argument("--waves", action="store_true",
                    help="time the slow-wave analysis (Sec. 2.3, Eq. 4) of 3 s of the 24x24 "
                         "F/B/I SW network instead of the step")
    ap.add_argument("--wave-speed", action="store_true",
                    help="slow-wave speed against lambda (Sec. 3.3.2): the 24x24 F/B/I swv "
                         "state, lambda 0.4-0.7, seeds 1-4, 20 s each, analysed by "
                         "dpsnn_waves")
    args = ap.parse_args()
    if args.summarize_rocprof:
        summarize_rocprof(*args.summarize_rocprof)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[:-1], args.summarize_counters[-1])
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (there is no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    wl = args.workload
    if args.lam is None:
        args.lam = 0.5 if wl == "fbi48" else 1.0
    big = wl in ("sweep64", "grid96")
    steps = args.steps if args.steps is not None else (2 if big else 10)
    S = args.dt_steps if args.dt_steps is not None else (
        2000 if big else 4000 if wl in ("grid48", "fbi48") else 10000)
    if big:
        args.profile_steps = min(args.profile_steps, 200)
    weights = [w for w in args.weights.split(",") if w]

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
    if args.wave_speed:
        wave_speed(dpsnn, workloads, torch)
        return
    stream = torch.cuda.Stream()        # default priority; graphs need a non-default stream
    # rate bins: warm-up and timed steps, the autotuner's two passes over
    # at most 17 candidates, the per-kernel timing steps
    tune_steps = 34 * min(1000, S // 2) if args.autotune else 0
    total_bins = ((args.warmup + steps) * S + tune_steps + args.profile_steps) // 50 + 100
    groups = workload_groups(wl, workloads, args.lam, weights)
    records = {}
    cpu = None
    with torch.cuda.stream(stream):
        for gi, (gname, group) in enumerate(groups.items()):
            nets = build_group(wl, group, dpsnn, workloads, total_bins, not args.separate)
            res = time_group(nets, dpsnn, torch, stream, args, steps, S)
            records[gname] = group_record(wl, gname, nets, res, steps, S, args)
            progress(f"group {gname} timed: {records[gname]['events_per_s']:.3e} events/s")
            if gi == 0 and not args.no_cpu_baseline and wl in ("grid48", "grid24"):
                h, pl, labels = next(iter(nets.values()))
                p = pl[0]
                cpu = cpu_baseline(p, 1, h, 0, dpsnn, workloads,
                                   f"{p['grid_w']}x{p['grid_h']} {labels[0].upper()}", 200,
                                   args.cpu_budget)
                progress("cpu baseline done")
            for h, _, _ in nets.values():
                h.close()
            del nets
            torch.cuda.synchronize()

    head_name = next(iter(records))
    head = records[head_name]
    out = {
        "metric": "synaptic events/sec on 1 MI355X (SWA & AW), FP16/int8 vs FP32 weights",
        "value": head["events_per_s"],
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head_name,
        "data": "synthetic",
        "config": {
            "workload": DESCRIPTIONS[wl].format(lam=args.lam),
            "bench_step": f"{S} steps of dt = 0.1 ms ({S * 1e-4:g} s biological) of every "
                          "network of the headline group" + ("" if args.separate else
                                                             ", advanced in one batched handle"),
            "events": "recurrent synaptic events = K_out x spikes, counted on the device",
            "handles": head["handles"],
        },
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "paper_equivalent_events_per_s": head["paper_equivalent_events_per_s"],
        "paper_equivalent_events": f"spikes x (K_out + {EXT_TRAINS} external trains "
                                   "of the paper's model), labelled as such",
        "per_network": head["per_network"],
        "gpu_ms_timed": head["gpu_ms_timed"],
        "weight_variants": {k: v for k, v in records.items() if k != head_name},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
