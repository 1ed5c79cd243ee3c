"""GPU parity at the largest single-GPU sizes, through the C-ABI.

The 96x96 grid (11.52M neurons, 11.52G synapses, lambda = 2, int8
efficacies with int64 input slots and Q = 32; the paper's grid of Table 2)
and a batch of networks with more 1024-neuron tiles than the routing grid
has blocks take paths that smaller networks do not: routing blocks that walk
several tiles, per-tile spike lists scanned over 11 250 tiles, int8 code
entries with int64 slots.  The oracle (MIRROR32, rows regenerated from
Philox) recomputes whole steps at these sizes: the first steps from the
start, and single steps re-run from the GPU's state, slots and step counter
(teacher-forced).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1902_08410_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_08410_amd import dpsnn
    dpsnn.lib()
    return dpsnn


def _compare_step_from_state(L, net, p, seed, t, what, base=0, n=None):
    """Re-run the next step of network [base, base + n) of the handle in a
    fresh oracle from the GPU's state, slots and step counter, then compare
    the step's spikes, state and slots."""
    n = net.N if n is None else n
    V, c, r = L.dpsnn_read_state(net)
    slots = L.dpsnn_read_slots(net)
    o = O.Oracle(p, seed, store_rows=False)
    o.set_state(V[base:base + n].astype(np.float64), c[base:base + n].astype(np.float64),
                r[base:base + n].astype(np.int32))
    o.set_ring(np.ascontiguousarray(slots[:, base:base + n]))
    o.set_time(t)
    del V, c, r, slots
    return o


def _check_step(L, net, o, what, base=0, n=None, k=None):
    n = net.N if n is None else n
    if k is None:
        st, ids = L.dpsnn_read_spikes(net)
    else:
        st, ids = L.dpsnn_read_spikes_net(net, k)
    ost, oids = o.spikes()
    assert len(st) == len(ost), (what, len(st), len(ost))
    assert np.array_equal(st, ost) and np.array_equal(ids, oids), what
    V, c, r = L.dpsnn_read_state(net)
    oV, oc, orr = o.state()
    assert np.array_equal(V[base:base + n].astype(np.float64), oV), what
    assert np.array_equal(c[base:base + n].astype(np.float64), oc), what
    assert np.array_equal(r[base:base + n].astype(np.int32), orr), what
    del V, c, r, oV, oc, orr
    slots = L.dpsnn_read_slots(net)
    assert np.array_equal(slots[:, base:base + n], o.ring()), what
    return len(st)


def _grid96():
    return dict(W.grid96("swa"), spike_log_cap=1 << 26, rate_bins_cap=512)


@pytest.mark.timeout(420)
def test_96x96_full_size_start_and_teacher_forced_step(L):
    """96x96 in the split schedule with appended spike lists and merged
    reservations (the delivery the autotuner picks at this size): 300
    sampled rows bit-exact, the first 4 steps bit-exact from the start
    (spikes, state, every slot), then after 1000 more steps one step re-run
    by the oracle from the GPU's state."""
    p = _grid96()
    _say("96x96 build")
    net = L.dpsnn_build(p, 1)
    st = net.stats()
    assert st["n_neurons"] == 11_520_000 and st["route_blocks"] == 4096
    assert st["queue_entry_bytes"] == 4
    L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
    L.dpsnn_set_delivery(net, 0, 2)
    orc = O.Oracle(p, 1, store_rows=False)
    rng = np.random.default_rng(5)
    d_min = p["d_min"]
    for s in sorted(rng.choice(net.N, 300, replace=False).tolist()):
        t1, w1, d1 = L.dpsnn_read_rows(net, s, 1)
        ot, od, ow, _ = orc.gen_row(s)
        order = np.lexsort((np.arange(len(ot)), od, ot))
        assert np.array_equal(t1[0], ot[order]), s
        assert np.array_equal(d1[0].astype(np.int64), od[order].astype(np.int64) - d_min), s
        q = orc.pop_of(s)
        assert np.array_equal(w1[0], orc.table(f"wq8_{q}", np.int8)[ow[order]]), s
    _say("96x96 first 4 steps")
    for t in range(4):
        L.dpsnn_step(net, 1)
        orc.step(1)
        _say("96x96 step", t)
    n0 = _check_step(L, net, orc, "96x96 start")
    assert n0 > 1000
    orc.close()
    _say("96x96 1000 steps, teacher-forced step")
    for _ in range(10):  # the start has bursts of 10^5 spikes per step
        L.dpsnn_step(net, 100)
        L.dpsnn_read_spikes(net)
    o = _compare_step_from_state(L, net, p, 1, 1004, "96x96 appended")
    L.dpsnn_step(net, 1)
    o.step(1)
    assert _check_step(L, net, o, "96x96 teacher-forced, appended lists") > 1000
    assert o.status == 0
    net.close()


@pytest.mark.timeout(420)
def test_96x96_per_tile_lists_teacher_forced_step(L):
    """The same network with per-tile spike lists (every delivery block
    scans the counts of 11 250 tiles) and 1024 delivery blocks: one step
    after 1000 steps re-run by the oracle from the GPU's state."""
    p = _grid96()
    _say("96x96 per-tile lists build")
    net = L.dpsnn_build(p, 2)
    L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
    L.dpsnn_set_delivery(net, 1024, 0)
    assert net.stats()["spike_lists"] == 0
    for _ in range(10):
        L.dpsnn_step(net, 100)
        L.dpsnn_read_spikes(net)
    o = _compare_step_from_state(L, net, p, 2, 1000, "96x96 per-tile")
    L.dpsnn_step(net, 1)
    o.step(1)
    assert _check_step(L, net, o, "96x96 teacher-forced, per-tile lists") > 1000
    net.close()


@pytest.mark.timeout(420)
def test_batch_beyond_4096_tiles_teacher_forced(L):
    """Three networks of 40x40, 36x36 and 30x30 full-size modules (binary16
    efficacies, lambda 1 and 2, adaptation swept) in one handle: 4635 tiles,
    so each of the 4096 routing blocks walks one or two tiles.  After 300
    steps, one step of every network re-run by the oracle from the GPU's
    state, read back per network."""
    plist = [W.grid(40, 40, "swa", weight_dtype="f16"),
             W.grid(36, 36, "aw", weight_dtype="f16", **{"lambda": 2.0}),
             W.grid(30, 30, "swa", weight_dtype="f16", gc=[0.0063, 0.0])]
    plist = [dict(p, spike_log_cap=1 << 24, rate_bins_cap=256) for p in plist]
    seeds = [31, 32, 33]
    _say("batch > 4096 tiles build")
    net = L.dpsnn_build_batch(plist, seeds)
    st = net.stats()
    assert st["route_blocks"] == 4096 and net.N > 4096 * 1024
    L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
    L.dpsnn_step(net, 300)
    L.dpsnn_read_spikes(net)
    orcs = []
    for k, (p, sd) in enumerate(zip(plist, seeds)):
        info = L.dpsnn_net_info(net, k)
        orcs.append((_compare_step_from_state(L, net, p, sd, 300, k, info["base"],
                                              info["n_neurons"]), info))
    L.dpsnn_step(net, 1)
    for k, (o, info) in enumerate(orcs):
        _say("batch network", k)
        o.step(1)
        assert _check_step(L, net, o, ("batch", k), info["base"], info["n_neurons"], k=k) > 50
    net.close()


@pytest.mark.timeout(420)
@pytest.mark.parametrize("wd", ["f32", "f16", "i8"])
def test_48x48_swa_aw_batch_in_the_benchmark_configuration(L, wd):
    """The benchmark's 48x48 groups: SWA and AW networks (2.88M neurons,
    2.88G synapses each) in one handle, seed 1 for both, split schedule,
    1024 delivery blocks, appended spike lists with merged reservations,
    128-step graph replays.  After 300 steps, one step of each network
    re-run by the oracle from the GPU's state, read back per network."""
    import torch
    plist = [dict(W.grid(48, 48, r, weight_dtype=wd), spike_log_cap=1 << 24, rate_bins_cap=256)
             for r in ("swa", "aw")]
    seeds = [1, 1]
    _say("48x48 batch build", wd)
    stream = torch.cuda.Stream()  # graph replay needs a stream of its own
    net = L.dpsnn_build_batch(plist, seeds, stream=stream.cuda_stream)
    L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
    L.dpsnn_set_delivery(net, 1024, 2)
    L.dpsnn_set_graph_steps(net, 128)
    st = net.stats()
    assert st["deliver_blocks"] == 1024 and st["spike_lists"] == 2 and st["queue_cap"] > 0
    L.dpsnn_step(net, 300)
    L.dpsnn_read_spikes(net)
    orcs = []
    for k, (p, sd) in enumerate(zip(plist, seeds)):
        info = L.dpsnn_net_info(net, k)
        orcs.append((_compare_step_from_state(L, net, p, sd, 300, k, info["base"],
                                              info["n_neurons"]), info))
    L.dpsnn_step(net, 1)
    for k, (o, info) in enumerate(orcs):
        _say("48x48 network", k, wd)
        o.step(1)
        assert _check_step(L, net, o, ("48x48", wd, k), info["base"], info["n_neurons"],
                           k=k) > 100
        assert o.status == 0
    net.close()


@pytest.mark.timeout(420)
def test_48x48_fbi_batch_in_the_benchmark_configuration(L):
    """The benchmark's 48x48 F/B/I group: the slow-wave state swv and the AW
    8.8 Hz state (2.88M neurons, 3.24G synapses each, three populations whose
    Eq. 2 constants form two classes) in one handle, split schedule, 1024
    delivery blocks, appended lists with one reservation per run, 128-step
    graph replays.  After 300 steps, one step of each network re-run by the
    oracle from the GPU's state."""
    import torch
    plist = [dict(W.fbi(48, 48, s, lam=0.5), spike_log_cap=1 << 24, rate_bins_cap=256)
             for s in ("swv", "aw88")]
    seeds = [1, 1]
    _say("48x48 F/B/I batch build")
    stream = torch.cuda.Stream()
    net = L.dpsnn_build_batch(plist, seeds, stream=stream.cuda_stream)
    L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
    L.dpsnn_set_delivery(net, 1024, 1)
    L.dpsnn_set_graph_steps(net, 128)
    L.dpsnn_step(net, 300)
    L.dpsnn_read_spikes(net)
    orcs = []
    for k, (p, sd) in enumerate(zip(plist, seeds)):
        info = L.dpsnn_net_info(net, k)
        orcs.append((_compare_step_from_state(L, net, p, sd, 300, k, info["base"],
                                              info["n_neurons"]), info))
    L.dpsnn_step(net, 1)
    for k, (o, info) in enumerate(orcs):
        _say("48x48 F/B/I network", k)
        o.step(1)
        assert _check_step(L, net, o, ("48x48 F/B/I", k), info["base"], info["n_neurons"],
                           k=k) > 100
        assert o.status == 0
    net.close()


@pytest.mark.timeout(420)
def test_sweep64_in_the_benchmark_configuration(L):
    """The benchmark's batched sweep: 64 networks of 4x4 to 16x16 full-size
    modules (9.54M neurons, binary16 efficacies, adaptation and lambda drawn
    per network) in one handle, split schedule, 1024 delivery blocks,
    appended lists with merged reservations, 128-step graph replays.  After
    300 steps, one step of six networks (the first, the last, and the
    largest and smallest of the rest) re-run by the oracle from the GPU's
    state."""
    import torch
    plist, seeds = W.sweep()
    plist = [dict(p, spike_log_cap=1 << 25, rate_bins_cap=256) for p in plist]
    _say("sweep64 build")
    stream = torch.cuda.Stream()
    net = L.dpsnn_build_batch(plist, seeds, stream=stream.cuda_stream)
    assert sum(L.dpsnn_net_info(net, k)["n_neurons"] for k in range(len(plist))) == 9_540_000
    L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
    L.dpsnn_set_delivery(net, 1024, 2)
    L.dpsnn_set_graph_steps(net, 128)
    for _ in range(6):  # the start has bursts: drain the log as it fills
        L.dpsnn_step(net, 50)
        L.dpsnn_read_spikes(net)
    sizes = [p["grid_w"] * p["grid_h"] for p in plist]
    mid = range(1, len(plist) - 1)
    pick = sorted({0, len(plist) - 1, max(mid, key=lambda k: sizes[k]),
                   min(mid, key=lambda k: sizes[k]), 17, 40})
    orcs = []
    for k in pick:
        info = L.dpsnn_net_info(net, k)
        orcs.append((k, _compare_step_from_state(L, net, plist[k], seeds[k], 300, k,
                                                 info["base"], info["n_neurons"]), info))
    L.dpsnn_step(net, 1)
    for k, o, info in orcs:
        _say("sweep network", k)
        o.step(1)
        assert _check_step(L, net, o, ("sweep", k), info["base"], info["n_neurons"], k=k) > 0
        assert o.status == 0
    net.close()
