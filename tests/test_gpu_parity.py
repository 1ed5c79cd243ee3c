"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

The binary32-weight path must reproduce the oracle's MIRROR32 spike rasters,
neuron state and fixed-point input slots bit for bit; the binary16 and int8
paths are bit-exact against the oracle run with the same stored formats.
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


def _pair(p, seed, store_rows=True, **over):
    from paper_1902_08410_amd import dpsnn
    q = dict(p)
    q.setdefault("spike_log_cap", 1 << 22)
    q.setdefault("rate_bins_cap", 4096)
    q.update(over)
    net = dpsnn.dpsnn_build(q, seed)
    orc = O.Oracle(q, seed, store_rows=store_rows)
    return net, orc


def _compare_rows(L, net, orc, rows, wd):
    """Rows on the device are sorted by (target, delay, draw index); the
    oracle's are sorted by delay in draw order.  The same order is taken from
    the oracle's row by a stable sort, then targets, delays and stored
    efficacies (from the table of the synapse's source population and
    block) must agree bit for bit."""
    tgt, w, dk = L.dpsnn_read_rows(net, rows[0], len(rows)) if len(rows) and \
        rows == list(range(rows[0], rows[0] + len(rows))) else (None, None, None)
    stem = {"f32": ("wt32", np.float32), "f16": ("wt16", np.uint16), "i8": ("wq8", np.int8)}[wd]
    P = orc.P
    tabs = {}
    d_min = int(orc.params["d_min"])
    for k, s in enumerate(rows):
        if tgt is None:
            t1, w1, d1 = L.dpsnn_read_rows(net, s, 1)
            t1, w1, d1 = t1[0], w1[0], d1[0]
        else:
            t1, w1, d1 = tgt[k], w[k], dk[k]
        ot, od, ow, oo, ob = orc.gen_row_blocks(s)
        order = np.lexsort((np.arange(len(ot)), od, ot))
        q = orc.pop_of(s)
        assert np.array_equal(t1, ot[order]), s
        assert np.array_equal(d1.astype(np.int64), od[order].astype(np.int64) - d_min), s
        want = np.empty(len(ot), stem[1])
        for b in np.unique(ob):
            if (q, b) not in tabs:
                tabs[(q, b)] = orc.table(f"{stem[0]}_{q}_{b}", stem[1])
            sel = ob == b
            want[sel] = tabs[(q, b)][ow[sel]]
        assert w1.tobytes() == want[order].tobytes(), s
        assert np.all(np.diff(t1.astype(np.int64)) >= 0), s
        assert P in (2, 3, 4)


@pytest.mark.parametrize("case", ["2x2_f32", "tiny_f16", "tiny_i8", "ragged_3x3",
                                  "odd_7x5", "delays64", "single_delay", "open_6x3"])
def test_rows_bitwise_equal(L, case):
    p = {"2x2_f32": W.swa(),
         "tiny_f16": W.tiny(w=3, h=2, K=40, K_out=30, weight_dtype="f16"),
         "tiny_i8": W.tiny(w=2, h=3, K=40, K_out=30, weight_dtype="i8"),
         "ragged_3x3": W.tiny(w=3, h=3, K=47, K_out=37, d_max=11),
         "odd_7x5": W.grid(7, 5, "swa", K=60, K_out=130, **{"lambda": 1.7}),
         "delays64": W.tiny(w=2, h=2, K=50, K_out=300, d_min=1, d_max=64),
         "single_delay": W.tiny(w=2, h=2, K=50, K_out=40, d_min=3, d_max=3),
         "open_6x3": W.grid(6, 3, "aw", K=50, K_out=90, torus=0, **{"lambda": 1.3})}[case]
    _say("rows", case)
    net, orc = _pair(p, 7, store_rows=False)
    rows = list(range(net.N)) if net.N <= 5000 else list(range(0, net.N, 3))
    _compare_rows(L, net, orc, list(range(net.N)) if net.N <= 5000 else rows,
                  p["weight_dtype"])
    net.close()


def test_initial_state_equal(L):
    _say("initial state 2x2")
    net, orc = _pair(W.swa(), 3, store_rows=False)
    V, c, r = L.dpsnn_read_state(net)
    oV, oc, orr = orc.state()
    assert np.array_equal(V.astype(np.float64), oV)
    assert np.all(c == 0) and np.all(r == 0)
    net.close()


def _compare_state(L, net, orc, what=""):
    V, c, r = L.dpsnn_read_state(net)
    oV, oc, orr = orc.state()
    assert np.array_equal(V.astype(np.float64), oV), what
    assert np.array_equal(c.astype(np.float64), oc), what
    assert np.array_equal(r.astype(np.int32), orr), what


def _new_oracle_spikes(orc):
    """Oracle spikes emitted since the previous call (the GPU log drains)."""
    st, ids = orc.spikes()
    k = getattr(orc, "_seen", 0)
    orc._seen = len(st)
    return st[k:], ids[k:]


def _compare_all(L, net, orc, what=""):
    st, ids = L.dpsnn_read_spikes(net)
    ost, oids = _new_oracle_spikes(orc)
    assert len(st) == len(ost), (what, len(st), len(ost))
    assert np.array_equal(st, ost) and np.array_equal(ids, oids), what
    _compare_state(L, net, orc, what)
    assert np.array_equal(L.dpsnn_read_slots(net), orc.ring()), what
    return len(st)


def test_uncoupled_trace_bit_exact(L):
    p = W.tiny(w=2, h=2, K=300, K_out=0, nu_ext_hz=[3000.0, 2500.0],
               Jext_mean=[1.0, 1.2], Jext_sd=[0.4, 0.3])
    _say("uncoupled", p["K"])
    net, orc = _pair(p, 11)
    total = 0
    for k in range(10):
        L.dpsnn_step(net, 200)
        orc.step(200)
        _compare_state(L, net, orc, k)
    st, ids = L.dpsnn_read_spikes(net)
    ost, oids = orc.spikes()
    assert np.array_equal(st, ost) and np.array_equal(ids, oids)
    assert len(st) > 100
    net.close()


RASTER_CASES = {
    "tiny_f32_acc32": W.tiny(w=3, h=3, K=60, K_out=50, nu_ext_hz=[3500.0, 3500.0]),
    "tiny_f16_acc32": W.tiny(w=2, h=3, K=60, K_out=50, weight_dtype="f16",
                             nu_ext_hz=[3500.0, 3500.0]),
    "tiny_i8_acc32": W.tiny(w=3, h=2, K=60, K_out=50, weight_dtype="i8",
                            nu_ext_hz=[3500.0, 3500.0]),
    "tiny_f32_acc64": W.tiny(w=2, h=2, K=70, K_out=60, acc_bits=64, q_frac_bits=32,
                             nu_ext_hz=[3500.0, 3500.0]),
    "tiny_i8_acc64": W.tiny(w=3, h=3, K=50, K_out=40, weight_dtype="i8", acc_bits=64,
                            q_frac_bits=32, nu_ext_hz=[3500.0, 3500.0]),
    "mid_f32_local_only_1x1": W.tiny(w=1, h=1, K=900, K_out=100, frac_local=[1.0, 1.0],
                                     nu_ext_hz=[1200.0, 1200.0]),
    "mid_f32_strong_adapt": W.tiny(w=2, h=2, K=500, K_out=200, tau_c=[5.0, 5.0],
                                   gc=[0.5, 0.0], alpha_c=[3.0, 0.0],
                                   nu_ext_hz=[3000.0, 3000.0]),
    "const_drive": W.tiny(w=2, h=2, K=30, K_out=20, I_const=[1.3, 2.1],
                          nu_ext_hz=[0.0, 0.0]),
    "open_edges_f32": W.tiny(w=4, h=3, K=60, K_out=50, torus=0, nu_ext_hz=[3500.0, 3500.0]),
}


@pytest.mark.parametrize("sched", [0, 1])
@pytest.mark.parametrize("case", sorted(RASTER_CASES))
def test_raster_bit_exact(L, case, sched):
    p = RASTER_CASES[case]
    _say("raster", case, "schedule", sched)
    net, orc = _pair(p, 5)
    L.dpsnn_set_schedule(net, sched)
    n = 0
    for k in range(4):
        L.dpsnn_step(net, 500)
        orc.step(500)
        n += _compare_all(L, net, orc, (case, k))
    assert n > 50
    assert np.array_equal(L.dpsnn_read_rates(net), orc.rates()[: 2000 // p["rate_bin_steps"]])
    assert orc.status == 0
    net.close()


@pytest.mark.parametrize("sched", [0, 1, 2])
def test_degenerate_networks_bit_exact(L, sched):
    """Edge cases of the step: a network that never fires (no external drive,
    no constant current: empty spike lists, nothing delivered, every bin
    zero, the leak alone moving the state), and the smallest network, one
    module of 5 neurons (4 excitatory, 1 inhibitory) with 4 local synapses
    each, driven hard (ragged tile, runs of one event)."""
    cases = {"silent": (W.tiny(w=2, h=2, K=30, K_out=20, nu_ext_hz=[0.0, 0.0]), False),
             "minimal_1x1": (W.tiny(w=1, h=1, K=5, K_out=4, frac_local=[1.0, 1.0],
                                    nu_ext_hz=[6000.0, 6000.0]), True)}
    for case, (p, fires) in cases.items():
        _say("degenerate", case, "schedule", sched)
        net, orc = _pair(p, 3)
        L.dpsnn_set_schedule(net, sched)
        n = 0
        for k, steps in enumerate((1, 127, 900, 972)):
            L.dpsnn_step(net, steps)
            orc.step(steps)
            n += _compare_all(L, net, orc, (case, k))
        rates = L.dpsnn_read_rates(net)
        assert np.array_equal(rates, orc.rates()[: 2000 // p["rate_bin_steps"]])
        assert (n > 100) == fires and (rates.sum() > 0) == fires, (case, n)
        assert orc.status == 0
        net.close()


def test_raster_bit_exact_2x2_two_seconds(L):
    """2x2 grid of 1250-neuron modules (5000 neurons), FP32 weights, SWA, 2 s =
    20000 steps."""
    _say("2x2 2 s")
    net, orc = _pair(W.swa(), 1)
    total = 0
    for k in range(4):
        L.dpsnn_step(net, 5000)
        orc.step(5000)
        total += _compare_all(L, net, orc, k)
    assert total > 10000
    st = net.stats()
    assert st["n_spikes"] == total and st["n_events"] == total * 1000
    net.close()


def test_24x24_full_size_start_and_teacher_forced_step(L):
    """24x24 grid at full size (720k neurons, 0.72G synapses) in the
    benchmark's launch configuration: sampled rows, the first 30 steps
    bit-exact, then after 2000 more steps one step re-run by the oracle from
    the GPU's state, slots and time."""
    p = W.grid(24, 24, "swa")
    _say("24x24 build")
    net, orc = _pair(p, 1, store_rows=False)
    rng = np.random.default_rng(0)
    rows = sorted(rng.choice(net.N, 300, replace=False).tolist())
    _compare_rows(L, net, orc, rows, "f32")
    _say("24x24 first 30 steps")
    L.dpsnn_step(net, 30)
    orc.step(30)
    _compare_all(L, net, orc, "24x24 start")
    _say("24x24 2000 steps + teacher forced step")
    L.dpsnn_step(net, 2000)
    L.dpsnn_read_spikes(net)
    V, c, r = L.dpsnn_read_state(net)
    slots = L.dpsnn_read_slots(net)
    orc2 = O.Oracle(p, 1, store_rows=False)
    orc2.set_state(V.astype(np.float64), c.astype(np.float64), r.astype(np.int32))
    orc2.set_ring(slots)
    orc2.set_time(2030)
    L.dpsnn_step(net, 1)
    orc2.step(1)
    st, ids = L.dpsnn_read_spikes(net)
    ost, oids = _new_oracle_spikes(orc2)
    assert np.array_equal(st, ost) and np.array_equal(ids, oids)
    assert len(st) > 0
    _compare_state(L, net, orc2, "teacher forced")
    assert np.array_equal(L.dpsnn_read_slots(net), orc2.ring())
    net.close()


def test_rerun_and_chunking_identical(L):
    p = W.tiny(w=3, h=3, K=80, K_out=60, nu_ext_hz=[3000.0, 3000.0])
    _say("determinism")
    from paper_1902_08410_amd import dpsnn
    a = dpsnn.dpsnn_build(dict(p, rate_bins_cap=64), 9)
    b = dpsnn.dpsnn_build(dict(p, rate_bins_cap=64), 9)
    dpsnn.dpsnn_step(a, 1000)
    for _ in range(10):
        dpsnn.dpsnn_step(b, 100)
    sa, sb = dpsnn.dpsnn_read_spikes(a), dpsnn.dpsnn_read_spikes(b)
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    assert np.array_equal(dpsnn.dpsnn_read_slots(a), dpsnn.dpsnn_read_slots(b))
    a.close()
    b.close()


def test_error_paths(L):
    from paper_1902_08410_amd import dpsnn
    p = W.tiny(w=2, h=2, K=40, K_out=20, nu_ext_hz=[5000.0, 5000.0])
    _say("errors")
    net = dpsnn.dpsnn_build(dict(p, rate_bins_cap=2, spike_log_cap=10), 1)
    with pytest.raises(dpsnn.DpsnnError) as e:
        dpsnn.dpsnn_step(net, 101)              # needs 3 bins of 50 steps
    assert e.value.code == -7
    dpsnn.dpsnn_step(net, 100)
    assert dpsnn.dpsnn_sync(net) == -5          # more than 10 spikes
    with pytest.raises(dpsnn.DpsnnError) as e:
        dpsnn.dpsnn_read_spikes(net)
    assert e.value.code == -5
    assert dpsnn.dpsnn_read_rates(net).shape[0] == 2
    dpsnn.dpsnn_step(net, 100)                  # bins drained: room again
    with pytest.raises(dpsnn.DpsnnError) as e:
        dpsnn.dpsnn_step(net, -1)
    assert e.value.code == -1
    net.close()


def test_graph_replay_and_schedule_switching(L):
    """Steps replayed from captured HIP graphs on a non-default stream, with
    the schedule switched between chunks, stay bit-exact."""
    import torch
    p = W.tiny(w=3, h=3, K=120, K_out=90, nu_ext_hz=[3000.0, 3000.0])
    _say("graphs + schedule switching")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        net, orc = _pair(p, 13)
        L.dpsnn_set_graph_steps(net, 64)
        total = 0
        for k, (sched, n) in enumerate([(1, 300), (0, 257), (1, 64), (0, 1), (1, 700),
                                        (0, 130), (0, 128)]):
            L.dpsnn_set_schedule(net, sched)
            L.dpsnn_step(net, n)
            orc.step(n)
            total += _compare_all(L, net, orc, ("chunk", k, sched))
        assert total > 200
        t0 = net.stats()["t"]
        chosen = L.dpsnn_autotune(net, 200)
        st = net.stats()
        assert chosen in (0, 1) and st["schedule"] == chosen
        # runs of 64 steps (the graph length): one untimed run and 200 // 64
        # timed ones per candidate (the fused schedule; split delivery grids
        # with both spike-list kinds)
        assert (st["t"] - t0) % (4 * 64) == 0 and st["t"] - t0 >= 2 * 4 * 64
        assert st["deliver_blocks"] in (256, 512, 1024, 2048)
        orc.step(st["t"] - t0)
        _compare_all(L, net, orc, "after autotune")
        L.dpsnn_step(net, 300)               # the tuned grid, replayed from graphs
        orc.step(300)
        _compare_all(L, net, orc, "tuned")
        net.close()


def test_2x2_graph_stream_two_seconds(L):
    """2x2 grid of 1250-neuron modules for 2 s on a non-default stream with
    graph replay."""
    import torch
    _say("2x2 graphs")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        net, orc = _pair(W.swa(), 2)
        for sched in (1, 0):
            L.dpsnn_set_schedule(net, sched)
            for k in range(2):
                L.dpsnn_step(net, 5000)
                orc.step(5000)
                _compare_all(L, net, orc, (sched, k))
        net.close()


BATCH = [
    (W.tiny(w=2, h=2, K=60, K_out=40, nu_ext_hz=[3500.0, 3500.0]), 101),
    (W.tiny(w=3, h=2, K=60, K_out=40, gc=[0.002, 0.0], nu_ext_hz=[4000.0, 3000.0],
            **{"lambda": 2.0}), 202),
    (W.tiny(w=1, h=3, K=50, K_out=40, tau_c=[300.0, 300.0], Jext_mean=[1.0, 1.3],
            nu_ext_hz=[3000.0, 3500.0]), 303),
]


def _split_spikes(L, net, st, ids):
    out = []
    for k in range(net.n_nets):
        info = L.dpsnn_net_info(net, k)
        sel = (ids >= info["base"]) & (ids < info["base"] + info["n_neurons"])
        out.append((st[sel], ids[sel] - info["base"], info))
    return out


@pytest.mark.parametrize("sched", [0, 1])
def test_batch_matches_oracle_per_network(L, sched):
    """Networks of different sizes, parameters and seeds advanced together
    in one handle each reproduce their own oracle run bit for bit."""
    _say("batch vs oracle", sched)
    params = [dict(p, spike_log_cap=1 << 20, rate_bins_cap=256) for p, _ in BATCH]
    seeds = [s for _, s in BATCH]
    net = L.dpsnn_build_batch(params, seeds)
    L.dpsnn_set_schedule(net, sched)
    orcs = [O.Oracle(p, s) for p, s in zip(params, seeds)]
    L.dpsnn_step(net, 1500)
    for o in orcs:
        o.step(1500)
    st, ids = L.dpsnn_read_spikes(net)
    V, c, r = L.dpsnn_read_state(net)
    slots = L.dpsnn_read_slots(net)
    rates = L.dpsnn_read_rates(net)
    total = 0
    for (s_k, i_k, info), o in zip(_split_spikes(L, net, st, ids), orcs):
        ost, oids = o.spikes()
        assert np.array_equal(s_k, ost) and np.array_equal(i_k, oids)
        b, n = info["base"], info["n_neurons"]
        oV, oc, orr = o.state()
        assert np.array_equal(V[b:b + n].astype(np.float64), oV)
        assert np.array_equal(c[b:b + n].astype(np.float64), oc)
        assert np.array_equal(r[b:b + n].astype(np.int32), orr)
        assert np.array_equal(slots[:, b:b + n], o.ring())
        mb, m = info["module_base"], info["n_modules"]
        assert np.array_equal(rates[:, mb:mb + m, :], o.rates()[:rates.shape[0]])
        total += len(ost)
    assert total > 300 and len(st) == total
    net.close()


def test_batch_matches_solo_runs(L):
    """A batch of larger networks (uneven sizes, adaptation and lambda
    swept) against each network built and run alone on the GPU."""
    _say("batch vs solo")
    plist = [W.grid(4, 4, "swa", **{"gc": [0.02, 0.0], "lambda": 1.0, "weight_dtype": "f16"}),
             W.grid(2, 6, "swa", **{"gc": [0.002, 0.0], "lambda": 2.0, "weight_dtype": "f16"}),
             W.grid(3, 3, "swa", **{"gc": [0.0063, 0.0], "lambda": 2.0, "weight_dtype": "f16"})]
    plist = [dict(p, spike_log_cap=1 << 22, rate_bins_cap=256) for p in plist]
    seeds = [11, 12, 13]
    net = L.dpsnn_build_batch(plist, seeds)
    L.dpsnn_step(net, 3000)
    st, ids = L.dpsnn_read_spikes(net)
    parts = _split_spikes(L, net, st, ids)
    for (s_k, i_k, info), p, sd in zip(parts, plist, seeds):
        solo = L.dpsnn_build(p, sd)
        L.dpsnn_step(solo, 3000)
        ss, si = L.dpsnn_read_spikes(solo)
        assert np.array_equal(s_k, ss) and np.array_equal(i_k, si)
        assert len(ss) > 1000
        solo.close()
    net.close()


@pytest.mark.parametrize("sched", [0, 1])
@pytest.mark.parametrize("cap", [-1, 1, 7, 0])
def test_queue_capacity_bit_exact(L, cap, sched):
    """Events go through the tile inboxes and per-slot queues, past a full
    inbox or queue into the slots, or (cap -1) all into the slots: rasters,
    state and slots stay those of the oracle.  Cases: modules of 1500
    neurons (three tiles), int8 efficacies with int64 slots (8-byte queue
    entries), a minimum delay of 3 steps (no event arrives in the step after
    its spike), modules of 3100 neurons (four tiles and more)."""
    cases = [W.tiny(w=2, h=2, K=1500, K_out=120, nu_ext_hz=[2600.0, 2600.0]),
             W.tiny(w=2, h=2, K=1100, K_out=100, weight_dtype="i8", acc_bits=64,
                    q_frac_bits=32, nu_ext_hz=[2600.0, 2600.0]),
             W.tiny(w=3, h=2, K=700, K_out=90, d_min=3, d_max=11,
                    nu_ext_hz=[2600.0, 2600.0]),
             W.tiny(w=1, h=2, K=3100, K_out=60, nu_ext_hz=[2600.0, 2600.0])]
    for k, p in enumerate(cases):
        _say("queue cap", cap, "schedule", sched, "case", k)
        net, orc = _pair(p, 3, queue_cap=cap)
        L.dpsnn_set_schedule(net, sched)
        want = {-1: 0, 0: 4096}.get(cap, cap)
        assert net.stats()["queue_cap"] == want
        n = 0
        for j in range(3):
            L.dpsnn_step(net, 300)
            orc.step(300)
            n += _compare_all(L, net, orc, (cap, sched, k, j))
        assert n > 200
        net.close()


def test_queues_off_past_128_slots(L):
    p = W.tiny(w=2, h=2, K=200, K_out=40, d_min=100, d_max=130,
               nu_ext_hz=[2600.0, 2600.0])
    _say("131 slots")
    net, orc = _pair(p, 2)
    assert net.stats()["queue_cap"] == 0
    L.dpsnn_step(net, 400)
    orc.step(400)
    assert _compare_all(L, net, orc, "131 slots") > 0
    net.close()


@pytest.mark.parametrize("sched", [0, 1])
def test_more_work_items_than_delivery_wavefronts(L, sched):
    """A 4x4 grid driven hard enough that about a third of the steps have
    more (spike, chunk) work items than the delivery kernel has wavefronts,
    with the inbox-routing blocks present: rasters, state and slots equal
    the oracle's."""
    p = W.tiny(w=4, h=4, K=700, K_out=1000, nu_ext_hz=[60000.0, 60000.0])
    _say("many work items, schedule", sched)
    net, orc = _pair(p, 4)
    L.dpsnn_set_schedule(net, sched)
    n = 0
    for j in range(3):
        L.dpsnn_step(net, 100)
        orc.step(100)
        n += _compare_all(L, net, orc, ("many items", sched, j))
    assert n > 50000
    net.close()


# ---------------------------------------------------------------------------
# Population model (Sec. 2.2, Table S1): F/B/I populations, per-pair
# efficacies, Eq. 1 from d = 0, open or periodic boundaries

POP_CASES = {
    "fbi_sw_open_f32": W.fbi(4, 3, "sw", scale=0.1),
    "fbi_aw88_torus_f32": W.fbi(3, 3, "aw88", scale=0.1, open_boundary=0, lam=0.7),
    "fbi_aw28_open_f16": W.fbi(3, 4, "aw28", scale=0.1, weight_dtype="f16", lam=0.4),
    "fbi_aw88_open_i8_q32": W.fbi(4, 2, "aw88", scale=0.1, weight_dtype="i8",
                                  acc_bits=64, q_frac_bits=32),
    "fbi_swv_open_f16": W.fbi(4, 4, "swv", scale=0.1, weight_dtype="f16", lam=0.6),
    # F and B share their Eq. 2 constants in the cases above (two classes);
    # here every population has its own membrane time constant
    "fbi_three_classes_f32": W.fbi(3, 3, "aw88", scale=0.1, p_tau_m=[20.0, 16.0, 10.0]),
}


@pytest.mark.parametrize("case", sorted(POP_CASES))
def test_population_rows_bitwise_equal(L, case):
    p = POP_CASES[case]
    _say("population rows", case)
    net, orc = _pair(p, 7)
    _compare_rows(L, net, orc, list(range(net.N)), p["weight_dtype"])
    net.close()


@pytest.mark.parametrize("sched", [0, 1])
@pytest.mark.parametrize("case", sorted(POP_CASES))
def test_population_raster_bit_exact(L, case, sched):
    p = POP_CASES[case]
    _say("population raster", case, "schedule", sched)
    net, orc = _pair(p, 11)
    L.dpsnn_set_schedule(net, sched)
    n = 0
    for k in range(3):
        L.dpsnn_step(net, 1000)
        orc.step(1000)
        n += _compare_all(L, net, orc, (case, sched, k))
    assert n > 200
    r = L.dpsnn_read_rates(net)
    assert r.shape[2] == 3
    assert np.array_equal(r, orc.rates()[: 3000 // p["rate_bin_steps"]])
    net.close()


def test_population_full_size_start_and_teacher_forced_step(L):
    """F/B/I SW network of 24x24 full-size modules (720k neurons, 0.81G
    synapses, open edges): sampled rows, the first 30 steps bit-exact, then
    after 1000 more steps one step re-run by the oracle from the GPU's state,
    slots and time."""
    p = W.fbi(24, 24, "sw")
    _say("F/B/I 24x24 build")
    net, orc = _pair(p, 1, store_rows=False)
    rng = np.random.default_rng(0)
    rows = sorted(rng.choice(net.N, 200, replace=False).tolist())
    _compare_rows(L, net, orc, rows, "f32")
    L.dpsnn_step(net, 30)
    orc.step(30)
    _compare_all(L, net, orc, "fbi start")
    L.dpsnn_step(net, 1000)
    L.dpsnn_read_spikes(net)
    V, c, r = L.dpsnn_read_state(net)
    slots = L.dpsnn_read_slots(net)
    orc2 = O.Oracle(p, 1, store_rows=False)
    orc2.set_state(V.astype(np.float64), c.astype(np.float64), r.astype(np.int32))
    orc2.set_ring(slots)
    orc2.set_time(1030)
    L.dpsnn_step(net, 1)
    orc2.step(1)
    st, ids = L.dpsnn_read_spikes(net)
    ost, oids = _new_oracle_spikes(orc2)
    assert np.array_equal(st, ost) and np.array_equal(ids, oids)
    assert len(st) > 0
    _compare_state(L, net, orc2, "fbi teacher forced")
    assert np.array_equal(L.dpsnn_read_slots(net), orc2.ring())
    net.close()


def test_population_batch_matches_solo_runs(L):
    plist = [W.fbi(3, 3, "sw", scale=0.1), W.fbi(2, 4, "aw88", scale=0.1, lam=0.7),
             W.fbi(4, 4, "aw28", scale=0.1, open_boundary=0)]
    seeds = [3, 4, 5]
    _say("population batch vs solo")
    net = L.dpsnn_build_batch(plist, seeds)
    L.dpsnn_step(net, 2000)
    st, ids = L.dpsnn_read_spikes(net)
    parts = _split_spikes(L, net, st, ids)
    for (s_k, i_k, info), p, sd in zip(parts, plist, seeds):
        solo = L.dpsnn_build(p, sd)
        L.dpsnn_step(solo, 2000)
        ss, si = L.dpsnn_read_spikes(solo)
        assert np.array_equal(s_k, ss) and np.array_equal(i_k, si)
        assert len(ss) > 500
        solo.close()
    net.close()


@pytest.mark.parametrize("side,K_out", [(3, 200), (9, 100)])
def test_spike_list_kinds_and_grids(L, side, K_out):
    """The split schedule's delivery with per-tile and with appended spike
    lists (with and without merged reservations) and several grids,
    switched between calls (graphs and direct launches): bit-exact; 11
    tiles (lists of one tile or none) and 99 tiles (several tiles in some of
    the 64 lists)."""
    import torch
    _say("spike list kinds", side, K_out)
    p = W.grid(side, side, "swa", K=1250, K_out=K_out)
    with torch.cuda.stream(torch.cuda.Stream()):
        net, orc = _pair(p, 9)
        L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
        for k, (blocks, lists) in enumerate([(0, 1), (7, 0), (256, 2), (1024, 0), (3, 1),
                                             (512, 2), (256, 0), (5, 2), (1024, 1)]):
            L.dpsnn_set_delivery(net, blocks, lists)
            st = net.stats()
            assert st["spike_lists"] == lists
            assert blocks == 0 or st["deliver_blocks"] == blocks
            n = 300 if k % 2 else 47      # graph replays and direct launches; direct only
            L.dpsnn_step(net, n)
            orc.step(n)
            assert _compare_all(L, net, orc, f"lists {lists} blocks {blocks}") > 0
        for bad in [(-1, 0), (0, 3), (0, -2)]:
            with pytest.raises(L.DpsnnError):
                L.dpsnn_set_delivery(net, *bad)
        net.close()


def test_queue_entry_formats(L):
    """Binary32 efficacies: 4-byte queue entries when every fixed-point
    efficacy fits 21 bits (the benchmark's networks), 8 bytes otherwise: two
    words with int32 inputs (bit-exact with efficacies of up to 40 mV), one
    packed word with int64 inputs.  Binary16 and int8 efficacies: 4-byte
    code entries with either slot width (bit-exact, both schedules, also
    with efficacies of up to 40 mV)."""
    _say("queue entry formats")
    p = W.tiny(2, 2, K=64, K_out=32)
    net = L.dpsnn_build(dict(p, spike_log_cap=1 << 20), 1)
    assert net.stats()["queue_entry_bytes"] == 4
    net.close()
    net = L.dpsnn_build(dict(p, acc_bits=64, q_frac_bits=32, spike_log_cap=1 << 20), 1)
    assert net.stats()["queue_entry_bytes"] == 8
    net.close()
    big = dict(p, J_mean=[35.0, -40.0], J_sd=[5.0, 5.0])
    net, orc = _pair(big, 4)
    assert net.stats()["queue_entry_bytes"] == 8
    for sched in (L.SCHED_SPLIT, L.SCHED_FUSED):
        L.dpsnn_set_schedule(net, sched)
        L.dpsnn_step(net, 150)
        orc.step(150)
        assert _compare_all(L, net, orc, f"8-byte entries {sched}") > 0
    net.close()
    for wd in ("f16", "i8"):
        for acc in (32, 64):
            q = dict(big, weight_dtype=wd)
            if acc == 64:
                q.update(acc_bits=64, q_frac_bits=32)
            net, orc = _pair(q, 6)
            assert net.stats()["queue_entry_bytes"] == 4, (wd, acc)
            for sched in (L.SCHED_SPLIT, L.SCHED_FUSED, L.SCHED_SPLIT):
                L.dpsnn_set_schedule(net, sched)
                L.dpsnn_step(net, 100)
                orc.step(100)
                assert _compare_all(L, net, orc, f"code entries {wd} {acc} {sched}") > 0
            net.close()


def test_per_network_reads(L):
    """dpsnn_read_spikes_net / dpsnn_read_rates_net return one network's
    spikes (network-local ids) and rate bins; what the other networks have
    not read stays for later reads, and the whole-handle reads return the
    rest (counts already drained read 0)."""
    _say("per-network reads")
    params = [dict(p, spike_log_cap=1 << 20, rate_bins_cap=256) for p, _ in BATCH]
    seeds = [s for _, s in BATCH]
    net = L.dpsnn_build_batch(params, seeds)
    orcs = [O.Oracle(p, s) for p, s in zip(params, seeds)]
    L.dpsnn_step(net, 700)
    for o in orcs:
        o.step(700)
    st1, id1 = L.dpsnn_read_spikes_net(net, 1)
    ost, oids = orcs[1].spikes()
    assert len(st1) > 50
    assert np.array_equal(st1, ost) and np.array_equal(id1, oids)
    r0 = L.dpsnn_read_rates_net(net, 0)
    assert np.array_equal(r0, orcs[0].rates()[:r0.shape[0]])
    assert L.dpsnn_read_spikes_net(net, 1)[0].size == 0       # drained
    L.dpsnn_step(net, 300)
    for o in orcs:
        o.step(300)
    # network 1 again: only its spikes of the last 300 steps
    st1b, id1b = L.dpsnn_read_spikes_net(net, 1)
    ost, oids = orcs[1].spikes()
    late = ost >= 700
    assert np.array_equal(st1b, ost[late]) and np.array_equal(id1b, oids[late])
    # the whole handle: networks 0 and 2 from the start, global ids
    st, ids = L.dpsnn_read_spikes(net)
    parts = _split_spikes(L, net, st, ids)
    for k in (0, 2):
        s_k, i_k, _ = parts[k]
        ost, oids = orcs[k].spikes()
        assert np.array_equal(s_k, ost) and np.array_equal(i_k, oids), k
    assert parts[1][0].size == 0
    rates = L.dpsnn_read_rates(net)
    info0 = L.dpsnn_net_info(net, 0)
    mb, m = info0["module_base"], info0["n_modules"]
    nb0 = r0.shape[0]
    assert np.all(rates[:nb0, mb:mb + m, :] == 0)          # network 0 read them already
    assert np.array_equal(rates[nb0:, mb:mb + m, :], orcs[0].rates()[nb0:nb0 + rates.shape[0] -
                                                                        nb0])
    for k in (1, 2):
        info = L.dpsnn_net_info(net, k)
        mb, m = info["module_base"], info["n_modules"]
        assert np.array_equal(rates[:, mb:mb + m, :], orcs[k].rates()[:rates.shape[0]]), k
    assert L.dpsnn_read_rates_net(net, 2).shape[0] == 0
    with pytest.raises(L.DpsnnError):
        L.dpsnn_read_spikes_net(net, 3)
    net.close()


def test_routing_grid_below_tile_count(L):
    """Routing blocks that each walk several tiles (1, 3 and 7 blocks for 11
    tiles; the 96x96 and batched networks have more tiles than the default
    4096 blocks), switched between graph replays and direct launches: rasters,
    state and slots equal the oracle's."""
    import torch
    p = W.grid(3, 3, "swa", K=1250, K_out=200)
    _say("routing grid")
    with torch.cuda.stream(torch.cuda.Stream()):
        net, orc = _pair(p, 21)
        L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
        assert net.stats()["route_blocks"] == 11
        for k, rb in enumerate([1, 3, 7, 0, 2]):
            L.dpsnn_set_routing(net, rb)
            assert net.stats()["route_blocks"] == (rb or 11)
            n = 300 if k % 2 == 0 else 53
            L.dpsnn_step(net, n)
            orc.step(n)
            assert _compare_all(L, net, orc, f"routing {rb}") > 0
        for bad in (-1, 12):
            with pytest.raises(L.DpsnnError):
                L.dpsnn_set_routing(net, bad)
        net.close()


def test_spike_order_per_tile_lists_is_deterministic(L):
    """Each tile lists its spikes in neuron order (wavefront ballot and block
    prefix sum), so with per-tile spike lists the split schedule writes the
    device log in (step, id) order, identically on a rerun; with appended
    lists (either delivery) every tile's run of the log is in id order."""
    p = W.grid(3, 3, "swa", K=1250, K_out=200, spike_log_cap=1 << 22)
    _say("spike order")
    logs = []
    for lists in (0, 0, 1, 2):
        net = L.dpsnn_build(p, 5)
        L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
        L.dpsnn_set_delivery(net, 0, lists)
        L.dpsnn_step(net, 700)
        st, ids = L.dpsnn_read_log(net)
        sst, sids = L.dpsnn_read_spikes(net)      # sorted and drained
        assert len(st) == len(sst) > 1000
        key = st.astype(np.int64) * (1 << 32) + ids
        if lists == 0:
            assert np.all(np.diff(key) > 0)
            assert np.array_equal(st, sst) and np.array_equal(ids, sids)
        else:
            # within one step and one tile, ids increase along the log
            same = (st[1:] == st[:-1]) & ((ids[1:] >> 10) == (ids[:-1] >> 10))
            assert np.all(ids[1:][same] > ids[:-1][same])
        logs.append((st, ids))
        net.close()
    assert np.array_equal(logs[0][0], logs[1][0]) and np.array_equal(logs[0][1], logs[1][1])


@pytest.mark.parametrize("case", ["tiny_f32_acc32", "tiny_i8_acc64", "tiny_f16_acc32",
                                  "mid_f32_strong_adapt"])
def test_persistent_schedule_bit_exact(L, case):
    """The persistent schedule (many steps per cooperative launch, grid
    synchronisation between update and delivery) against the oracle, with
    switches to the split and fused schedules between chunks."""
    p = RASTER_CASES[case]
    _say("persistent", case)
    net, orc = _pair(p, 8)
    n = 0
    for k, (sched, steps) in enumerate([(2, 300), (1, 130), (2, 1), (0, 77), (2, 700)]):
        L.dpsnn_set_schedule(net, sched)
        assert net.stats()["schedule"] == sched
        L.dpsnn_step(net, steps)
        orc.step(steps)
        n += _compare_all(L, net, orc, (case, k, sched))
    assert n > 50
    assert np.array_equal(L.dpsnn_read_rates(net), orc.rates()[: 1208 // p["rate_bin_steps"]])
    net.close()


def test_persistent_schedule_population_model_and_batch(L):
    """Persistent schedule on a batch of F/B/I networks (three populations)
    against each network's solo run with the split schedule."""
    plist = [W.fbi(3, 3, "sw", scale=0.1), W.fbi(2, 4, "aw88", scale=0.1, lam=0.7)]
    seeds = [3, 4]
    _say("persistent batch")
    net = L.dpsnn_build_batch(plist, seeds)
    L.dpsnn_set_schedule(net, 2)
    L.dpsnn_step(net, 1500)
    st, ids = L.dpsnn_read_spikes(net)
    parts = _split_spikes(L, net, st, ids)
    for (s_k, i_k, info), p, sd in zip(parts, plist, seeds):
        solo = L.dpsnn_build(p, sd)
        L.dpsnn_set_schedule(solo, 1)
        L.dpsnn_step(solo, 1500)
        ss, si = L.dpsnn_read_spikes(solo)
        assert np.array_equal(s_k, ss) and np.array_equal(i_k, si)
        assert len(ss) > 300
        solo.close()
    net.close()


@pytest.mark.timeout(300)
def test_merged_reservations_under_hash_pressure(L):
    """Merged reservations with most of the LDS hash in use: 30x30 modules
    (1099 tiles), every synapse remote and its module drawn almost
    uniformly (lambda = 100), 256 synapses per row, so the four chunks of a
    block reach ~660 distinct tiles per round (linear probing in a
    1024-entry table).  Bit-exact against the oracle with the merged
    delivery, then with the per-run one on the same handle."""
    _say("merged reservations, hash pressure")
    p = W.grid(30, 30, "swa", K=1250, K_out=256, frac_local=[0.0, 0.0], **{"lambda": 100.0})
    net, orc = _pair(p, 21, store_rows=False)
    assert -(-net.N // 1024) == 1099
    L.dpsnn_set_schedule(net, L.SCHED_SPLIT)
    L.dpsnn_set_delivery(net, 1024, 2)
    # the start: thousands of spikes per step (the oracle is the slow side)
    for k, (lists, n) in enumerate([(2, 12), (2, 17), (1, 9)]):
        L.dpsnn_set_delivery(net, 0, lists)
        L.dpsnn_step(net, n)
        orc.step(n)
        assert _compare_all(L, net, orc, f"hash pressure {k}") > 100
    net.close()
    orc.close()
