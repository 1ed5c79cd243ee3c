"""Spike-timing-dependent plasticity on the GPU against the oracle.

Bit-exact: the spike rasters and neuron state with plasticity on, and every
synapse's efficacy, last activation step and plasticity signal (binary32,
same operation order on both sides) after several update periods.  Synapses
are matched per row after sorting both rows by (target, delay, efficacy,
activation step, signal): two synapses of a row with the same target share
their activations, so equal keys carry equal state.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1902_08410_amd import workloads as W

pytestmark = pytest.mark.gpu

FAST = dict(plastic=1, stdp_update_steps=150, stdp_A_plus=0.02, stdp_A_minus=0.05,
            stdp_tau_plus=1.5, stdp_tau_minus=2.0, stdp_tau_y=6.0, stdp_eta=10.0,
            stdp_w_max=0.8)


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


def _pair(L, p, seed):
    q = dict(p, spike_log_cap=1 << 22, rate_bins_cap=4096)
    return L.dpsnn_build(q, seed), O.Oracle(q, seed, store_rows=True)


def _compare_synapses(L, net, orc, rows):
    tgt, w, dk = L.dpsnn_read_rows(net, rows[0], len(rows))
    ta, y = L.dpsnn_read_plasticity(net, rows[0], len(rows))
    d_min = int(orc.params["d_min"])
    changed = 0
    for k, s in enumerate(rows):
        otgt, odel, _, _, _ = orc.gen_row_blocks(s)
        ota, oy, ow = orc.plasticity(s)
        a = sorted(zip(tgt[k].tolist(), dk[k].tolist(), w[k].view(np.uint32).tolist(),
                       ta[k].tolist(), y[k].view(np.uint32).tolist()))
        b = sorted(zip(otgt.tolist(), (odel.astype(np.int32) - d_min).tolist(),
                       ow.astype(np.float32).view(np.uint32).tolist(), ota.tolist(),
                       oy.astype(np.float32).view(np.uint32).tolist()))
        assert a == b, s
        changed += int((ta[k] >= 0).sum())
    return changed


def _run_and_compare(L, p, seed, steps, chunk):
    net, orc = _pair(L, p, seed)
    assert net.stats()["schedule"] == L.SCHED_SPLIT
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        L.dpsnn_step(net, n)
        orc.step(n)
        done += n
        st, ids = L.dpsnn_read_spikes(net)
        ost, oids = orc.spikes()
        ost, oids = ost[getattr(orc, "_seen", 0):], oids[getattr(orc, "_seen", 0):]
        orc._seen = len(orc.spikes()[0])
        assert np.array_equal(st, ost) and np.array_equal(ids, oids), done
        V, c, r = L.dpsnn_read_state(net)
        oV, oc, orr = orc.state()
        assert np.array_equal(V.astype(np.float64), oV), done
    return net, orc


@pytest.mark.parametrize("chunk", [150, 97])
def test_plastic_tiny_grid_bit_exact(L, chunk):
    """Six update periods of 150 steps, stepped in whole periods and in
    chunks of 97 steps (updates inside a call)."""
    _say("stdp tiny", chunk)
    p = W.tiny(2, 2, K=40, K_out=20, **FAST)
    net, orc = _run_and_compare(L, p, 3, 900, chunk)
    n = orc.N
    act = _compare_synapses(L, net, orc, list(range(n)))
    net.close()
    assert act > 100


def test_plastic_grid_with_queues_and_graphs(L):
    """4x4 grid of 1250-neuron modules (two populations, queues, captured
    graphs): 2000 steps with an update every 500 steps."""
    _say("stdp 4x4")
    p = W.grid(4, 4, "swa", plastic=1, stdp_update_steps=500, stdp_A_plus=0.01,
               stdp_A_minus=0.012, stdp_tau_plus=2.0, stdp_tau_minus=2.0, stdp_tau_y=20.0,
               stdp_eta=5.0, stdp_w_max=1.0)
    net, orc = _run_and_compare(L, p, 5, 2000, 1000)
    rows = list(range(0, orc.N, 997))[:20]
    act = 0
    for s in rows:
        act += _compare_synapses(L, net, orc, [s])
    net.close()
    assert act > 0


def test_zero_amplitudes_match_the_fixed_network(L):
    _say("stdp zero amplitudes")
    p = W.tiny(2, 2, K=40, K_out=20, **dict(FAST, stdp_A_plus=0.0, stdp_A_minus=0.0,
                                            stdp_w_max=10.0))
    q = dict(p, plastic=0)
    a = L.dpsnn_build(dict(p, spike_log_cap=1 << 20), 7)
    b = L.dpsnn_build(dict(q, spike_log_cap=1 << 20), 7)
    L.dpsnn_set_schedule(b, L.SCHED_SPLIT)
    w0 = L.dpsnn_read_rows(a, 0, 100)[1].copy()
    L.dpsnn_step(a, 600)
    L.dpsnn_step(b, 600)
    sa, ia = L.dpsnn_read_spikes(a)
    sb, ib = L.dpsnn_read_spikes(b)
    assert len(sa) > 50 and np.array_equal(sa, sb) and np.array_equal(ia, ib)
    assert np.array_equal(L.dpsnn_read_rows(a, 0, 100)[1], w0)
    a.close()
    b.close()


def test_plastic_handle_rules(L):
    """Plastic handles run the split schedule only; the plasticity state of
    a fixed handle does not exist."""
    _say("stdp rules")
    p = dict(W.tiny(2, 2, K=40, K_out=20, **FAST), spike_log_cap=1 << 16)
    net = L.dpsnn_build(p, 1)
    with pytest.raises(L.DpsnnError):
        L.dpsnn_set_schedule(net, L.SCHED_FUSED)
    assert L.dpsnn_autotune(net, 50) == L.SCHED_SPLIT
    net.close()
    fixed = L.dpsnn_build(dict(p, plastic=0), 1)
    with pytest.raises(L.DpsnnError) as e:
        L.dpsnn_read_plasticity(fixed, 0, 1)
    assert e.value.code == -6
    fixed.close()
