"""Pins of the binary64 reductions in oracle/stats.py (CPU): population
rates in 5 ms bins, the Up/Down detector on module activity (Sec. 2.3),
per-neuron count histograms and the Kolmogorov-Smirnov distance, each
against values fixed by construction or by an independent library routine."""
import numpy as np
import pytest

from oracle import stats


def _square_wave(levels_and_lengths):
    return np.concatenate([np.full(n, v, np.float64) for v, n in levels_and_lengths])


def test_up_states_of_a_planted_square_wave():
    # 5 ms bins: Up episodes of 12, 20 and 11 bins (60, 100, 55 ms) and a
    # 4-bin (20 ms) burst; Down level 1, Up level 11
    x = _square_wave([(1, 30), (11, 12), (1, 25), (11, 20), (1, 10), (11, 4), (1, 30),
                      (11, 11), (1, 40)])
    ep = stats.up_states(x, min_up=10)
    assert ep == [(30, 12), (67, 20), (131, 11)]
    # with a 10 ms minimum the burst counts too
    assert [n for _, n in stats.up_states(x, min_up=2)] == [12, 20, 4, 11]


def test_hysteresis_keeps_a_shallow_dip_inside_one_up_state():
    # p5 = 1, p95 = 11: mid 6, thresholds 7 (up) and 5 (down); a dip to 6
    # does not end the Up state, a dip to 4 does
    x = _square_wave([(1, 40), (11, 15), (6, 2), (11, 15), (1, 40), (11, 15), (4, 2),
                      (11, 15), (1, 40)])
    ep = stats.up_states(x, min_up=10)
    assert [n for _, n in ep] == [32, 15, 15]


def test_up_state_frequency_counts_modules_and_skips_the_transient():
    bin_ms = 5.0
    # 3 s of bins; module 0: an Up state of 100 ms every 500 ms after 0.5 s
    # (5 in the analysed 2.5 s), module 1 flat (0 Hz) -> mean 1 Hz
    n = 600
    m0 = np.ones(n)
    for k in range(5):
        a = 100 + 100 * k + 30
        m0[a:a + 20] = 12.0
    m0[10:40] = 12.0  # inside the skipped transient
    counts = np.zeros((n, 2, 2), np.uint32)
    counts[:, 0, 0] = m0.astype(np.uint32)
    counts[:, 1, 0] = 3
    s = stats.up_state_stats(counts, bin_ms, skip_s=0.5, min_up_ms=50.0)
    assert s["freq_hz"] == pytest.approx(0.5 * 5 / 2.5)
    assert s["mean_up_ms"] == pytest.approx(100.0)
    assert s["up_fraction"] == pytest.approx(5 * 20 / (500 * 2))


def test_module_rates():
    counts = np.zeros((4, 3, 2), np.uint32)
    counts[:, 1, 0] = 10   # 10 spikes of 1000 exc neurons per 5 ms = 2 Hz
    counts[:, 2, 1] = 5    # 5 spikes of 250 inh neurons per 5 ms = 4 Hz
    e, i = stats.module_rates_hz(counts, 1000, 250, 5.0)
    assert e.shape == (4, 3)
    assert np.allclose(e[:, 1], 2.0) and np.allclose(i[:, 2], 4.0)
    assert np.all(e[:, 0] == 0) and np.all(i[:, 1] == 0)


def test_population_rates_brute_force():
    """Mean rate of each population after the skipped bins, against a loop
    over bins and modules."""
    rng = np.random.default_rng(4)
    counts = rng.integers(0, 40, size=(300, 5, 3)).astype(np.uint32)
    sizes = [250, 750, 250]
    got = stats.population_rates_hz(counts, sizes, 5.0, skip_s=0.5)
    for q in range(3):
        spikes, bins = 0, 0
        for b in range(100, 300):          # 0.5 s = 100 bins of 5 ms skipped
            bins += 1
            for m in range(5):
                spikes += int(counts[b, m, q])
        want = spikes / (sizes[q] * 5) / (bins * 5e-3)
        assert got[q] == pytest.approx(want, rel=1e-12)


def test_neuron_rate_hist_brute_force():
    rng = np.random.default_rng(3)
    ids = rng.integers(0, 50, size=700)
    h = stats.neuron_rate_hist(ids, 60, max_count=30)
    per = [int(np.sum(ids == k)) for k in range(60)]
    ref = [0] * 31
    for c in per:
        ref[min(c, 30)] += 1
    assert h.tolist() == ref
    assert h.sum() == 60


def test_ks_from_hists_matches_scipy():
    from scipy.stats import ks_2samp
    rng = np.random.default_rng(7)
    a = rng.poisson(12.0, size=3000)
    b = rng.poisson(13.0, size=2000)
    ha = np.bincount(a)
    hb = np.bincount(b)
    assert stats.ks_from_hists(ha, hb) == pytest.approx(ks_2samp(a, b).statistic, abs=1e-12)
    assert stats.ks_from_hists(ha, ha * 3) == 0.0
