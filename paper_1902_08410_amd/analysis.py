"""Host-side analysis of simulation output (binary64 reductions).

Population rates in bins of 5 ms (Sec. 2.3), a multi-unit-activity
Up/Down detector for the slow-wave regime (Sec. 2.3: the module's average
rate alternates between high and low states; the Down-to-Up transition is
found with a threshold), per-neuron rate distributions and the
two-sample Kolmogorov-Smirnov distance between them.

The paper does not give the threshold.  The detector here: per module,
MUA = spike count of the module per bin; mid = (p5 + p95) / 2 over the
analysed window, hysteresis +-20 % of (p95 - p5) / 2 around mid, an Up
state must last 50 ms to count; the up-state frequency is the number of
counted Down-to-Up transitions per second, averaged over modules.  The
same detector with a 10 ms minimum gives the rate of shorter population
bursts.
"""
import numpy as np


def module_rates_hz(counts: np.ndarray, n_exc: int, n_inh: int, bin_ms: float):
    """counts [bins][modules][2] -> (exc Hz, inh Hz), each [bins][modules]."""
    c = counts.astype(np.float64)
    s = bin_ms * 1e-3
    return c[:, :, 0] / n_exc / s, c[:, :, 1] / n_inh / s


def up_state_frequency(counts: np.ndarray, bin_ms: float, skip_s: float = 0.5,
                       min_up_ms: float = 50.0, hyst: float = 0.2) -> float:
    """Down-to-Up transitions per second, averaged over modules."""
    mua = counts.astype(np.float64).sum(axis=2)          # [bins][modules]
    k0 = int(round(skip_s * 1e3 / bin_ms))
    mua = mua[k0:]
    if mua.shape[0] < 2:
        return 0.0
    dur_s = mua.shape[0] * bin_ms * 1e-3
    min_up = max(1, int(round(min_up_ms / bin_ms)))
    freqs = []
    for m in range(mua.shape[1]):
        x = mua[:, m]
        p5, p95 = np.percentile(x, [5, 95])
        if p95 <= p5:
            freqs.append(0.0)
            continue
        mid, half = 0.5 * (p5 + p95), 0.5 * (p95 - p5)
        hi_t, lo_t = mid + hyst * half, mid - hyst * half
        up = False
        start = 0
        n = 0
        for i, v in enumerate(x):
            if not up and v > hi_t:
                up, start = True, i
            elif up and v < lo_t:
                if i - start >= min_up:
                    n += 1
                up = False
        if up and len(x) - start >= min_up:
            n += 1
        freqs.append(n / dur_s)
    return float(np.mean(freqs))


def neuron_rate_hist(ids: np.ndarray, n_neurons: int, duration_s: float,
                     max_count: int = 2000) -> np.ndarray:
    """Histogram of per-neuron spike counts (index = count)."""
    per = np.bincount(ids, minlength=n_neurons)[:n_neurons]
    return np.bincount(np.minimum(per, max_count), minlength=max_count + 1)


def ks_from_hists(a: np.ndarray, b: np.ndarray) -> float:
    """Two-sample Kolmogorov-Smirnov distance of two count histograms."""
    n = max(len(a), len(b))
    a = np.pad(a.astype(np.float64), (0, n - len(a)))
    b = np.pad(b.astype(np.float64), (0, n - len(b)))
    return float(np.max(np.abs(np.cumsum(a) / a.sum() - np.cumsum(b) / b.sum())))


def summary(counts: np.ndarray, steps: np.ndarray, ids: np.ndarray, n_neurons: int,
            K: int, K_exc: int, bin_ms: float, dt_ms: float, t_end: int,
            skip_s: float = 0.5) -> dict:
    """Statistics of one run of t_end steps: mean rates after the transient,
    up-state frequency, histogram of per-neuron spike counts after the
    transient."""
    k0 = int(round(skip_s * 1e3 / bin_ms))
    e, i = module_rates_hz(counts[k0:], K_exc, K - K_exc, bin_ms)
    t0 = int(round(skip_s * 1e3 / dt_ms))
    late = ids[steps >= t0]
    hist = neuron_rate_hist(late, n_neurons, (t_end - t0) * dt_ms * 1e-3)
    last = int(np.nonzero(hist)[0].max()) + 1 if hist.any() else 1
    return {"rate_exc_hz": float(e.mean()), "rate_inh_hz": float(i.mean()),
            "up_freq_hz": up_state_frequency(counts, bin_ms, skip_s),
            "burst_freq_hz": up_state_frequency(counts, bin_ms, skip_s, min_up_ms=10.0),
            "count_hist": hist[:last].tolist()}
