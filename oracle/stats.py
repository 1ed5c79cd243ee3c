"""Binary64 reductions of simulation output (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the stored binary64
statistics and the precision tests reduce spike rasters and rate bins with
these functions, on the oracle's output and on the library's alike.

What they compute:
  - population rates in bins of 5 ms and their means (Sec. 2.3: firing
    rates per sub-population);
  - an Up/Down detector on the multi-unit activity of each module (Sec. 2.3:
    in the slow-wave state the module activity alternates between high and
    low states; the Down-to-Up transition is found with a threshold the paper
    does not give).  Here: MUA = the module's spike count per bin, threshold
    mid = (p5 + p95) / 2 over the analysed window, hysteresis +-20 % of
    (p95 - p5) / 2 around it, an Up state counts when it lasts at least
    min_up_ms (50 ms for slow-wave Up states, 10 ms for population bursts);
    the frequency is counted Down-to-Up transitions per second, averaged
    over modules;
  - per-neuron spike-count histograms and the two-sample Kolmogorov-Smirnov
    distance between two of them.
"""
import numpy as np


def module_rates_hz(counts: np.ndarray, n_exc: int, n_inh: int, bin_ms: float):
    """counts [bins][modules][2] -> (exc Hz, inh Hz), each [bins][modules]."""
    c = counts.astype(np.float64)
    s = bin_ms * 1e-3
    return c[:, :, 0] / n_exc / s, c[:, :, 1] / n_inh / s


def population_rates_hz(counts: np.ndarray, sizes, bin_ms: float, skip_s: float = 0.5):
    """counts [bins][modules][P], sizes[P] neurons per module -> mean rate
    (Hz) of each population over all modules after the first skip_s."""
    k0 = int(round(skip_s * 1e3 / bin_ms))
    c = counts[k0:].astype(np.float64)
    dur_s = c.shape[0] * bin_ms * 1e-3
    tot = c.sum(axis=(0, 1))
    return [float(tot[q] / (sizes[q] * c.shape[1]) / dur_s) for q in range(c.shape[2])]


def up_states(x: np.ndarray, min_up: int, hyst: float = 0.2):
    """Up states of one MUA trace x (counts per bin): list of (start bin,
    length in bins) of the episodes that rise above mid + hyst * half and
    stay until the trace falls below mid - hyst * half, at least min_up bins
    long.  An episode still Up at the end counts if long enough."""
    x = np.asarray(x, np.float64)
    p5, p95 = np.percentile(x, [5, 95])
    if p95 <= p5:
        return []
    mid, half = 0.5 * (p5 + p95), 0.5 * (p95 - p5)
    hi_t, lo_t = mid + hyst * half, mid - hyst * half
    out = []
    up, start = False, 0
    for i, v in enumerate(x):
        if not up and v > hi_t:
            up, start = True, i
        elif up and v < lo_t:
            if i - start >= min_up:
                out.append((start, i - start))
            up = False
    if up and len(x) - start >= min_up:
        out.append((start, len(x) - start))
    return out


def up_state_stats(counts: np.ndarray, bin_ms: float, skip_s: float = 0.5,
                   min_up_ms: float = 50.0, hyst: float = 0.2) -> dict:
    """Up states of every module after the transient: frequency (Down-to-Up
    transitions per second averaged over modules), mean Up duration (ms, over
    all episodes; 0 without any) and the fraction of time spent Up."""
    mua = counts.astype(np.float64).sum(axis=2)          # [bins][modules]
    k0 = int(round(skip_s * 1e3 / bin_ms))
    mua = mua[k0:]
    if mua.shape[0] < 2:
        return {"freq_hz": 0.0, "mean_up_ms": 0.0, "up_fraction": 0.0}
    dur_s = mua.shape[0] * bin_ms * 1e-3
    min_up = max(1, int(round(min_up_ms / bin_ms)))
    freqs, lens = [], []
    for m in range(mua.shape[1]):
        ep = up_states(mua[:, m], min_up, hyst)
        freqs.append(len(ep) / dur_s)
        lens.extend(n for _, n in ep)
    total_up = float(np.sum(lens)) if lens else 0.0
    return {"freq_hz": float(np.mean(freqs)),
            "mean_up_ms": float(np.mean(lens) * bin_ms) if lens else 0.0,
            "up_fraction": total_up / (mua.shape[0] * mua.shape[1])}


def up_state_frequency(counts: np.ndarray, bin_ms: float, skip_s: float = 0.5,
                       min_up_ms: float = 50.0, hyst: float = 0.2) -> float:
    """Down-to-Up transitions per second, averaged over modules."""
    return up_state_stats(counts, bin_ms, skip_s, min_up_ms, hyst)["freq_hz"]


def neuron_rate_hist(ids: np.ndarray, n_neurons: int, max_count: int = 2000) -> np.ndarray:
    """Histogram of per-neuron spike counts (index = count; counts above
    max_count land in the last entry)."""
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
    """Statistics of one run of t_end steps of the two-population model:
    mean rates after the transient, Up states (>= 50 ms) and population
    bursts (>= 10 ms), histogram of per-neuron spike counts after the
    transient."""
    k0 = int(round(skip_s * 1e3 / bin_ms))
    e, i = module_rates_hz(counts[k0:], K_exc, K - K_exc, bin_ms)
    t0 = int(round(skip_s * 1e3 / dt_ms))
    late = ids[steps >= t0]
    hist = neuron_rate_hist(late, n_neurons)
    last = int(np.nonzero(hist)[0].max()) + 1 if hist.any() else 1
    up = up_state_stats(counts, bin_ms, skip_s)
    return {"rate_exc_hz": float(e.mean()), "rate_inh_hz": float(i.mean()),
            "up_freq_hz": up["freq_hz"], "mean_up_ms": up["mean_up_ms"],
            "up_fraction": up["up_fraction"],
            "burst_freq_hz": up_state_frequency(counts, bin_ms, skip_s, min_up_ms=10.0),
            "count_hist": hist[:last].tolist()}
