"""Slow-wave analysis on the GPU (Sec. 2.3, Eq. 4) against the oracle.

Bit-exact: the transitions (module, time in binary64, wave), the waves'
first times and sizes.  Wave speeds and their mean: within 1e-12 relative,
the two sides summing the same binary64 terms in different orders (at most
8192 terms of magnitude below 1e6 imd/s: the rounding differences stay
below 8192 * 2^-53 relative).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1902_08410_amd import workloads as W

pytestmark = pytest.mark.gpu
BIN_STEPS, DT = 50, 0.1


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


def _compare(got, ref):
    n = len(ref["T"])
    assert got["n_transitions"] == n
    assert np.array_equal(got["module"], ref["module"])
    assert np.array_equal(got["T"], ref["T"])
    assert np.array_equal(got["wave"], ref["wave"])
    assert got["n_waves"] == len(ref["speed"])
    assert np.array_equal(got["n"], ref["n"])
    assert np.array_equal(got["t0"], ref["t0"])
    a, b = got["speed"], ref["speed"]
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(b)
    np.testing.assert_allclose(a[ok], b[ok], rtol=1e-12, atol=0)
    mean = float(np.mean(b[ok])) if ok.any() else float("nan")
    if ok.any():
        assert got["mean_speed"] == pytest.approx(mean, rel=1e-12)
    else:
        assert np.isnan(got["mean_speed"])


def _on_gpu(L, c, Wd, Hd, **kw):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(c, np.uint32).view(np.int32)).cuda()
    return L.dpsnn_waves_counts(t, Wd, Hd, BIN_STEPS, DT, **kw)


def _noisy(rng, Wd, Hd, nb, P=2):
    c = rng.poisson(2.0, size=(nb, Wd * Hd, P)).astype(np.uint32)
    for m in range(Wd * Hd):
        x, y = m % Wd, m // Wd
        for k0 in range(20, nb - 60, 110):
            k = k0 + 2 * x + y + int(rng.integers(0, 3))
            c[k:k + int(rng.integers(20, 50)), m, 0] += np.uint32(rng.poisson(30.0))
    return c


def _planted(Wd, Hd, nb, up_bin, up_len=15):
    c = np.ones((nb, Wd * Hd, 2), np.uint32)
    c[:, :, 1] = 0
    for m in range(Wd * Hd):
        k = up_bin(m % Wd, m // Wd)
        c[k:k + up_len, m, 0] = 50
    return c


@pytest.mark.parametrize("case", ["plane", "diagonal", "two_waves"])
def test_planted_waves_match_oracle(L, case):
    _say("waves planted", case)
    if case == "plane":
        Wd, Hd, nb = 9, 5, 120
        c = _planted(Wd, Hd, nb, lambda x, y: 20 + 2 * x)
    elif case == "diagonal":
        Wd, Hd, nb = 8, 8, 100
        c = _planted(Wd, Hd, nb, lambda x, y: 10 + x + 2 * y)
    else:
        Wd, Hd, nb = 6, 4, 160
        c = np.maximum(_planted(Wd, Hd, nb, lambda x, y: 20 + x, 10),
                       _planted(Wd, Hd, nb, lambda x, y: 90 + 2 * x, 10))
    got = _on_gpu(L, c, Wd, Hd, noise_var=0.0)
    ref = O.waves(c, Wd, Hd, BIN_STEPS, DT, noise_var=0.0)
    _compare(got, ref)


@pytest.mark.parametrize("Wd,Hd,nb,P,noise,bin0,mins", [
    (7, 6, 600, 2, 0.5, 0, (2, 2, 1)),
    (13, 5, 1000, 3, 0.5, 12345, (3, 2, 10)),     # ragged grid, three pops
    (4, 4, 4096, 2, 0.5, 7, (2, 2, 1)),           # the longest window
    (5, 3, 1, 2, 0.5, 0, (1, 1, 1)),              # one bin: nothing to find
    (90, 90, 48, 2, 0.5, 3, (2, 2, 1)),           # 8100 modules
    (128, 64, 40, 1, 0.5, 0, (1, 1, 1)),          # the largest grid, 8192 modules
    (11, 9, 300, 2, 2.0, (1 << 32) + 5, (1, 1, 1)),  # bins past 2^32, loud noise
])
def test_noisy_activity_matches_oracle(L, Wd, Hd, nb, P, noise, bin0, mins):
    _say("waves noisy", Wd, Hd, nb, P, noise, bin0, mins)
    rng = np.random.default_rng(Wd * 1000 + nb)
    c = _noisy(rng, Wd, Hd, nb, P)
    md, mu, mm = mins
    got = _on_gpu(L, c, Wd, Hd, bin0=bin0, noise_var=noise, seed=11, min_down=md,
                  min_up=mu, min_modules=mm)
    ref = O.waves(c, Wd, Hd, BIN_STEPS, DT, bin0=bin0, noise_var=noise, seed=11,
                  min_down=md, min_up=mu, min_modules=mm)
    _compare(got, ref)
    assert got["bin0"] == bin0 and got["n_bins"] == nb


@pytest.mark.parametrize("regime", ["swa", "fbi"])
def test_rate_bins_of_a_simulation_match_oracle(L, regime):
    """The handle's own bins (two-population SWA grid, and the F/B/I model
    with its three populations), analysed in place, then drained and given
    to the oracle."""
    _say("waves of a simulation", regime)
    if regime == "swa":
        p = dict(W.grid(6, 6, "swa"), rate_bins_cap=2048)
    else:
        p = dict(W.fbi(5, 4, "sw", scale=0.2), rate_bins_cap=2048)
    net = L.dpsnn_build(p, 3)
    L.dpsnn_step(net, 12000)          # 1.2 s: 240 bins of 5 ms
    got = L.dpsnn_waves(net, noise_var=0.5, seed=2)
    got_last = L.dpsnn_waves(net, n_bins=100, noise_var=0.5, seed=2)
    counts = L.dpsnn_read_rates(net)
    net.close()
    assert counts.shape[0] == 240 and got["n_bins"] == 240 and got["bin0"] == 0
    ref = O.waves(counts, p["grid_w"], p["grid_h"], BIN_STEPS, DT, noise_var=0.5, seed=2)
    _compare(got, ref)
    ref_last = O.waves(counts[140:], p["grid_w"], p["grid_h"], BIN_STEPS, DT, bin0=140,
                       noise_var=0.5, seed=2)
    _compare(got_last, ref_last)
    assert got_last["bin0"] == 140


def test_batch_network_index(L):
    """Network k of a batch handle: its own modules and grid."""
    _say("waves batch")
    ps = [dict(W.grid(3, 2, "swa"), rate_bins_cap=1024),
          dict(W.grid(4, 5, "aw"), rate_bins_cap=1024)]
    net = L.dpsnn_build_batch(ps, [1, 2])
    L.dpsnn_step(net, 5000)
    got = L.dpsnn_waves(net, net_index=1, noise_var=0.5, seed=4)
    rates = L.dpsnn_read_rates(net)
    info = L.dpsnn_net_info(net, 1)
    net.close()
    mb, m = info["module_base"], info["n_modules"]
    ref = O.waves(rates[:, mb:mb + m, :], 4, 5, BIN_STEPS, DT, noise_var=0.5, seed=4)
    _compare(got, ref)


@pytest.mark.timeout(300)
def test_slow_waves_speed_grows_with_lambda(L):
    """The F/B/I "swv" state on 24x24 modules: after 1 s of transient, 8 s
    hold Up states that cross the whole grid as waves (about one every
    3 s), and their speed (Eq. 4 averaged over the modules, Sec. 2.3) grows
    with the decay length lambda of Eq. 1, as Sec. 3.3.2 reports.  Analysis
    without added noise, Down and Up dwell of 4 bins, waves of at least 50
    modules."""
    import torch

    def waves(state, lam, seed=1):
        with torch.cuda.stream(torch.cuda.Stream()):
            net = L.dpsnn_build(W.fbi(24, 24, state, lam=lam, rate_bins_cap=2048), seed)
            L.dpsnn_step(net, 10000)
            L.dpsnn_read_rates(net)
            L.dpsnn_step(net, 80000)
            r = L.dpsnn_waves(net, noise_var=0.0, seed=1, min_down=4, min_up=4, min_modules=50)
            net.close()
        measured = r["speed"] > 0 if r["n_waves"] else np.zeros(0, bool)
        _say("waves", state, lam, r["n_transitions"], r["n_waves"], int(measured.sum()),
             float(r["mean_speed"]))
        return int(measured.sum()), float(r["mean_speed"])

    n4, v4 = waves("swv", 0.4)
    n7, v7 = waves("swv", 0.7)
    assert n4 >= 2 and n7 >= 2
    assert v7 > 2.0 * v4 > 0.0
