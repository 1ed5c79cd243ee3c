"""Pins of the slow-wave analysis oracle (Sec. 2.3, Eq. 4) on the CPU.

Planted activity whose Down-to-Up times are known in closed form: plane
waves of known speed (Eq. 4 then gives that speed exactly, central and
one-sided differences alike), a hand-worked interpolation, the dwell
rules, and the statistics of the added noise (the rate
of noise-made crossings of a known threshold follows from the normal
distribution).  The grouping into waves is checked through the properties
that define it.
"""
import math

import numpy as np
import pytest

import oracle as O

BIN_STEPS, DT = 50, 0.1          # 5 ms bins
DBIN = BIN_STEPS * DT


def planted(W, H, nb, up_bin, up_len=15, down=1, up=50, pops=2):
    """Counts [nb][W*H][pops]: population 0 of module m is at `up` from bin
    up_bin(x, y) for up_len bins, else `down`; population 1 is silent."""
    c = np.zeros((nb, W * H, pops), np.uint32)
    c[:, :, 0] = down
    for m in range(W * H):
        k = up_bin(m % W, m // W)
        if k is not None:
            c[k:k + up_len, m, 0] = up
    return c


@pytest.mark.parametrize("n", [1, 2, 3])
def test_plane_wave_along_x_has_its_planted_speed(n):
    W, H, nb = 9, 5, 120
    c = planted(W, H, nb, lambda x, y: 20 + n * x)
    r = O.waves(c, W, H, BIN_STEPS, DT, noise_var=0.0)
    # one module per n bins of 5 ms: 1000 / (5 n) modules per second
    assert len(r["speed"]) == 1 and r["n"][0] == W * H
    assert r["speed"][0] == pytest.approx(1000.0 / (n * DBIN), rel=1e-14)
    # the step from count 1 to 50 crosses the mid level halfway between
    # the bin centres: T is the bin edge
    T = dict(zip(r["module"].tolist(), r["T"].tolist()))
    for m in range(W * H):
        assert T[m] == (20 + n * (m % W)) * DBIN


def test_diagonal_wave_speed():
    W, H, nb = 8, 8, 100
    c = planted(W, H, nb, lambda x, y: 10 + x + 2 * y)
    r = O.waves(c, W, H, BIN_STEPS, DT, noise_var=0.0)
    # grad T = (1, 2) bins per module -> |grad T| = sqrt(5) * 5 ms
    assert r["speed"][0] == pytest.approx(1000.0 / (math.sqrt(5.0) * DBIN), rel=1e-14)


def test_interpolated_time():
    # one module, 12 bins: counts 0 x4, 9, 99 x3, 0 x4.  Lower median = 0,
    # Down mean 0 -> log(c_down + 1) = 0; Up bins 9, 99, 99, 99: mean 76.5,
    # rounded 77 -> theta = log(78) / 2 = 2.178 < log(10) = 2.303, so the
    # transition is at bin 4, interpolated between log(1) = 0 at bin 3 and
    # log(10) at bin 4.
    c = np.zeros((12, 1, 1), np.uint32)
    c[4, 0, 0] = 9
    c[5:8, 0, 0] = 99
    r = O.waves(c, 1, 1, BIN_STEPS, DT, noise_var=0.0, min_down=2, min_up=2)
    theta = 0.5 * math.log(78.0)
    frac = theta / math.log(10.0)
    assert len(r["T"]) == 1
    assert r["T"][0] == pytest.approx((4 - 0.5 + frac) * DBIN, rel=1e-15)


def test_dwell_rules():
    base = np.zeros((40, 1, 1), np.uint32)
    blip = base.copy()
    blip[10, 0, 0] = 80            # one bin above the threshold
    blip[20:30, 0, 0] = 80         # a real Up state
    r2 = O.waves(blip, 1, 1, BIN_STEPS, DT, noise_var=0.0, min_up=2)
    r1 = O.waves(blip, 1, 1, BIN_STEPS, DT, noise_var=0.0, min_up=1)
    assert len(r2["T"]) == 1 and len(r1["T"]) == 2
    dip = base.copy()
    dip[10:20, 0, 0] = 80
    dip[21:30, 0, 0] = 80          # one Down bin inside the Up state
    assert len(O.waves(dip, 1, 1, BIN_STEPS, DT, noise_var=0.0, min_down=2)["T"]) == 1
    assert len(O.waves(dip, 1, 1, BIN_STEPS, DT, noise_var=0.0, min_down=1)["T"]) == 2


def test_constant_activity_has_no_transitions():
    c = np.full((50, 12, 2), 7, np.uint32)
    r = O.waves(c, 4, 3, BIN_STEPS, DT, noise_var=0.5)
    assert len(r["T"]) == 0 and len(r["speed"]) == 0


def test_two_waves_in_sequence():
    W, H, nb = 6, 4, 160
    c = planted(W, H, nb, lambda x, y: 20 + x, up_len=10)
    c2 = planted(W, H, nb, lambda x, y: 90 + 2 * x, up_len=10)
    c = np.maximum(c, c2)
    r = O.waves(c, W, H, BIN_STEPS, DT, noise_var=0.0)
    assert list(r["n"]) == [W * H, W * H]
    assert r["speed"][0] == 1000.0 / DBIN and r["speed"][1] == 1000.0 / (2 * DBIN)
    assert r["t0"][0] == 20 * DBIN and r["t0"][1] == 90 * DBIN


def test_grouping_properties_on_noisy_activity():
    rng = np.random.default_rng(3)
    W, H, nb = 7, 6, 600
    c = rng.poisson(3.0, size=(nb, W * H, 2)).astype(np.uint32)
    # slow waves: Up states of 30-60 bins drifting across x
    for m in range(W * H):
        x = m % W
        for k0 in range(30, nb - 80, 140):
            k = k0 + 3 * x + int(rng.integers(0, 4))
            c[k:k + int(rng.integers(30, 60)), m, 0] += np.uint32(rng.poisson(40.0))
    r = O.waves(c, W, H, BIN_STEPS, DT, noise_var=0.5, seed=9)
    T, mod, wave = r["T"], r["module"], r["wave"]
    assert len(T) > 0
    # order: by bin, then fraction: times never decrease
    assert np.all(np.diff(T) >= 0)
    # waves are numbered in order, each a contiguous run
    assert wave[0] == 0 and np.all(np.diff(wave) >= 0) and np.all(np.diff(wave) <= 1)
    starts = np.flatnonzero(np.diff(wave)) + 1
    bounds = np.concatenate([[0], starts, [len(wave)]])
    for i in range(len(bounds) - 1):
        members = mod[bounds[i]:bounds[i + 1]]
        assert len(set(members.tolist())) == len(members)   # each module once
        if i > 0:   # a wave starts where its first module would repeat
            prev = mod[bounds[i - 1]:bounds[i]]
            assert mod[bounds[i]] in set(prev.tolist())
    assert list(r["n"]) == list(np.diff(bounds))
    assert len(r["speed"]) == len(bounds) - 1


def test_noise_variance_from_crossing_rate():
    # Down level at the median (count 0: the log term is 0 and L = eta in
    # every Down bin); one Up bin of count 54 in 256, so theta = log(55) / 2.
    # With noise variance v, eta exceeds theta with p = 1 - Phi(theta /
    # sqrt v); a crossing between two Down bins (min_down = min_up = 1)
    # happens with probability (1 - p) p.
    v = 4.0
    M, nb = 64, 4096
    c = np.zeros((nb, M, 1), np.uint32)
    c[::256, :, 0] = 54
    r = O.waves(c, 8, 8, BIN_STEPS, DT, noise_var=v, seed=5, min_down=1, min_up=1)
    theta = 0.5 * math.log(55.0)
    p = 0.5 * math.erfc(theta / math.sqrt(v) / math.sqrt(2.0))
    ups = np.arange(0, nb, 256)
    kk = np.floor(r["T"] / DBIN + 0.5).astype(int)          # bin of each crossing
    n = int((~(np.isin(kk, ups) | np.isin(kk - 1, ups))).sum())
    pairs = (nb - 1 - 2 * len(ups) + 1) * M                 # Down-Down bin pairs
    exp = pairs * p * (1 - p)
    sd = math.sqrt(exp)
    assert abs(n - exp) < 6 * sd + 0.02 * exp, (n, exp, sd)
    # the standard deviation taken for the variance would be far off
    p_bad = 0.5 * math.erfc(theta / v / math.sqrt(2.0))
    assert abs(n - pairs * p_bad * (1 - p_bad)) > 0.2 * exp


def test_threshold_is_strict():
    # Down bins 0 (c_down = 0); Up bins {2, 9 x6}: mean 56 / 7 = 8, so
    # theta = log(9) / 2, which equals log(3) in binary64: the bin of count
    # 2 sits exactly at the threshold and is not Up.  Only the rise into the
    # 9s is a transition (min_down = min_up = 1).
    assert math.log(3.0) == 0.5 * math.log(9.0)
    c = np.zeros((28, 1, 1), np.uint32)
    c[10, 0, 0] = 2
    c[12:18, 0, 0] = 9
    r = O.waves(c, 1, 1, BIN_STEPS, DT, noise_var=0.0, min_down=1, min_up=1)
    assert len(r["T"]) == 1
    frac = math.log(3.0) / math.log(10.0)
    assert r["T"][0] == pytest.approx((12 - 0.5 + frac) * DBIN, rel=1e-15)


def test_down_bins_are_at_or_below_the_lower_median():
    # an even window, half the bins Up: the lower median is the Down level
    # (the upper median would leave no Up bins at all)
    c = np.zeros((20, 1, 1), np.uint32)
    c[10:20, 0, 0] = 50
    assert len(O.waves(c, 1, 1, BIN_STEPS, DT, noise_var=0.0)["T"]) == 1


def test_down_level_is_the_rounded_mean():
    # Down bins alternate 2 and 3 (mean 2.5, rounded half up to 3), Up bins
    # 99: theta = (log(100) - log(4)) / 2 and the bin before the rise has
    # count 3, i.e. L = 0, so the crossing is halfway: T is the bin edge.
    # (With the mean floored to 2 the crossing would move by 0.04 bin.)
    c = np.array([2, 3] * 5 + [99] * 8, np.uint32).reshape(18, 1, 1)
    r = O.waves(c, 1, 1, BIN_STEPS, DT, noise_var=0.0)
    assert len(r["T"]) == 1 and r["T"][0] == 10 * DBIN
