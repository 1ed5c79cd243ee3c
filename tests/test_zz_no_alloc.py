"""The allocation-free slow-wave analysis (dpsnn_waves_counts_static, for
callers that cannot allocate device memory) against the allocating entry
point dpsnn_waves_counts, through the C-ABI: identical transitions, waves,
speeds and mean speed on two calls in a row, the second with a smaller
input (the fixed scratch keeps the first call's contents), and the limits
of the fixed buffer reported as DPSNN_E_SCRATCH."""
import sys

import numpy as np
import pytest

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


def _noisy(rng, Wd, Hd, nb, P):
    c = rng.poisson(2.0, size=(nb, Wd * Hd, P)).astype(np.uint32)
    for m in range(Wd * Hd):
        x, y = m % Wd, m // Wd
        for k0 in range(20, nb - 60, 110):
            k = k0 + 2 * x + y + int(rng.integers(0, 3))
            c[k:k + int(rng.integers(20, 50)), m, 0] += np.uint32(rng.poisson(30.0))
    return c


def _same(a, b):
    assert a["n_transitions"] == b["n_transitions"] and a["n_waves"] == b["n_waves"]
    assert a["bin0"] == b["bin0"] and a["n_bins"] == b["n_bins"]
    for k in ("module", "T", "wave", "n", "t0"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(np.isnan(a["speed"]), np.isnan(b["speed"]))
    ok = ~np.isnan(a["speed"])
    assert np.array_equal(a["speed"][ok], b["speed"][ok])
    assert (np.isnan(a["mean_speed"]) and np.isnan(b["mean_speed"])) or \
        a["mean_speed"] == b["mean_speed"]


def test_static_scratch_matches_allocating_entry_point(L):
    import torch
    rng = np.random.default_rng(17)
    cases = [(24, 24, 1200, 3, 12345, (2, 2, 10)),    # F/B/I-sized grid, 6 s of bins
             (7, 6, 300, 2, 0, (1, 1, 1))]            # then a smaller one
    for Wd, Hd, nb, P, bin0, (md, mu, mm) in cases:
        _say("static scratch", Wd, Hd, nb, P)
        c = _noisy(rng, Wd, Hd, nb, P)
        t = torch.from_numpy(c.view(np.int32)).cuda()
        kw = dict(bin0=bin0, noise_var=0.5, seed=3, min_down=md, min_up=mu, min_modules=mm)
        got = L.dpsnn_waves_counts_static(t, Wd, Hd, BIN_STEPS, DT, **kw)
        ref = L.dpsnn_waves_counts(t, Wd, Hd, BIN_STEPS, DT, **kw)
        assert ref["n_transitions"] > 100 and ref["n_waves"] > 1
        _same(got, ref)
        again = L.dpsnn_waves_counts_static(t, Wd, Hd, BIN_STEPS, DT, **kw)
        _same(again, ref)


def test_static_scratch_limits(L):
    import torch
    _say("static scratch limits")
    # a count above 65535 in one bin: the log table of the fixed buffer ends there
    c = np.ones((50, 4, 2), np.uint32)
    c[10, 2, 0] = 70000
    t = torch.from_numpy(c.view(np.int32)).cuda()
    with pytest.raises(L.DpsnnError) as e:
        L.dpsnn_waves_counts_static(t, 2, 2, BIN_STEPS, DT)
    assert e.value.code == -8
    # the allocating entry point takes it, and the fixed buffer still works after
    assert L.dpsnn_waves_counts(t, 2, 2, BIN_STEPS, DT)["n_bins"] == 50
    c[10, 2, 0] = 60
    t = torch.from_numpy(c.view(np.int32)).cuda()
    _same(L.dpsnn_waves_counts_static(t, 2, 2, BIN_STEPS, DT),
          L.dpsnn_waves_counts(t, 2, 2, BIN_STEPS, DT))
