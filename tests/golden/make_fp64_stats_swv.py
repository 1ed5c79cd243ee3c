"""Write fp64_stats_swv4x4.json: statistics of the binary64 oracle (EXACT64:
the same random draws as the library, binary64 efficacies, sums and state)
for the F/B/I population model in its "swv" state (slow waves) on 4x4
modules, seeds 1-4, 6 s each: mean rate of each population and the Up
states (>= 50 ms) of the module activity after 1 s of transient, and the
per-neuron spike-count histogram of the last 5 s.

Calls only the oracle package (its EXACT64 simulation and the binary64
reductions of oracle/stats.py).  Run from the repository root (a few CPU
minutes, four runs at a time):
  python tests/golden/make_fp64_stats_swv.py
"""
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))

SIDE = 4
STEPS = 60000
SKIP_S = 1.0
SEEDS = [1, 2, 3, 4]


def params():
    from paper_1902_08410_amd import workloads as W
    return W.fbi(SIDE, SIDE, "swv")


def one(seed):
    import oracle as O
    from oracle import stats
    p = params()
    o = O.Oracle(p, seed, mode=O.EXACT64, store_rows=False)
    o.step(STEPS)
    counts = o.rates()
    st, ids = o.spikes()
    bin_ms = p["rate_bin_steps"] * p["dt_ms"]
    t0 = int(round(SKIP_S * 1e3 / p["dt_ms"]))
    hist = stats.neuron_rate_hist(ids[st >= t0], o.N)
    last = int(hist.nonzero()[0].max()) + 1 if hist.any() else 1
    up = stats.up_state_stats(counts, bin_ms, SKIP_S, 50.0)
    out = {"rates_hz": stats.population_rates_hz(counts, p["pop_size"], bin_ms, SKIP_S),
           "up_freq_hz": up["freq_hz"], "mean_up_ms": up["mean_up_ms"],
           "up_fraction": up["up_fraction"], "count_hist": hist[:last].tolist()}
    o.close()
    return seed, out


def main():
    with mp.Pool(len(SEEDS)) as pool:
        res = dict(pool.map(one, SEEDS))
    out = {"side": SIDE, "steps": STEPS, "skip_s": SKIP_S, "seeds": SEEDS, "state": "swv",
           "mode": "EXACT64", "runs": {str(s): res[s] for s in SEEDS}}
    json.dump(out, open(os.path.join(HERE, "fp64_stats_swv4x4.json"), "w"))
    for s in SEEDS:
        r = res[s]
        print(s, [round(x, 3) for x in r["rates_hz"]], round(r["up_freq_hz"], 3),
              round(r["mean_up_ms"], 1), round(r["up_fraction"], 3))


if __name__ == "__main__":
    main()
