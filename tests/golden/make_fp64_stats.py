"""Write fp64_stats_2x2.json: statistics of the binary64 oracle (EXACT64
mode) on the 2x2 grid of 1250-neuron modules, SWA and AW, seeds
1-5, 2 s of biological time each: mean rates after a 0.5 s transient,
up-state and burst frequencies and per-neuron spike-count histograms.

Calls only the oracle package (its EXACT64 simulation and the binary64
reductions of oracle/stats.py); run from the repository root:
  python tests/golden/make_fp64_stats.py
"""
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

STEPS = 20000
SEEDS = [1, 2, 3, 4, 5]


def one(job):
    import oracle as O
    from oracle import stats
    from paper_1902_08410_amd import workloads as W
    regime, seed = job
    p = W.swa() if regime == "swa" else W.aw()
    o = O.Oracle(p, seed, mode=O.EXACT64, store_rows=True)
    o.step(STEPS)
    st, ids = o.spikes()
    K, Kexc = p["K"], round(p["frac_exc"] * p["K"])
    s = stats.summary(o.rates(), st, ids, o.N, K, Kexc, p["rate_bin_steps"] * p["dt_ms"],
                         p["dt_ms"], STEPS)
    return regime, seed, s


def main():
    jobs = [(r, s) for r in ("swa", "aw") for s in SEEDS]
    with mp.Pool(min(8, len(jobs))) as pool:
        res = pool.map(one, jobs)
    out = {"steps": STEPS, "seeds": SEEDS, "config": "2x2 grid, K=1250, K_out=1000",
           "mode": "EXACT64", "runs": {}}
    for regime, seed, s in res:
        out["runs"].setdefault(regime, {})[str(seed)] = s
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp64_stats_2x2.json")
    json.dump(out, open(path, "w"))
    for regime in ("swa", "aw"):
        for seed in SEEDS:
            s = out["runs"][regime][str(seed)]
            print(regime, seed, round(s["rate_exc_hz"], 3), round(s["rate_inh_hz"], 3),
                  round(s["up_freq_hz"], 3), round(s["burst_freq_hz"], 3))


if __name__ == "__main__":
    main()
