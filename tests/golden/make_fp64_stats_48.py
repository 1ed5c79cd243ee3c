"""Write fp64_stats_48x48.json: statistics of the binary64 oracle (EXACT64
mode: the same random draws as the library, unrounded binary64 efficacies,
sums and state) on the 48x48 grid of 1250-neuron modules (2.88M neurons,
2.88G synapses), SWA and AW, lambda in {0.5, 1, 2, 4}, seeds 1 and 2,
1.5 s of biological time each: mean rates after a 0.5 s transient, Up-state
(>= 50 ms) and population-burst (>= 10 ms) frequencies, and the per-neuron
spike-count histogram of the last 1.0 s.

Calls only the oracle package (its EXACT64 simulation and the binary64
reductions of oracle/stats.py).  Each run writes fp64_48/<job>.json when it
ends, so that an interrupted generation resumes; the combined file is
written once every run is there.  Run from the repository root (several
hours of CPU: about 0.5 s per step and run, 8 runs at a time):
  python tests/golden/make_fp64_stats_48.py [processes]
"""
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "fp64_48")

STEPS = 15000
SKIP_S = 0.5
SEEDS = [1, 2]
LAMBDAS = [0.5, 1.0, 2.0, 4.0]


def job_name(regime, lam, seed):
    return f"{regime}_l{lam:g}_s{seed}"


def params(regime, lam):
    from paper_1902_08410_amd import workloads as W
    return W.grid(48, 48, regime, **{"lambda": lam})


def one(job):
    import oracle as O
    from oracle import stats
    regime, lam, seed = job
    path = os.path.join(OUT_DIR, job_name(*job) + ".json")
    if os.path.exists(path):
        return job, json.load(open(path))
    p = params(regime, lam)
    o = O.Oracle(p, seed, mode=O.EXACT64, store_rows=False)
    t0 = time.time()
    for k in range(0, STEPS, 500):
        o.step(500)
        print(f"{job_name(*job)}: {k + 500} steps, {time.time() - t0:.0f} s", flush=True)
    st, ids = o.spikes()
    K, Kexc = p["K"], round(p["frac_exc"] * p["K"])
    s = stats.summary(o.rates(), st, ids, o.N, K, Kexc, p["rate_bin_steps"] * p["dt_ms"],
                      p["dt_ms"], STEPS, skip_s=SKIP_S)
    s["oracle_seconds"] = time.time() - t0
    o.close()
    tmp = path + ".tmp"
    json.dump(s, open(tmp, "w"))
    os.replace(tmp, path)
    return job, s


def main():
    os.makedirs(OUT_DIR, exist_ok=True)
    nproc = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    jobs = [(r, lam, s) for s in SEEDS for lam in LAMBDAS for r in ("swa", "aw")]
    with mp.Pool(nproc) as pool:
        res = list(pool.imap_unordered(one, jobs))
    out = {"steps": STEPS, "skip_s": SKIP_S, "seeds": SEEDS, "lambdas": LAMBDAS,
           "config": "48x48 grid, K=1250, K_out=1000, torus", "mode": "EXACT64", "runs": {}}
    for (regime, lam, seed), s in res:
        out["runs"].setdefault(regime, {}).setdefault(f"{lam:g}", {})[str(seed)] = s
    json.dump(out, open(os.path.join(HERE, "fp64_stats_48x48.json"), "w"))
    for (regime, lam, seed), s in sorted(res):
        print(regime, lam, seed, round(s["rate_exc_hz"], 3), round(s["rate_inh_hz"], 3),
              round(s["up_freq_hz"], 3), round(s["burst_freq_hz"], 3))


if __name__ == "__main__":
    main()
