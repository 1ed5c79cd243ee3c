"""Parameter sets of the synthetic workloads (plain data, no arithmetic).

Both the HIP library binding and the CPU oracle take these dicts; the keys
are the fields of the C parameter structs, pairs are [excitatory,
inhibitory].  Units: mV, ms, Hz, inter-module distance units for lambda.

Neuron constants follow Table S1 of the paper (tau_m 20/10 ms, E = 0,
V_theta = 20 mV, V_r = 15 mV, tau_arp 2/1 ms, alpha_c = 1 mV,
g_c/C_m = 0.02 nS/pF = 0.02 1/ms, no adaptation for inhibitory neurons).
The network structure of the workloads is a fixed 80/20 split, out-degree
1000 with half the synapses local, exponential remote connectivity (Eq. 1)
on a torus, delays of 1-20 steps of 0.1 ms, and Gaussian efficacies
N(0.5, 0.1) mV from excitatory and N(-2.0, 0.4) mV from inhibitory sources.
"""
import copy

# Slow-wave (SWA) regime: strong adaptation, tau_c = 500 ms.
_SWA = dict(
    grid_w=2, grid_h=2, K=1250, K_out=1000, frac_exc=0.8,
    frac_local=[0.5, 0.5], torus=1, d_min=1, d_max=20, dt_ms=0.1,
    weight_dtype="f32", acc_bits=32, q_frac_bits=16,
    J_mean=[0.5, -2.0], J_sd=[0.1, 0.4],
    nu_ext_hz=[1000.0, 1000.0], Jext_mean=[0.86, 1.12], Jext_sd=[0.172, 0.224],
    tau_m=[20.0, 10.0], E=[0.0, 0.0], V_th=[20.0, 20.0], V_r=[15.0, 15.0],
    tau_arp=[2.0, 1.0], alpha_c=[1.0, 0.0], tau_c=[500.0, 500.0],
    gc=[0.02, 0.0], I_const=[0.0, 0.0], rate_bin_steps=50,
)
_SWA["lambda"] = 1.0


def swa(**over) -> dict:
    p = copy.deepcopy(_SWA)
    p.update(over)
    return p


def aw(**over) -> dict:
    """Asynchronous-wake regime: adaptation x0.1 and a higher external rate."""
    p = swa(gc=[0.002, 0.0], nu_ext_hz=[1500.0, 1500.0])
    p.update(over)
    return p


def grid(w: int, h: int, regime: str = "swa", **over) -> dict:
    base = swa if regime == "swa" else aw
    return base(grid_w=w, grid_h=h, **over)


def tiny(w: int = 2, h: int = 2, K: int = 16, K_out: int = 8, **over) -> dict:
    """Small grids for exhaustive checks (brute-force delivery, rasters)."""
    p = swa(grid_w=w, grid_h=h, K=K, K_out=K_out, d_max=5)
    p.update(over)
    return p


def stdp(**over) -> dict:
    """Plasticity fields (Sec. 2.1; the paper gives no constants): pair
    windows of 20 ms with slightly stronger depression, a 1 s low-pass filter
    and a 1 s update period, efficacies kept in [0, 1] mV."""
    p = dict(plastic=1, stdp_update_steps=10000, stdp_A_plus=0.01, stdp_A_minus=0.0105,
             stdp_tau_plus=20.0, stdp_tau_minus=20.0, stdp_tau_y=1000.0, stdp_eta=1.0,
             stdp_w_max=1.0)
    p.update(over)
    return p


def sweep(n: int = 64, seed: int = 1):
    """Batched sweep: n networks, grids uniform in {4x4, 8x8, 12x12, 16x16}
    modules, adaptation g_c/C_m log-uniform on [0.002, 0.02] 1/ms (AW to
    SWA), lambda in {1, 2}, binary16 efficacies.  Returns (params, seeds)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sides = rng.choice([4, 8, 12, 16], size=n)
    gcs = np.exp(rng.uniform(np.log(0.002), np.log(0.02), size=n))
    lams = rng.choice([1.0, 2.0], size=n)
    params = [swa(grid_w=int(s), grid_h=int(s), gc=[float(g), 0.0], weight_dtype="f16",
                  **{"lambda": float(lam)}) for s, g, lam in zip(sides, gcs, lams)]
    return params, list(range(1, n + 1))


def grid96(regime: str) -> dict:
    """96x96 grid (11.52M neurons), lambda = 2, int8 efficacies, int64 slots."""
    return grid(96, 96, regime, **{"lambda": 2.0, "weight_dtype": "i8",
                                   "acc_bits": 64, "q_frac_bits": 32})


# ---------------------------------------------------------------------------
# Population model of Sec. 2.2 and Table S1: per module 250 foreground (F),
# 750 background (B) excitatory and 250 inhibitory (I) neurons; every neuron
# projects 0.9 K_t synapses into each population t (1125 in all);
# excitatory projections reach any module with probability proportional to
# exp(-d / lambda) (Eq. 1 from d = 0), inhibitory ones stay in the module;
# open boundaries.  Efficacies J_{t,s} of Table S1 with SD 0.25 |J|; the SW
# row's inhibitory entries repeat the external-rate row (garbled) and are
# read as the AW rows' -1.5 mV.  External drive: 400 Poisson trains of
# 3.17 / 3.17 / 3.0 Hz with the J_{t,ext} of the state.
# "swv" is not a state of Table S1: the SW row with the excitatory
# efficacies x1.15, inhibitory ones of -0.8 mV and g_w/C_m = 0.01 1/ms, a
# state whose modules alternate between Down and Up states and whose Up
# states travel across the grid as waves (found by a parameter search; the
# paper does not print the parameters of its wave simulations).
_FBI_J = {
    #        F<-F   B<-F   I<-F   F<-B   B<-B   I<-B   F<-I  B<-I  I<-I
    "sw": [0.600, 0.382, 0.560, 0.382, 0.429, 0.560, -1.5, -1.5, -1.5],
    "aw28": [0.515, 0.412, 0.560, 0.412, 0.429, 0.560, -1.5, -1.5, -1.5],
    "aw88": [0.515, 0.412, 0.560, 0.412, 0.429, 0.560, -1.5, -1.5, -1.5],
    "swv": [0.690, 0.4393, 0.644, 0.4393, 0.49335, 0.644, -0.8, -0.8, -0.8],
}
_FBI_JEXT = {"sw": [0.832, 0.858, 1.120], "aw28": [0.858, 0.858, 1.120],
             "aw88": [1.416, 1.416, 1.120], "swv": [0.832, 0.858, 1.120]}
_FBI_GC = {"swv": 0.01}  # g_w / C_m of F and B (1/ms); Table S1: 0.02


def fbi(w: int, h: int, state: str = "sw", lam: float = 0.5, scale: float = 1.0,
        **over) -> dict:
    """The F/B/I network of w x h modules in state "sw", "aw28", "aw88" or
    "swv" (propagating slow waves, see above);
    scale < 1 shrinks the populations (and out-degrees) for quick tests."""
    j = _FBI_J[state]
    # J_mean_ts[t][s]: target t, source s (order F, B, I)
    jts = [[j[0], j[3], j[6]], [j[1], j[4], j[7]], [j[2], j[5], j[8]]]
    sizes = [round(250 * scale), round(750 * scale), round(250 * scale)]
    nsyn = [[round(0.9 * sizes[t])] * 3 for t in range(3)]
    p = swa(grid_w=w, grid_h=h, K=sum(sizes), K_out=sum(r[0] for r in nsyn),
            n_pops=3, open_boundary=1, pop_size=sizes, pop_exc=[1, 1, 0],
            n_syn=nsyn, J_mean_ts=jts,
            J_sd_ts=[[0.25 * abs(x) for x in row] for row in jts],
            p_nu_ext_hz=[400 * 3.17, 400 * 3.17, 400 * 3.0],
            p_Jext_mean=_FBI_JEXT[state],
            p_Jext_sd=[0.25 * x for x in _FBI_JEXT[state]],
            p_tau_m=[20.0, 20.0, 10.0], p_E=[0.0, 0.0, 0.0], p_V_th=[20.0] * 3,
            p_V_r=[15.0] * 3, p_tau_arp=[2.0, 2.0, 1.0], p_alpha_c=[1.0, 1.0, 0.0],
            p_tau_c=[1000.0] * 3, p_gc=[_FBI_GC.get(state, 0.02)] * 2 + [0.0],
            p_I_const=[0.0] * 3)
    p["lambda"] = lam
    p.update(over)
    return p
