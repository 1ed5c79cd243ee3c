/*
 * dpsnn_oracle.h -- plain CPU oracle for the DPSNN cortical-grid hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this code: it exists so that tests, the smoke check and the
 * benchmark's CPU-baseline leg can check the HIP library against an
 * independent, slow, obviously-correct implementation.  It shares no source,
 * header, table generator or helper with the library; both are written from
 * the paper (Pastorelli et al., "Scaling of a large-scale simulation of
 * synchronous slow-wave and asynchronous awake-like activity of a cortical
 * model with long-range interconnections", Front. Syst. Neurosci. 2019).
 *
 * What it computes (paper references by section / equation / table):
 *   - the 2-D grid of modules of K point-like LIF neurons, 4:1 exc:inh, or
 *     the foreground / background / inhibitory populations (Sec. 2.2);
 *   - inter-module connectivity with probability decaying as exp(-d/lambda)
 *     (Eq. 1), Gaussian efficacies (Sec. 2.2), integer synaptic delays;
 *   - the LIF neuron with spike-frequency adaptation (Eq. 2, Table S1),
 *     integrated with its exact propagator on a dt grid;
 *   - external Poisson drive with Gaussian efficacy generated on the fly,
 *     with no stored synapses (Sec. 2.1, neuron data structure paragraph);
 *   - spike delivery through per-delay input queues (Sec. 2.1.1, steps 3-4),
 *     here as fixed-point ring slots so that summation order cannot matter;
 *   - population spike counts in 5 ms bins (Sec. 2.3).
 *
 * Two precisions:
 *   ORC_MIRROR32 - neuron state in binary32, inputs summed in fixed point,
 *                  the operation order fixed below; the HIP FP32-weight path
 *                  must reproduce its spike rasters bit for bit.
 *   ORC_EXACT64  - the same random draws (targets, delays, table indices,
 *                  Poisson counts) but unrounded binary64 efficacies, binary64
 *                  input sums and binary64 state: the error reference.
 */
#ifndef DPSNN_ORACLE_H
#define DPSNN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_WF32 = 0, ORC_WF16 = 1, ORC_WI8 = 2 };
enum { ORC_MIRROR32 = 0, ORC_EXACT64 = 1 };

enum {
  ORC_OK = 0,
  ORC_E_INVAL = -1,
  ORC_E_NOMEM = -2,
  ORC_E_RANGE = -4   /* a per-step fixed-point input sum left int32 range */
};

/* Philox counter word 3 carries the stream tag (low byte) and a block index. */
enum { ORC_TAG_SYN = 1, ORC_TAG_EXT = 2, ORC_TAG_EXTJ = 3, ORC_TAG_INIT = 4 };

/* Network parameters.  Index [0] = excitatory, [1] = inhibitory population.
 * Units: mV, ms, Hz; lambda and distances in inter-module distance units. */
typedef struct orc_params {
  int32_t grid_w, grid_h;     /* modules per row / column                    */
  int32_t K;                  /* neurons per module (1250 in the paper)      */
  int32_t K_out;              /* recurrent out-degree of every neuron        */
  double  frac_exc;           /* excitatory fraction of each module (0.8)    */
  double  frac_local[2];      /* share of a source's synapses kept local     */
  double  lambda;             /* connectivity decay length, Eq. 1            */
  int32_t torus;              /* 1: periodic grid; 0: open boundaries        */
  int32_t d_min, d_max;       /* synaptic delays, in steps                   */
  double  dt_ms;              /* integration step                            */
  int32_t weight_dtype;       /* ORC_WF32 / ORC_WF16 / ORC_WI8               */
  int32_t acc_bits;           /* 32 or 64: width of the fixed-point ring     */
  int32_t q_frac_bits;        /* Q: fractional bits of the fixed point       */
  double  J_mean[2], J_sd[2]; /* recurrent efficacy by SOURCE population     */
  double  nu_ext_hz[2];       /* total external Poisson rate by target pop   */
  double  Jext_mean[2], Jext_sd[2];
  double  tau_m[2], E[2], V_th[2], V_r[2], tau_arp[2];
  double  alpha_c[2], tau_c[2], gc[2]; /* gc = g_c / C_m in 1/ms           */
  double  I_const[2];         /* constant drive in mV/ms (tests only)        */
  int32_t rate_bin_steps;     /* steps per population-rate bin               */
  /* Population model of Sec. 2.2 (n_pops = 2..4; 0 = the two-population
   * model above).  Module neurons are split into consecutive populations of
   * pop_size[] (sum K); a neuron of population s projects n_syn[t][s]
   * synapses into population t: excitatory sources (pop_exc = 1) to a module
   * drawn with probability proportional to exp(-d/lambda) over all modules
   * including its own (Eq. 1 from d = 0), inhibitory sources to their own
   * module.  Efficacy N(J_mean_ts[t][s], J_sd_ts[t][s]).  Boundaries open
   * (open_boundary = 1) or periodic.  The per-population arrays replace
   * frac_exc, frac_local, J_*, nu_ext_hz, Jext_*, tau_m, E, V_th, V_r,
   * tau_arp, alpha_c, tau_c, gc and I_const; K_out must equal every
   * population's total out-degree. */
  int32_t n_pops;
  int32_t open_boundary;
  int32_t pop_size[4];
  int32_t pop_exc[4];
  int32_t n_syn[4][4];
  double  J_mean_ts[4][4], J_sd_ts[4][4];
  double  p_nu_ext_hz[4], p_Jext_mean[4], p_Jext_sd[4];
  double  p_tau_m[4], p_E[4], p_V_th[4], p_V_r[4], p_tau_arp[4];
  double  p_alpha_c[4], p_tau_c[4], p_gc[4], p_I_const[4];
  /* Spike-timing-dependent plasticity (Sec. 2.1; off in the paper's
   * experiments).  plastic = 1 makes every synapse of an excitatory source
   * plastic (binary32 efficacies only).  A synapse keeps the step of its
   * last activation and a low-pass filtered plasticity signal y; at each
   * activation (a spike of its source, at the emission step ta) y decays by
   * exp(-lag / tau_y), gains A_plus exp(-(tp - t_act) / tau_plus) decayed
   * from tp to ta when the target's last spike tp came after the previous
   * activation t_act (LTP), and loses A_minus exp(-(ta - tp) / tau_minus)
   * for the target's last spike tp <= ta (LTD).  Every stdp_update_steps
   * steps each plastic efficacy becomes clip(w + eta y(T), 0, w_max) and y
   * is reset.  Lags of stdp_update_steps steps or more contribute 0. */
  int32_t plastic, stdp_update_steps;
  double  stdp_A_plus, stdp_A_minus;     /* mV of plasticity signal        */
  double  stdp_tau_plus, stdp_tau_minus, stdp_tau_y;  /* ms                */
  double  stdp_eta, stdp_w_max;          /* gain; largest efficacy (mV)    */
} orc_params;

typedef struct orc_net orc_net;

/* Counter-based generator of Salmon et al., "Parallel random numbers: as
 * easy as 1, 2, 3" (SC'11): Philox4x32 with 10 rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);

/* Standard normal quantile by bisection on 0.5*erfc(-x/sqrt 2). */
double orc_normal_quantile(double p);

/* binary64 -> binary16 bit pattern, round to nearest even. */
uint16_t orc_f64_to_f16(double x);
double   orc_f16_to_f64(uint16_t h);

/* Build a network: tables, initial state, (optionally) the stored rows.
 * store_rows = 0 regenerates a source's row from Philox whenever it spikes.
 * Returns NULL and sets *err on failure. */
orc_net* orc_create(const orc_params* p, uint64_t seed, int32_t mode,
                    int32_t store_rows, int32_t* err);
void     orc_free(orc_net* n);

int64_t  orc_n_neurons(const orc_net* n);
int32_t  orc_n_slots(const orc_net* n);
int64_t  orc_time(const orc_net* n);
int32_t  orc_status(const orc_net* n);

/* Copy a host table into out (cap bytes).  Returns the table's size in bytes
 * (also when out is NULL), or ORC_E_INVAL for an unknown name. */
int64_t  orc_table(const orc_net* n, const char* name, void* out, int64_t cap);

/* One row of the connectivity, sorted stably by delay (draw order kept
 * within a delay).  Arrays hold K_out entries; doff holds d_max-d_min+2
 * offsets (doff[k] = first position with delay >= d_min + k); blk (may be
 * NULL) receives each synapse's block: the index of its target population
 * in the source population's projection list, which selects the efficacy
 * table. */
int32_t  orc_gen_row(const orc_net* n, int64_t s, int32_t* tgt,
                     uint8_t* delay, uint16_t* widx, uint16_t* doff);
int32_t  orc_gen_row_blocks(const orc_net* n, int64_t s, int32_t* tgt,
                            uint8_t* delay, uint16_t* widx, uint16_t* doff,
                            uint8_t* blk);
/* Populations per module (2 for the two-population model). */
int32_t  orc_n_pops(const orc_net* n);

/* External Poisson input of neuron i at step t: count and the fixed-point
 * (MIRROR32) / binary64 (EXACT64) sum of its efficacies. */
int32_t  orc_ext_input(const orc_net* n, int64_t i, int64_t t,
                       int64_t* fix_sum, double* f64_sum);

int32_t  orc_step(orc_net* n, int64_t n_steps);

/* State access (tests).  V and c as binary64 (exact copies of binary32
 * values in MIRROR32); ref as int32.  Ring: D*N values, slot-major; int64 in
 * MIRROR32, binary64 in EXACT64. */
int32_t  orc_get_state(const orc_net* n, double* V, double* c, int32_t* ref);
int32_t  orc_set_state(orc_net* n, const double* V, const double* c,
                       const int32_t* ref);
int32_t  orc_get_ring(const orc_net* n, int64_t* ring_fix, double* ring_f64);
int32_t  orc_set_ring(orc_net* n, const int64_t* ring_fix, const double* ring_f64);
/* Move the step counter (state restored from elsewhere, e.g. to re-run
 * one step of a longer simulation). */
int32_t  orc_set_time(orc_net* n, int64_t t);

/* Spikes since creation as (step, id) in the order they were emitted
 * (step-major, id ascending). Returns the count; copies min(count, cap). */
int64_t  orc_spikes(const orc_net* n, int32_t* step, int32_t* id, int64_t cap);
/* Population counts: [bins][modules][n_pops]; returns number of bins
 * touched. */
int64_t  orc_rates(const orc_net* n, uint32_t* counts, int64_t cap_bins);

/* Plasticity state of row s, in the oracle's row order (that of
 * orc_gen_row_blocks): last activation step (-1: never), signal y and
 * efficacy w of each synapse (binary32 values widened in MIRROR32 mode).
 * ORC_E_INVAL without plasticity. */
int32_t  orc_plasticity(const orc_net* n, int64_t s, int32_t* t_act, double* y, double* w);

#ifdef __cplusplus
}
#endif
#endif
