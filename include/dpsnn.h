/*
 * dpsnn.h -- C-ABI of libdpsnn, the MI355X (gfx950) hot path of the
 * cortical-grid spiking simulation of Pastorelli et al., "Scaling of a
 * large-scale simulation of synchronous slow-wave and asynchronous
 * awake-like activity of a cortical model with long-range
 * interconnections" (Front. Syst. Neurosci. 2019).
 *
 * The network (Sec. 2.2): a W x H grid of modules of K point-like neurons,
 * a fraction frac_exc excitatory with spike-frequency adaptation, the rest
 * inhibitory; every neuron projects K_out synapses, a fixed share inside
 * its own module and the rest to other modules chosen with probability
 * proportional to exp(-d / lambda) (Eq. 1); Gaussian efficacies; integer
 * delays; an external Poisson drive generated on the fly.  The neuron is
 * the LIF neuron with adaptation of Eq. 2 with the constants of Table S1.
 *
 * One step of dt advances every neuron (Eq. 2, exact propagator), collects
 * the spikes, and pushes each spike along its synapse row into per-target
 * input slots indexed by the arrival step (the per-delay input queues of
 * Sec. 2.1.1, steps 3-4).  Inputs are summed in fixed point, so the order
 * in which concurrent additions land cannot change any result.  Rows are
 * stored sorted by target, so the events of a spike to one 1024-neuron tile
 * are contiguous: delivery reserves room for each such run in the tile's
 * inbox with one atomic (by default one atomic per target tile for the runs
 * of four spikes delivered together) and appends the events; in the next
 * step the tile
 * moves them into its per-slot queues, and sums the queue of the current
 * slot when it reaches it.  Events that find a queue full are added into
 * the slot directly.
 *
 * Conventions for every entry point:
 *  - return 0 on success or a negative DPSNN_E_* code;
 *  - pointers named host_* or documented as host memory are plain host
 *    buffers owned by the caller; the handle owns all device memory and
 *    dpsnn_free releases it;
 *  - a handle is used by one host thread at a time;
 *  - work is enqueued on the handle's stream (dpsnn_set_stream); calls that
 *    return data synchronise that stream first.
 */
#ifndef DPSNN_H
#define DPSNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPSNN_ABI_VERSION 3u

/* Error codes. */
#define DPSNN_OK 0
#define DPSNN_E_INVAL (-1)         /* invalid argument or parameter set      */
#define DPSNN_E_NOMEM (-2)         /* device or host allocation failed       */
#define DPSNN_E_DEVICE (-3)        /* a HIP runtime call failed              */
#define DPSNN_E_RANGE (-4)         /* fixed-point bound violated at build    */
#define DPSNN_E_SPIKELOG_FULL (-5) /* spike log overflowed; spikes were lost */
#define DPSNN_E_STATE (-6)         /* call not valid in the handle's state   */
#define DPSNN_E_RATES_FULL (-7)    /* rate bins would be overwritten         */
#define DPSNN_E_SCRATCH (-8)       /* request exceeds the fixed scratch      */

/* Step schedules (results are bit-identical; only speed differs). */
#define DPSNN_SCHED_FUSED 0 /* one kernel per step; a tile delivers its own
                               spikes (small networks) */
#define DPSNN_SCHED_SPLIT 1 /* neuron kernel, then a delivery kernel that
                               spreads the spiking rows over the whole GPU */
#define DPSNN_SCHED_PERSIST 2 /* the split schedule's work for many steps in
                                 one cooperative launch of resident blocks,
                                 with a grid synchronisation between update
                                 and delivery (no graphs) */

/* Stored synaptic efficacy formats. */
#define DPSNN_W_F32 0
#define DPSNN_W_F16 1
#define DPSNN_W_I8 2 /* int8 code times a per-(module, source pop) scale */

/*
 * Parameters of one network (plain data, copied at build).  Pairs are
 * [excitatory, inhibitory]: J_* by source population, everything else by
 * the population of the neuron itself.  Units: mV, ms, Hz; lambda in
 * inter-module distance units.  Defaults in brackets are those of the
 * paper's Table S1 / the benchmark workloads.
 */
typedef struct dpsnn_params {
  uint32_t abi_version;    /* must be DPSNN_ABI_VERSION                     */
  int32_t grid_w, grid_h;  /* modules per row / column                      */
  int32_t K;               /* neurons per module [1250]                     */
  int32_t K_out;           /* recurrent out-degree, <= 4096 [1000]          */
                           /* (network size W*H*K <= 2^26 neurons)          */
  double frac_exc;         /* excitatory share of a module [0.8]            */
  double frac_local[2];    /* share of a source's synapses kept local [0.5] */
  double lambda;           /* decay length of Eq. 1 [1]                     */
  int32_t torus;           /* 1: periodic grid [1]; 0: the grid has edges,
                              and each remote synapse draws among the other
                              modules that exist (Eq. 1, Sec. 2.2)        */
  int32_t d_min, d_max;    /* delays in steps, 1 <= d_min <= d_max,
                              d_max - d_min < 64 [1, 20]                    */
  double dt_ms;            /* step [0.1]                                    */
  int32_t weight_dtype;    /* DPSNN_W_*                                     */
  int32_t acc_bits;        /* 32 or 64: fixed-point input slot width        */
  int32_t q_frac_bits;     /* fractional bits Q of the fixed point [16]     */
  double J_mean[2], J_sd[2];           /* recurrent efficacy [0.5, -2.0] /
                                          [0.1, 0.4]                        */
  double nu_ext_hz[2];                 /* external Poisson rate [1000]      */
  double Jext_mean[2], Jext_sd[2];     /* external efficacy                 */
  double tau_m[2], E[2], V_th[2], V_r[2], tau_arp[2]; /* Eq. 2, Table S1    */
  double alpha_c[2], tau_c[2];         /* adaptation increment and decay    */
  double gc[2];                        /* g_c / C_m in 1/ms [0.02, 0]       */
  double I_const[2];                   /* constant drive, mV/ms [0]         */
  int32_t rate_bin_steps;              /* steps per rate bin [50 = 5 ms]    */
  int64_t spike_log_cap;               /* device spike-log entries; 0 = off */
  int64_t rate_bins_cap;               /* device rate bins kept [>= 1]      */
  int32_t queue_cap;                   /* entries of each per-(tile, slot)
                                          input queue; each tile's inbox per
                                          step holds twice as many.  0 =
                                          default (4096, less if the queues
                                          would pass 16 GiB), -1 = no queues
                                          (every event is an atomic add into
                                          its slot), else 1 .. 2^20.  Results
                                          do not depend on it.              */
  /* Population model of Sec. 2.2 and Table S1 (n_pops = 2..4; 0 keeps the
   * two-population model above).  Each module's K neurons are split into
   * consecutive populations of pop_size[] neurons (sum K).  A neuron of
   * population s projects n_syn[t][s] synapses into population t (every
   * population's total must equal K_out): from an excitatory population
   * (pop_exc = 1) to a module drawn with probability proportional to
   * exp(-d / lambda) over all modules including its own (Eq. 1 from d = 0),
   * from an inhibitory one to its own module; efficacy
   * N(J_mean_ts[t][s], J_sd_ts[t][s]).  open_boundary = 1: the grid has
   * edges, and each source draws among the modules that exist; 0: torus.
   * The p_* arrays replace frac_exc, frac_local, J_*, nu_ext_hz, Jext_*,
   * tau_m, E, V_th, V_r, tau_arp, alpha_c, tau_c, gc and I_const, and the
   * rate bins count per population ([bins][modules][n_pops]). */
  int32_t n_pops;
  int32_t open_boundary;
  int32_t pop_size[4];
  int32_t pop_exc[4];
  int32_t n_syn[4][4];
  double J_mean_ts[4][4], J_sd_ts[4][4];
  double p_nu_ext_hz[4], p_Jext_mean[4], p_Jext_sd[4];
  double p_tau_m[4], p_E[4], p_V_th[4], p_V_r[4], p_tau_arp[4];
  double p_alpha_c[4], p_tau_c[4], p_gc[4], p_I_const[4];
  /* Spike-timing-dependent plasticity (Sec. 2.1: each synapse notes its
   * previous activation time; every synaptic event and postsynaptic spike
   * contributes to LTP / LTD through a slow first-order low-pass filter
   * whose state lives in the synapse; efficacies change every second).
   * The paper gives no constants (plasticity is off in its experiments); the
   * rule taken: plastic = 1 makes the synapses of excitatory sources
   * plastic (binary32 efficacies only, split schedule only).  A synapse
   * keeps its last activation step t_act and a binary32 signal y.  When its
   * source spikes at step ta (activation), with tp the target's last spike
   * step (-1: none): y decays by Dy(ta - t_act); if tp > t_act (a spike of
   * the target since the previous activation), y += Ep(tp - t_act) *
   * Dy(ta - tp) (LTP); if tp >= 0, y -= Em(ta - tp) (LTD); t_act = ta.
   * After every stdp_update_steps steps (T = steps done): w = clip(w + eta *
   * (y * Dy(T - t_act)), 0, w_max), y = 0.  Ep(k) = A_plus exp(-k dt /
   * tau_plus), Em(k) = A_minus exp(-k dt / tau_minus), Dy(k) =
   * exp(-k dt / tau_y), each rounded to binary32, and 0 for k >=
   * stdp_update_steps.  Adds 8 bytes per synapse (t_act, y). */
  int32_t plastic;
  int32_t stdp_update_steps;
  double stdp_A_plus, stdp_A_minus;      /* mV of signal per spike pair   */
  double stdp_tau_plus, stdp_tau_minus, stdp_tau_y;  /* ms                 */
  double stdp_eta;                       /* efficacy change per unit of y */
  double stdp_w_max;                     /* largest plastic efficacy, mV  */
} dpsnn_params;

typedef struct dpsnn_stats_t {
  int64_t t;              /* steps simulated                               */
  int64_t n_neurons;      /* neurons                                       */
  int64_t n_modules;      /* modules                                       */
  int64_t n_synapses;     /* recurrent synapses = n_neurons * K_out        */
  int64_t n_spikes;       /* spikes emitted so far                         */
  int64_t n_events;       /* recurrent synaptic events = n_spikes * K_out  */
  double build_ms;        /* wall time of dpsnn_build                      */
  int64_t bytes_rows;     /* device bytes of the synapse rows              */
  int64_t bytes_state;    /* device bytes of neuron state and input slots  */
  int64_t bytes_total;    /* all device bytes owned by the handle          */
  int32_t lds_bytes;      /* LDS per workgroup of the step kernels         */
  int32_t schedule;       /* current DPSNN_SCHED_*                         */
  int64_t n_index;        /* entries of the inspection arrays: the global
                             index space of all networks (see below)      */
  int32_t n_nets;         /* networks in the handle                        */
  int32_t queue_cap;      /* entries per input queue in use (0 = none)   */
  int32_t deliver_blocks; /* grid of the split schedule's delivery kernel  */
  int32_t route_blocks;   /* inbox-routing blocks beside it               */
  int32_t n_pops;         /* populations per module (rate-bin stride)     */
  int32_t queue_entry_bytes; /* bytes per per-slot queue entry: 4 (binary16
                             or int8 efficacy codes; binary32 efficacies
                             that all fit 21 bits in fixed point), else 8;
                             0 = no queues                                */
  int32_t spike_lists;    /* spike lists of the split schedule (see
                             dpsnn_set_delivery)                          */
} dpsnn_stats_t;

typedef struct dpsnn_net dpsnn_net; /* opaque handle */

/* Device memory hook: the allocator used by later dpsnn_build calls in
 * this process (NULL restores hipMalloc/hipFree).  alloc returns device
 * memory of at least `bytes` bytes aligned to 256 B, or NULL. */
typedef void* (*dpsnn_alloc_fn)(size_t bytes, void* ctx);
typedef void (*dpsnn_free_fn)(void* ptr, void* ctx);
int dpsnn_set_allocator(dpsnn_alloc_fn alloc, dpsnn_free_fn release, void* ctx);

/*
 * Build a network on the current HIP device: validates p, computes the host
 * tables in binary64 (propagators of Eq. 2, Poisson count thresholds,
 * Eq. 1 offset thresholds, efficacy quantile tables), allocates device
 * memory, generates every synapse row on the device from the counter-based
 * generator keyed by `seed`, and sets the initial state.  Blocks until
 * done.  Errors: INVAL (bad p or out == NULL), NOMEM, DEVICE, RANGE.
 */
int dpsnn_build(const dpsnn_params* p, uint64_t seed, dpsnn_net** out);

/*
 * Build several independent networks in one handle (batched sweep): they
 * advance together, one set of launches per step for all of them, and each
 * reproduces its own dpsnn_build run bit for bit.  p[k] and seeds[k]
 * describe network k; K_out, d_min, d_max, dt_ms, weight_dtype, acc_bits,
 * q_frac_bits and rate_bin_steps must agree, and the buffer capacities
 * (spike_log_cap, rate_bins_cap) of p[0] apply to the handle.  Networks
 * are laid end to end in one global index space, each padded to a multiple
 * of 1024 neurons (dpsnn_net_info); spike ids, rows, state and slots use
 * global indices, rate bins use global module indices.
 */
int dpsnn_build_batch(const dpsnn_params* p, const uint64_t* seeds, int32_t n_nets,
                      dpsnn_net** out);

/* Where network k of a handle lives in the global index spaces. */
int dpsnn_net_info(dpsnn_net* net, int32_t k, int64_t* base, int64_t* n_neurons,
                   int64_t* module_base, int64_t* n_modules);

/* Stream on which later work of this handle is enqueued (a hipStream_t;
 * NULL = the default stream). */
int dpsnn_set_stream(dpsnn_net* net, void* hip_stream);

/*
 * Enqueue n_steps steps of dt (Eq. 2 update of every neuron with its
 * input slot and external drive, spike collection, delivery of the spikes
 * along their rows into the input slots, 5 ms population counts, spike
 * log).  Asynchronous: returns once enqueued.  Errors: INVAL (n_steps < 0),
 * RATES_FULL (the steps would overwrite rate bins not yet read; nothing is
 * enqueued), DEVICE.
 */
int dpsnn_step(dpsnn_net* net, int64_t n_steps);

/* Choose the step schedule (DPSNN_SCHED_*).  INVAL: an unknown schedule,
 * or FUSED or PERSIST for a plastic network. */
int dpsnn_set_schedule(dpsnn_net* net, int32_t sched);

/* The split schedule's delivery: grid of the delivery kernel (blocks > 0;
 * 0 keeps the current one) and the spike lists it reads (0: one list per
 * tile of 1024 neurons, whose counts every delivery block scans, for at most
 * 14000 tiles; 1: lists appended by the tiles through 64 counters; 2: the
 * appended lists, with the four wavefronts of a delivery block taking the
 * same chunk of four consecutive spikes and reserving inbox room once per
 * target tile for all four instead of once per run (acts as 1 without
 * input queues); -1 keeps the current kind).  Results do not depend on
 * either.  The default: one block per tile, between 256 and 1024 blocks,
 * and kind 2 (kind 1 for a handle without queues).  INVAL otherwise. */
int dpsnn_set_delivery(dpsnn_net* net, int32_t deliver_blocks, int32_t spike_lists);

/* Grid of the inbox-routing blocks of the split schedule's delivery kernel
 * (each block moves the inboxes of every route_blocks-th tile into their
 * per-slot queues): 1 .. number of 1024-neuron tiles, or 0 for the default
 * (one block per tile, at most 4096).  Results do not depend on it.  INVAL
 * otherwise; STATE for a handle without input queues. */
int dpsnn_set_routing(dpsnn_net* net, int32_t route_blocks);

/* Steps captured per HIP graph replay (0 disables graphs; graphs are only
 * used on a non-default stream).  Default 128. */
int dpsnn_set_graph_steps(dpsnn_net* net, int64_t steps);

/*
 * Time real steps with each available schedule, and for the split schedule
 * with several grid sizes of the delivery kernel and both spike-list kinds
 * (they advance the simulation; results do not depend on any of them), and
 * keep the fastest.  Steps run in runs of K (the graph length when graphs
 * are in use, else min(probe_steps, 128)): one untimed run per candidate,
 * then max(1, probe_steps / K) rounds of one timed run per candidate, so
 * that every candidate sees the same mix of activity.  *chosen (may be
 * NULL) receives the schedule.  Synchronises.
 */
int dpsnn_autotune(dpsnn_net* net, int64_t probe_steps, int32_t* chosen);

/*
 * Run n_steps real steps with HIP events around each kernel and return the
 * summed kernel times in host_ms[0] (neuron update; the whole step for the
 * fused schedule) and host_ms[1] (delivery).  The per-block timing of the
 * execution flow the paper uses to guide optimisation (Sec. 2.1.1, Fig. 1
 * caption).  No graphs; synchronises.
 */
int dpsnn_profile_steps(dpsnn_net* net, int64_t n_steps, double* host_ms);

/* Wait for the handle's stream.  Returns SPIKELOG_FULL if the spike log
 * overflowed since it was last drained. */
int dpsnn_sync(dpsnn_net* net);

/*
 * Spikes as (time, neuron id) messages, the unit the paper's engine
 * exchanges and delivers (Sec. 2.1.1, steps 1-2; Sec. 2.1.2).  Drain the
 * spikes logged since the last read into host_step[] / host_id[] (each of
 * capacity `cap`), sorted by (step, neuron id); ids are global indices of
 * the handle.  *n_out = number of spikes available.  With cap < *n_out
 * nothing is copied or drained (query with cap = 0).  The device log holds
 * spike_log_cap entries between reads.  Synchronises.  Errors: INVAL,
 * SPIKELOG_FULL (the device log overflowed: what was kept is still returned
 * and drained), DEVICE.
 */
int dpsnn_read_spikes(dpsnn_net* net, int32_t* host_step, int32_t* host_id,
                      int64_t cap, int64_t* n_out);

/* The same for network k of a batch handle only, with network-local neuron
 * ids (0 .. its neuron count - 1); the spikes of the other networks stay
 * available to later reads. */
int dpsnn_read_spikes_net(dpsnn_net* net, int32_t k, int32_t* host_step,
                          int32_t* host_id, int64_t cap, int64_t* n_out);

/*
 * Drain the completed population-count bins (Sec. 2.3: firing rates per
 * sub-population in bins of rate_bin_steps): host_counts is
 * [bins][modules][n_pops] uint32 (n_pops = 2 for the two-population model)
 * with capacity cap_bins bins; *n_bins = bins available.  With cap_bins < *n_bins nothing is copied or drained.
 * Synchronises.
 */
int dpsnn_read_rates(dpsnn_net* net, uint32_t* host_counts, int64_t cap_bins,
                     int64_t* n_bins);

/* The same for network k of a batch handle only: host_counts is
 * [bins][modules of network k][n_pops], from the first bin that network
 * k has not drained.  dpsnn_read_rates returns every bin some network has
 * not drained; counts a network has already drained read 0 there. */
int dpsnn_read_rates_net(dpsnn_net* net, int32_t k, uint32_t* host_counts,
                         int64_t cap_bins, int64_t* n_bins);

/* Counters and sizes (synchronises): spikes and recurrent synaptic events
 * (the event count of Sec. 2.4), build time, device bytes.  dpsnn_stats_get
 * is the same call under its earlier name. */
int dpsnn_stats(dpsnn_net* net, dpsnn_stats_t* out);
int dpsnn_stats_get(dpsnn_net* net, dpsnn_stats_t* out);

void dpsnn_free(dpsnn_net* net);
const char* dpsnn_strerror(int code);

/* ---- inspection entry points (tests and tools; synchronise) ---------- */

/* Neuron state: V and c as binary32, ref (remaining refractory steps) as
 * uint8; each host array holds stats.n_index entries (= n_neurons for a
 * single network; any pointer may be NULL). */
int dpsnn_read_state(dpsnn_net* net, float* host_V, float* host_c,
                     uint8_t* host_ref);
int dpsnn_write_state(dpsnn_net* net, const float* host_V,
                      const float* host_c, const uint8_t* host_ref);

/* Input slots: D = d_max + 1 slots of stats.n_index fixed-point values,
 * slot-major, as int64 whatever the device width.  Pending local-queue
 * entries are folded into the slots first (the sums are unchanged). */
int dpsnn_read_slots(dpsnn_net* net, int64_t* host_slots);

/* The device spike log as it stands (not drained, not sorted): the entries
 * logged since the last dpsnn_read_spikes in the order the device wrote
 * them.  Each tile lists its spikes in neuron order (a wavefront ballot and
 * prefix sum); with per-tile spike lists (dpsnn_set_delivery) the split
 * schedule logs every step in (step, id) order, with appended lists the
 * tiles' runs follow the order in which the tiles appended them.  With
 * cap < *n_out nothing is copied. */
int dpsnn_read_log(dpsnn_net* net, int32_t* host_step, int32_t* host_id, int64_t cap,
                   int64_t* n_out);

/* Synapse rows first..first+count-1 (Eq. 1 targets, stored efficacies,
 * delays), each sorted by (target, delay, draw index j): host_tgt int32
 * [count][K_out]; host_w [count][K_out] of the stored format (float /
 * binary16 bits / int8 code); host_dk uint8 [count][K_out] = delay - d_min.
 * Any pointer may be NULL. */
int dpsnn_read_rows(dpsnn_net* net, int64_t first, int64_t count,
                    int32_t* host_tgt, void* host_w, uint8_t* host_dk);

/* ---- Slow-wave analysis (Sec. 2.3 and Eq. 4) ----
 *
 * The multi-unit activity of a module is its spike count per rate bin (all
 * populations); the analysed signal is log(MUA / MUA_down) plus zero-mean
 * white noise, a threshold gives the Down-to-Up transition time T(x, y) of
 * every module, and Eq. 4 the wavefront speed 1 / |grad T| averaged over
 * the modules of a wave.  The paper leaves the Down-state level, the
 * threshold and the grouping into waves open; the library takes: Down bins
 * = bins at or below the lower median count of the window, MUA_down and
 * MUA_up = rounded mean counts of the Down and Up bins, one spike added to
 * every count, threshold halfway between the two levels in log units, a
 * transition needs min_down bins at or below and min_up bins above the
 * threshold, its time interpolates the signal linearly between bin centres;
 * transitions of all modules in the order (bin, interpolation fraction in
 * 2^-32 units, module) are grouped greedily (a module entering the current
 * wave again starts the next one); grad T by central differences over the
 * wave's modules, one-sided at its edge, no wrap-around.  The noise of
 * module m in absolute bin b is sqrt(noise_var) * Phi^-1((i + 1/2) / 65536),
 * i = top 16 bits of word 0 of Philox4x32-10((m, b, b >> 32, 5), seed).
 * Limits: at most 4096 bins and 8192 modules.  Speeds are in inter-module
 * distances per second, times in ms. */
typedef struct dpsnn_wave_params {
  uint32_t abi_version;  /* must be DPSNN_ABI_VERSION                        */
  int32_t net;           /* network of a batch handle (dpsnn_waves)          */
  int64_t n_bins;        /* analyse the last n_bins bins not yet drained by
                            dpsnn_read_rates; 0 = all of them (dpsnn_waves)  */
  double noise_var;      /* variance of the added noise (the paper: 0.5)    */
  uint64_t seed;         /* key of the noise draws                           */
  int32_t min_down;      /* >= 1 */
  int32_t min_up;        /* >= 1 */
  int32_t min_modules;   /* smallest wave whose speed is measured            */
  int32_t reserved;
} dpsnn_wave_params;

typedef struct dpsnn_wave_result {
  int64_t bin0;          /* absolute index of the first analysed bin         */
  int64_t n_bins;
  int64_t n_transitions;
  int64_t n_waves;
  double mean_speed;     /* mean of the measured wave speeds; NaN if none    */
  double reserved[3];
} dpsnn_wave_result;

/* Analyse the rate bins a handle holds (not drained; they stay).  Host
 * outputs (each may be NULL; up to its capacity): transitions in order
 * with module (network-local), time and wave; per wave its speed (NaN where
 * not measured: fewer than min_modules modules, or no module with both
 * gradients defined), first transition time and number of modules.
 * Synchronises; allocates its scratch with the handle's allocator and
 * frees it before returning. */
int dpsnn_waves(dpsnn_net* net, const dpsnn_wave_params* wp, dpsnn_wave_result* out,
                int32_t* host_tr_module, double* host_tr_T, int32_t* host_tr_wave,
                int64_t cap_tr, double* host_wave_speed, double* host_wave_t0,
                int32_t* host_wave_n, int64_t cap_waves);

/* The same analysis of counts held in device memory: dev_counts is
 * [n_bins][grid_w * grid_h][n_pops] uint32 (module m at x = m % grid_w,
 * y = m / grid_w), bin b of it is absolute bin bin0 + b of width bin_steps
 * steps of dt_ms.  stream: a hipStream_t, or NULL for the default stream;
 * wp->net and wp->n_bins are ignored.  Scratch from hipMalloc, freed before
 * returning. */
int dpsnn_waves_counts(const uint32_t* dev_counts, int64_t n_bins, int32_t grid_w,
                       int32_t grid_h, int32_t n_pops, int32_t bin_steps, double dt_ms,
                       int64_t bin0, const dpsnn_wave_params* wp, void* stream,
                       dpsnn_wave_result* out, int32_t* host_tr_module, double* host_tr_T,
                       int32_t* host_tr_wave, int64_t cap_tr, double* host_wave_speed,
                       double* host_wave_t0, int32_t* host_wave_n, int64_t cap_waves);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the analysis
 * of dpsnn_waves_counts, same arguments and results, with its scratch in a
 * fixed device buffer of 64 MiB that the library holds on every GPU it runs
 * on until the process ends, instead of memory allocated per call.  It
 * calls no hipMalloc / hipFree and no allocator.  Limits: the buffers of
 * the request must fit 64 MiB (about 72 bytes per possible transition,
 * grid_w * grid_h * (n_bins / (min_down + min_up) + 1) of them, plus
 * 2 KiB per module and 1 MiB of tables), and no module may count more than
 * 65535 spikes in a bin; DPSNN_E_SCRATCH otherwise, before any device work
 * for the size limit.  Every call on one GPU shares that GPU's buffer:
 * calls that overlap on one GPU (from several host threads or streams) race
 * and must not be made.  Results are identical to dpsnn_waves_counts. */
int dpsnn_waves_counts_static(const uint32_t* dev_counts, int64_t n_bins, int32_t grid_w,
                              int32_t grid_h, int32_t n_pops, int32_t bin_steps,
                              double dt_ms, int64_t bin0, const dpsnn_wave_params* wp,
                              void* stream, dpsnn_wave_result* out, int32_t* host_tr_module,
                              double* host_tr_T, int32_t* host_tr_wave, int64_t cap_tr,
                              double* host_wave_speed, double* host_wave_t0,
                              int32_t* host_wave_n, int64_t cap_waves);

/* Plasticity state of rows first..first+count-1, in the order of
 * dpsnn_read_rows: host_t_act int32 [count][K_out] (last activation step,
 * -1: never), host_y float [count][K_out]; efficacies via dpsnn_read_rows.
 * DPSNN_E_STATE without plasticity.  Either pointer may be NULL. */
int dpsnn_read_plasticity(dpsnn_net* net, int64_t first, int64_t count,
                          int32_t* host_t_act, float* host_y);

/* Host table computed from p without any device (named arrays, see the
 * library source); returns the size in bytes, or a negative code. */
int64_t dpsnn_host_table(const dpsnn_params* p, const char* name, void* out,
                         int64_t cap);

#ifdef __cplusplus
}
#endif
#endif /* DPSNN_H */
