// Internal declarations of libdpsnn: host tables, the handle, kernel
// arguments and launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "dpsnn.h"

namespace dpsnn {

constexpr int kQuantN = 65536;  // entries of each efficacy quantile table
constexpr int kMaxPois = 16;    // Poisson count thresholds per population
constexpr int kMaxDelays = 64;  // distinct delays handled by one wavefront
constexpr int kMaxKout = 4096;
constexpr int kDelayShift = 26;  // target word = target | delay index << 26
constexpr int32_t kTargetMask = (1 << kDelayShift) - 1;
constexpr int kSpkLists = 64;          // appended spike lists per step
constexpr int kSpkListShift = 4;       // runs of 16 consecutive tiles share a list
constexpr int kMaxScanTiles = 14000;   // per-tile lists: LDS prefix of the tile counts
                                       // (with the entry staging and the static LDS,
                                       // within 64 KiB per block)
constexpr int kSpkStride = 16;         // their counters 64 bytes apart
constexpr int kQueueMaxSlots = 128;   // input queues need D <= 128 slots
constexpr int kQueueDefaultCap = 4096; // entries per (tile, slot) queue
constexpr int kInboxStride = 16;       // inbox counters 64 bytes apart
constexpr int kStage = 2048;           // LDS staging of a tile's routed events

// Queue entry, 8 bytes: x = in-tile index | delay index << 10 (17 bits at
// most) and the fixed-point efficacy w.  int32 inputs: two words; int64
// inputs: one word w << 17 | x (efficacies below 2^46 in fixed point; the
// build checks, and uses no queues otherwise).
template <typename Acc>
struct QEntry;
template <>
struct __attribute__((aligned(8))) QEntry<int32_t> {
  uint32_t xv;
  int32_t wv;
  __host__ __device__ uint32_t x() const { return xv; }
  __host__ __device__ int32_t w() const { return wv; }
  __host__ __device__ static QEntry make(uint32_t x, int32_t w) {
    QEntry q;
    q.xv = x;
    q.wv = w;
    return q;
  }
};
template <>
struct __attribute__((aligned(8))) QEntry<int64_t> {
  uint64_t v;
  __host__ __device__ uint32_t x() const { return (uint32_t)(v & 0x1FFFFu); }
  __host__ __device__ int64_t w() const { return (int64_t)v >> 17; }
  __host__ __device__ static QEntry make(uint32_t x, int64_t w) {
    QEntry q;
    q.v = ((uint64_t)w << 17) | x;
    return q;
  }
};
constexpr int64_t kQEntry64Max = (int64_t)1 << 46;  // |w| bound of the int64 entry

// Code entry, 4 bytes, for binary16 and int8 efficacies: the stored
// efficacy code << 16 | delay index << 10 | in-tile index, the code being
// the binary16 bits, or the int8 code | source population << 8.  The
// consumer converts the code to fixed point exactly as delivery does (the
// int8 scale of a source population is the same in every module of a
// network), so the sums do not change.
constexpr int kCodeShift = 16;
constexpr int kCodeF16 = 1;     // StepArgs::q_code
constexpr int kCodeI8 = 2;
__host__ __device__ inline uint32_t code_entry(uint32_t code, uint32_t x) {
  return (code << kCodeShift) | x;
}

constexpr int kMaxPops = 4;     // populations per module
constexpr int kMaxAttempts = 64; // draws of a module inside open boundaries
// how a block of a source's synapses picks the target module
constexpr int kRuleOwn = 0;      // the source's module
constexpr int kRuleOthers = 1;   // another module by Eq. 1
constexpr int kRuleAll = 2;      // any module by Eq. 1 from d = 0

// Everything dpsnn_build derives from the parameters on the host, in
// binary64 first and rounded once to the width the device uses.  The
// two-population parameters are expressed in the same terms as the
// population model: populations with module-local index ranges, and per
// source population an ordered list of synapse blocks.
struct HostTables {
  int64_t N = 0;          // neurons
  int64_t N_pad = 0;      // neurons rounded up to the step kernel's tile
  int32_t M = 0;          // modules
  int32_t P = 2;          // populations per module
  int32_t pop_lo[kMaxPops] = {0, 0, 0, 0}, pop_hi[kMaxPops] = {0, 0, 0, 0};
  int32_t D = 0;          // input slots = d_max + 1
  int32_t n_del = 0;      // distinct delays
  int32_t row_stride = 0; // K_out rounded up to a multiple of 4
  int32_t n_arp[kMaxPops] = {0, 0, 0, 0};

  double prop64[kMaxPops][4];    // Pm, Pc, PVc, Iterm
  float prop32[kMaxPops][4];
  double E[kMaxPops], Vth[kMaxPops], Vr[kMaxPops], alpha[kMaxPops];

  int32_t n_pois[kMaxPops] = {0, 0, 0, 0};
  uint32_t pois[kMaxPops][kMaxPois];

  int32_t n_blk[kMaxPops] = {0, 0, 0, 0};
  int32_t blk_n[kMaxPops][kMaxPops], blk_lo[kMaxPops][kMaxPops];
  int32_t blk_hi[kMaxPops][kMaxPops], blk_rule[kMaxPops][kMaxPops];
  double blk_J[kMaxPops][kMaxPops], blk_sd[kMaxPops][kMaxPops];

  int32_t open = 0;               // open boundaries (draws outside repeated)
  std::vector<uint32_t> off_thr;  // cumulative thresholds of the offsets
  std::vector<int32_t> off_xy;    // (ox, oy) per offset

  // efficacy tables by (source pop, block); a pop with no block has one
  std::vector<double> wt64[kMaxPops][kMaxPops];
  std::vector<float> wt32[kMaxPops][kMaxPops];
  std::vector<uint16_t> wt16[kMaxPops][kMaxPops];
  std::vector<int8_t> wq8[kMaxPops][kMaxPops];
  float s8[kMaxPops] = {1.f, 1.f, 1.f, 1.f};
  int64_t s8fix[kMaxPops] = {0, 0, 0, 0};
  std::vector<double> jx64[kMaxPops];    // external efficacy by target pop
  std::vector<float> jx32[kMaxPops];
  std::vector<int64_t> jxfix[kMaxPops];
  int64_t ext_bound = 0;          // largest |external sum| of one step

  int tables(int q) const { return n_blk[q] > 0 ? n_blk[q] : 1; }
};

int validate(const dpsnn_params& p);
int compute_tables(const dpsnn_params& p, HostTables& T);
int64_t host_table(const HostTables& T, const char* name, void* out, int64_t cap);

// Per-network constants, one entry per network of a handle (a batch of one
// for dpsnn_build).  Networks are laid end to end in one global index space,
// each padded to whole 1024-neuron tiles, so every tile belongs to exactly
// one network and the step kernels read these fields with uniform loads.
struct NetDev {
  int64_t base;             // global index of the network's neuron 0
  int64_t N;                // neurons of the network
  int32_t mbase;            // global index of the network's module 0
  int32_t K, P;             // neurons and populations per module
  int32_t pop_hi[kMaxPops]; // module-local end of each population (K past P)
  uint32_t key0, key1;      // Philox key (the network's seed)
  float Pm[kMaxPops], Pc[kMaxPops], PVc[kMaxPops], Iterm[kMaxPops];
  float E[kMaxPops], Vth[kMaxPops], Vr[kMaxPops], alpha[kMaxPops];
  int32_t n_arp[kMaxPops];
  int32_t n_pois[kMaxPops];
  uint32_t pois[kMaxPops][kMaxPois];
  int32_t exc[kMaxPops];    // 1: excitatory population (its synapses are plastic)
  // module of a network-local index x < 2^31: x / K = umulhi(x, kmag) >> kshift
  // (kshift = floor(log2 K), kmag = ceil(2^(32 + kshift) / K); kmag = 0 when K
  // is a power of two: x >> kshift)
  uint32_t kmag;
  int32_t kshift;
  // Populations whose Eq. 2 constants are equal bit for bit form classes;
  // when the populations [0, cls_rep) share one set and [cls_rep, P) another
  // (F and B against I in the three-population model), class 1 starts at
  // module-local index cls_hi and takes the constants of population cls_rep
  // (one class: cls_hi = K, cls_rep = 0).
  int32_t cls_hi, cls_rep;
};

// Module and module-local index of network-local neuron x (x < 2^31): the
// multiply-high is exact there because x * (kmag - 2^(32+s)/K) / 2^(32+s)
// stays below 1/K.
__host__ __device__ inline uint32_t module_of(const NetDev& nd, uint32_t x) {
  const uint32_t hi = (uint32_t)(((uint64_t)x * nd.kmag) >> 32);
  return (nd.kmag ? hi : x) >> nd.kshift;
}

// Step index and the values the kernels derive from it.  The device keeps
// them for the step counter t (StepArgs::t_base: t, t mod D, t mod
// rate_bin_steps, (t / rate_bin_steps) mod rate_bins_cap, written by
// k_tick); a launch for step t + t_off carries t_off and its own residues
// (StepOff, computed on the host), so that no kernel divides by D or by the
// rate-bin sizes.
struct StepOff {
  uint32_t t_off, d_slot, d_phase, d_bin;
};
struct StepTime {
  uint32_t t;     // step index
  uint32_t slot;  // input slot of the step: t mod D
  uint32_t bin;   // rate bin of the step in the ring
};

// Arguments of the step kernels (passed by value).
struct StepArgs {
  int64_t N_pad;           // size of the global index space
  int32_t K_out, row_stride, D, n_del, d_min, M;  // M: modules of all networks
  int32_t P;               // populations per module (rate-bin and scale stride)
  int32_t two_cls;         // P > 2 and every network's Eq. 2 constants fall
                           // into two contiguous classes (NetDev::cls_hi)
  int32_t n_tiles;         // neuron tiles of 1024 = N_pad / 1024
  int32_t deliver_blocks;  // delivery blocks of the delivery kernel
  int32_t route_blocks;    // inbox-routing blocks that follow them
  int32_t rate_bin_steps, rate_bins_cap;
  float inv2q, two_q;
  int64_t spike_log_cap;
  const NetDev* nets;
  const int32_t* tile_net;  // [n_tiles] network of each tile
  const void* jx;          // [networks][kMaxPops][65536] external fixed-point
                           // efficacies of the slot width
  float* V;
  float* c;
  uint8_t* ref;
  void* slots;
  const int32_t* tgt;      // global target | delay index << 26
  const void* w;
  const int64_t* sfix;     // [M][P] int8 scale in fixed point (int8 format)
  // Spikes of the step (split schedule).  Per-tile lists (spk_lists = 0):
  // tile b writes its spike ids to spk[b * 1024 ...] and their count to
  // blk_cnt[b]; each delivery block scans the counts.  Appended lists
  // (spk_lists = 1, the default; 2: the same lists, delivered with
  // reservations merged over each block's four chunks): tile b appends its
  // ids to list g = (b >> kSpkListShift) mod kSpkLists, spk[g * spk_cap ...],
  // counted in spk_n[((t & 1) * kSpkLists + g) * kSpkStride]; the delivery
  // of step t zeroes the counters of step t + 1, and so does the
  // step-counter kernel.
  int32_t spk_lists;
  int32_t* spk;            // [kSpkLists][spk_cap] (>= n_tiles * 1024)
  int64_t spk_cap;         // room for every neuron of the tiles of one list
  int32_t* blk_cnt;        // [n_tiles]
  uint32_t* spk_n;         // [2][kSpkLists][kSpkStride]
  int2* log;
  unsigned long long* log_base;  // [2]: log entries before step t at [t & 1]
  unsigned int* rates;
  unsigned long long* n_spikes;
  uint32_t* t_base;        // device step counter and its residues [4] (StepOff)
  // Event queues (q_cap = 0: none; every event is then an atomic add into
  // its slot).  Delivery appends each event to the inbox of its target tile
  // for the step (parity t & 1); in the next step the tile moves its inbox
  // into its own per-slot queues and sums the queue of the current slot.
  // An entry (QEntry) holds in-tile index | delay index << 10 and the
  // fixed-point efficacy.  Events that find a queue full are added into the
  // slot, and the slot is marked in s_dirty: the update reads and clears
  // the slots marked only (with queues every other slot holds zeros).
  int32_t q_cap, in_cap;
  int32_t q_packed;        // queue entries packed in 4 bytes (int32 inputs
                           // whose efficacies all fit 21 bits: w << 10 | idx)
  int32_t q_code;          // 0, or kCodeF16 / kCodeI8: inbox and queue entries
                           // are code entries (takes precedence over q_packed)
  uint32_t* in_cnt;        // [2][n_tiles * kInboxStride] (may exceed in_cap)
  void* in_q;              // [2][n_tiles][in_cap] entries
  uint32_t* q_cnt;         // [n_tiles][D], written by the owning tile only
  void* q_q;               // [n_tiles][D][q_cap] entries
  uint32_t* s_dirty;       // [n_tiles][D]: slot holds added input
  // Plasticity (plastic networks; the rule is documented with dpsnn_params).
  int32_t plastic, stdp_L;   // stdp_L = update period = table length
  float stdp_eta, stdp_wmax;
  int32_t* syn_t;          // [N_pad][row_stride] last activation step, -1 never
  float* syn_y;            // [N_pad][row_stride] plasticity signal
  int32_t* t_post;         // [N_pad] last spike step, -1 none
  const float* stdp_tab;   // [3][stdp_L]: Ep, Em, Dy
};

struct GenArgs {
  int64_t N;
  int64_t tgt_base;        // global index of the network's neuron 0
  int32_t K, K_out, row_stride, n_del, d_min;
  int32_t W, H, n_off, open;
  int32_t P, pop_hi[kMaxPops];
  // synapse blocks of each source pop: end (cumulative count), target range,
  // module rule
  int32_t n_blk[kMaxPops];
  int32_t blk_end[kMaxPops][kMaxPops], blk_lo[kMaxPops][kMaxPops];
  int32_t blk_hi[kMaxPops][kMaxPops], blk_rule[kMaxPops][kMaxPops];
  uint32_t key0, key1;
  const uint32_t* off_thr;
  const int32_t* off_xy;
  const void* wtab[kMaxPops][kMaxPops];  // stored-format table by (pop, block)
  int32_t* tgt;
  void* w;
  // fixed-point in-weight sums for the int32 range check (may be null)
  unsigned long long* absum;
  const int64_t* wfix_tab[kMaxPops][kMaxPops];
};

struct InitArgs {
  int64_t N, N_pad;
  int32_t K, P, pop_hi[kMaxPops];
  uint32_t key0, key1;
  float E[kMaxPops], Vth[kMaxPops];
  float* V;
  float* c;
  uint8_t* ref;
};

hipError_t launch_gen(const GenArgs& a, int wdt, hipStream_t s);
hipError_t launch_init(const InitArgs& a, hipStream_t s);
hipError_t launch_step(const StepArgs& a, int wdt, int acc_bits, int sched, uint32_t t_off,
                       hipStream_t s);
hipError_t launch_tick(const StepArgs& a, uint32_t n, int sync_logs, hipStream_t s);
// n steps of the persistent schedule in one cooperative launch (no tick).
hipError_t launch_persist(const StepArgs& a, int wdt, int acc_bits, uint32_t t_off, uint32_t n,
                          hipStream_t s);
hipError_t launch_phase(const StepArgs& a, int wdt, int acc_bits, int phase, uint32_t t_off,
                        hipStream_t s);
// Fold every pending queue entry into its slot and empty the queues; t is
// the number of steps taken.
hipError_t launch_drain(const StepArgs& a, int acc_bits, uint32_t t, hipStream_t s);
// LDS per block of the split schedule's delivery kernel (static and dynamic).
size_t deliver_lds_bytes(const StepArgs& a, int acc_bits);
// Periodic efficacy update of the plastic synapses after T steps.
hipError_t launch_stdp_update(const StepArgs& a, int32_t T, hipStream_t s);
hipError_t launch_absum_max(const unsigned long long* absum, int64_t n,
                            unsigned long long* out, hipStream_t s);

// Slow-wave analysis (waves.hip).  Counts of window bin k, module m,
// population q at counts[(((slot0 + k) % ring) * M_stride + mbase + m) * P + q];
// bin0 = absolute index of window bin 0 (noise draws and times).
struct WaveArgs {
  const uint32_t* counts;
  int64_t ring, slot0, M_stride, mbase, bin0;
  int32_t nb, M, W, H, P;
  int32_t min_down, min_up, min_modules, cap_pm;
  double dbin, sd;
  uint32_t key0, key1;
  const double* lnt;        // lnt[i] = log(i)
  const double* z;          // 65536 standard normal quantiles
  // per module: transitions in bin order
  uint32_t* cnt;            // [M]
  uint32_t* tr_k;           // [M][cap_pm] window bin
  uint32_t* tr_q;           // [M][cap_pm] interpolation fraction, 2^-32 units
  double* tr_T;             // [M][cap_pm] time, ms
  // ordering
  uint32_t* hist;           // [nb]
  uint32_t* fill;           // [nb]
  uint32_t* off;            // [nb + 1]
  unsigned long long* keys; // [M * cap_pm] fraction << 32 | module << 12 | index
  uint32_t* pos;            // [M][cap_pm] position of each transition in the order
  uint32_t* nxt;            // [M * cap_pm] next position of the module, then its
                            // suffix minimum (end of the wave starting there)
  // ordered transitions and waves
  int32_t* out_module;
  double* out_T;
  int32_t* out_wave;
  int32_t* wave_first;      // [M * cap_pm + 1]
  int32_t* n_waves;         // [1]
  double* wave_speed;
  double* wave_t0;
  int32_t* wave_n;
  double* grid;             // [batch][M] transition times of a wave batch
};
constexpr int kWaveMaxBins = 4096;
constexpr int kWaveMaxModules = 8192;
constexpr int kWaveBatch = 256;  // waves per launch of the speed kernel
hipError_t launch_wave_max(const WaveArgs& a, uint32_t* out, hipStream_t s);
hipError_t launch_wave_transitions(const WaveArgs& a, hipStream_t s);
hipError_t launch_wave_speed(const WaveArgs& a, int32_t w0, int32_t n, hipStream_t s);
hipError_t launch_wave_mean(const WaveArgs& a, double* out, hipStream_t s);
// The 65536 standard normal quantiles of the efficacy tables.
const std::vector<double>& standard_normal_grid();

}  // namespace dpsnn

// The opaque handle of the C-ABI.
struct dpsnn_net {
  std::vector<dpsnn_params> p;       // one per network; p[0] holds the
                                     // parameters shared by the batch
  std::vector<uint64_t> seed;
  std::vector<dpsnn::HostTables> T;
  std::vector<int64_t> base, mbase;  // global neuron / module offsets
  int64_t N_total = 0, N_index = 0, N_pad = 0;
  int32_t M_total = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  dpsnn_free_fn free_fn = nullptr;
  void* alloc_ctx = nullptr;
  std::vector<void*> blocks;   // every device allocation of this handle
  int64_t bytes_total = 0, bytes_rows = 0, bytes_state = 0;
  double build_ms = 0.0;
  int64_t t = 0;
  std::vector<int64_t> rate_first;  // per network: first rate bin it has not drained
  std::vector<std::vector<int2>> pend;  // per network: drained log entries not yet read
  bool log_overflow = false;   // the device log overflowed since the last read
  dpsnn::StepArgs sa;
  unsigned char* ctl = nullptr;  // log bases, spike total, step counter, spike-list counts
  int sched = DPSNN_SCHED_SPLIT;
  int last_sched = -1;
  // captured steps: graph_K steps of the current schedule on `stream`
  hipGraphExec_t graph = nullptr;
  int graph_K = 0, graph_sched = -1;
  int32_t graph_blocks = 0;     // delivery grid captured in the graph
  int32_t graph_lists = 0;      // spike-list kind captured in the graph
  int32_t graph_routes = 0;     // routing grid captured in the graph
  hipStream_t graph_stream = nullptr;
  int64_t graph_steps = 128;    // steps per captured graph (0 = no graphs)
};
