// HIP kernels of libdpsnn for gfx950 (64-lane wavefronts).
//
//  k_gen      one wavefront per source row: draws the K_out synapses of the
//             source from Philox (blocks of synapses per target population,
//             Eq. 1 targets, uniform delay, quantile-table efficacy), sorts
//             them by (target, delay, draw index) in LDS and writes the row.
//             The delay index rides in the top 6 bits of each target word,
//             so that delivery needs no lookup.
//  k_init     initial membrane potentials, fatigue and refractory counters.
//  k_neuron   one step of dt for a tile of 1024 neurons (4 per thread): the
//             tile's queued inputs summed in LDS, the input slot read and
//             cleared where marked, external Poisson drive, Eq. 2 update,
//             threshold, 5 ms population counts; the tile's spikes are
//             appended to one of the step's spike lists (or kept per tile).
//  k_deliver  delivery blocks: every wavefront takes chunks of 256 synapses
//             of spiking rows (16-byte loads, the next chunk's loads issued
//             before the current one is delivered); the events of a chunk to
//             one tile form a run in the target-sorted row.  With appended
//             spike lists the four wavefronts of a block take the same chunk
//             of four consecutive spikes together, and one returning atomic
//             per target tile reserves the runs of all four in that tile's
//             inbox of the step (an LDS hash merges them); otherwise one
//             atomic per run.  Routing blocks of the same grid move each
//             tile's inbox of the previous step into its per-slot queues.
//             Also appends the spike log.
//  k_step     fused schedule for small networks: update, routing and the
//             delivery of the tile's own spikes in one block per tile.
//  k_drain    folds pending queue entries into the slots (schedule switches
//             and inspection).
//  k_stdp_update  the periodic efficacy update of plastic networks.
//
// Event queues.  Per 1024-neuron tile: an inbox for each step parity and a
// queue per input slot.  Delivery of step t appends each event (in-tile
// index, delay index, efficacy) to its target tile's inbox; at step t + 1
// the update sums the events that arrive at once (delay d_min = 1) and the
// queue of the current slot, and the routing blocks move the other events of
// the inbox into the queues of their arrival slots.  Events that find an
// inbox, the routing stage or a queue full are added into the slot with an
// atomic instead, and the (tile, slot) is marked so that the update reads
// that slot.  Every path sums integers, so the result does not depend on
// the path or the order.
//
// A step reads only slot t mod D and delivery writes only slots t+d_min ..
// t+d_max, so update and delivery of one step need no grid-wide ordering;
// the kernel boundary orders consecutive steps.  The step index is read on
// the device (t = *t_base + t_off) so that launches can be captured in a graph.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "dpsnn_internal.h"
#include "philox.h"

namespace dpsnn {

// ------------------------------------------------------------------------
// LDS written by some lanes of a wavefront and read by others: the hardware
// performs one wavefront's LDS operations in order, so only the compiler
// must not move them across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup barrier that orders LDS only: global loads and stores issued
// before it stay in flight (a full __syncthreads waits for all of them).
// Used where threads share data through LDS alone.
// Clang vector types for the non-temporal loads and stores.
typedef float NtF4 __attribute__((ext_vector_type(4)));
typedef int NtI4 __attribute__((ext_vector_type(4)));
typedef unsigned short NtU16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Step index and residues of the launch for step t_base + o.t_off: one
// 16-byte uniform load, then conditional subtractions (each residue sum is
// below twice its modulus; the bin sum below 2 cap + 1).
__device__ __forceinline__ StepTime step_time(const StepArgs& a, const StepOff& o) {
  const uint4 c = *reinterpret_cast<const uint4*>(a.t_base);
  StepTime T;
  T.t = c.x + o.t_off;
  uint32_t sl = c.y + o.d_slot;
  if (sl >= (uint32_t)a.D) sl -= (uint32_t)a.D;
  T.slot = sl;
  const uint32_t carry = c.z + o.d_phase >= (uint32_t)a.rate_bin_steps ? 1u : 0u;
  uint32_t b = c.w + o.d_bin + carry;
  if (b >= (uint32_t)a.rate_bins_cap) b -= (uint32_t)a.rate_bins_cap;
  if (b >= (uint32_t)a.rate_bins_cap) b -= (uint32_t)a.rate_bins_cap;
  T.bin = b;
  return T;
}

// Module and population of global neuron id.
__device__ __forceinline__ void module_pop(const StepArgs& a, int32_t id, int32_t* mod,
                                           int* pop) {
  const NetDev& nd = a.nets[a.tile_net[id >> 10]];
  const uint32_t local = (uint32_t)(id - (int32_t)nd.base);
  const uint32_t m = module_of(nd, local);
  *mod = nd.mbase + (int32_t)m;
  const int32_t l = (int32_t)(local - m * (uint32_t)nd.K);
  *pop = (l >= nd.pop_hi[0]) + (l >= nd.pop_hi[1]) + (l >= nd.pop_hi[2]);
}

// ------------------------------------------------------------------------
// Connectivity generation
__host__ __device__ inline int gen_pow2(int Ko) {
  int P = 64;
  while (P < Ko) P <<= 1;
  return P;
}
__host__ __device__ inline int gen_stage_bytes(int Ko) {
  // sort keys (8 per slot of the power-of-two sort) + efficacy index (2) +
  // block (1)
  return gen_pow2(Ko) * 8 + ((3 * Ko + 15) / 16) * 16;
}

template <int WDT>
__global__ void __launch_bounds__(256) k_gen(GenArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int64_t s = (int64_t)blockIdx.x * wpb + wave;
  if (s >= a.N) return;  // whole wavefronts only: no block barrier below
  const int Ko = a.K_out;
  const int P = gen_pow2(Ko);

  unsigned char* base = smem + (size_t)wave * gen_stage_bytes(Ko);
  uint64_t* st_key = reinterpret_cast<uint64_t*>(base);
  uint16_t* st_w = reinterpret_cast<uint16_t*>(base + (size_t)P * 8);
  uint8_t* st_b = reinterpret_cast<uint8_t*>(st_w + Ko);

  const int32_t ls = (int32_t)(s % a.K);
  const int32_t ms = (int32_t)(s / a.K);
  const int pop = (ls >= a.pop_hi[0]) + (ls >= a.pop_hi[1]) + (ls >= a.pop_hi[2]);
  const int xs = ms % a.W, ys = ms / a.W;

  // draw synapse j of block b: sort key = target << 18 | delay index << 12 | j
  for (int j = lane; j < P; j += 64) {
    uint64_t key = ~0ull;
    if (j < Ko) {
      int b = 0;
      while (b + 1 < a.n_blk[pop] && j >= a.blk_end[pop][b]) ++b;
      const int lo = a.blk_lo[pop][b], size = a.blk_hi[pop][b] - lo;
      const int rule = a.blk_rule[pop][b];
      uint4 u;
      int32_t mt = ms;
      uint32_t nu;  // the word that picks the neuron
      if (rule == kRuleOwn) {
        u = philox10(make_uint4((uint32_t)s, (uint32_t)j, 0u, kTagSyn), a.key0, a.key1);
        nu = u.x;
      } else {
        // Eq. 1: module offset from word 0; with open edges a draw that
        // leaves the grid is repeated with counter word 2 = attempt
        for (uint32_t att = 0;; ++att) {
          u = philox10(make_uint4((uint32_t)s, (uint32_t)j, att, kTagSyn), a.key0, a.key1);
          int lo2 = 0, hi2 = a.n_off - 1;  // first threshold above u.x
          while (lo2 < hi2) {
            const int mid = (lo2 + hi2) >> 1;
            if (a.off_thr[mid] <= u.x)
              lo2 = mid + 1;
            else
              hi2 = mid;
          }
          int xt = xs + a.off_xy[2 * lo2];
          int yt = ys + a.off_xy[2 * lo2 + 1];
          if (!a.open) {
            if (xt >= a.W) xt -= a.W;
            if (yt >= a.H) yt -= a.H;
          }
          if (xt >= 0 && xt < a.W && yt >= 0 && yt < a.H) {
            mt = yt * a.W + xt;
            break;
          }
          if (att + 1 == (uint32_t)kMaxAttempts) break;  // own module
        }
        nu = u.y;
      }
      uint32_t r;
      if (mt == ms && ls >= lo && ls < lo + size) {  // no autapse
        r = scale32(nu, (uint32_t)(size - 1));
        r += r >= (uint32_t)(ls - lo) ? 1u : 0u;
      } else {
        r = scale32(nu, (uint32_t)size);
      }
      const int32_t tg = mt * a.K + lo + (int32_t)r;
      const uint32_t k = scale32(u.z, (uint32_t)a.n_del);
      st_w[j] = (uint16_t)(u.w >> 16);
      st_b[j] = (uint8_t)b;
      key = ((uint64_t)(uint32_t)tg << 18) | ((uint64_t)k << 12) | (uint64_t)j;
    }
    st_key[j] = key;
  }
  wave_lds_sync();
  // bitonic sort of the P keys, ascending (padding keys sort last); the
  // keys are distinct, so the order is that of (target, delay, j)
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int q = lane; q < P / 2; q += 64) {
        const int lo = 2 * q - (q & (stride - 1));
        const int hi = lo + stride;
        const uint64_t x = st_key[lo], y = st_key[hi];
        if ((x > y) == ((lo & size) == 0)) {
          st_key[lo] = y;
          st_key[hi] = x;
        }
      }
      wave_lds_sync();
    }
  }
  const int64_t rb = s * a.row_stride;
  for (int pos = lane; pos < Ko; pos += 64) {
    const uint64_t key = st_key[pos];
    const int32_t tg = (int32_t)(key >> 18);
    const int k = (int)((key >> 12) & 63u);
    const uint16_t wi = st_w[key & 4095u];
    const int b = st_b[key & 4095u];
    const int64_t o = rb + pos;
    const int32_t gt = tg + (int32_t)a.tgt_base;  // global target index
    a.tgt[o] = gt | (k << kDelayShift);
    if (WDT == DPSNN_W_F32)
      static_cast<float*>(a.w)[o] = static_cast<const float*>(a.wtab[pop][b])[wi];
    else if (WDT == DPSNN_W_F16)
      static_cast<uint16_t*>(a.w)[o] = static_cast<const uint16_t*>(a.wtab[pop][b])[wi];
    else
      static_cast<int8_t*>(a.w)[o] = static_cast<const int8_t*>(a.wtab[pop][b])[wi];
    if (a.absum) {
      const int64_t f = a.wfix_tab[pop][b][wi];
      atomicAdd(&a.absum[gt], (unsigned long long)(f < 0 ? -f : f));
    }
  }
  for (int j = Ko + lane; j < a.row_stride; j += 64) {
    a.tgt[rb + j] = 0;
    if (WDT == DPSNN_W_F32)
      static_cast<float*>(a.w)[rb + j] = 0.f;
    else if (WDT == DPSNN_W_F16)
      static_cast<uint16_t*>(a.w)[rb + j] = 0;
    else
      static_cast<int8_t*>(a.w)[rb + j] = 0;
  }
}

__global__ void k_absum_max(const unsigned long long* v, int64_t n,
                            unsigned long long* out) {
  unsigned long long m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = v[i] > m ? v[i] : m;
  atomicMax(out, m);
}

// ------------------------------------------------------------------------
// Initial state: V uniform on [E, V_th) from (i, 0, 0, INIT), c = 0, ref = 0.
__global__ void k_init(InitArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N_pad) return;
  float V = 0.f;
  if (i < a.N) {
    const int l = (int)(i % a.K);
    const int q = (l >= a.pop_hi[0]) + (l >= a.pop_hi[1]) + (l >= a.pop_hi[2]);
    const uint4 u = philox10(make_uint4((uint32_t)i, 0u, 0u, kTagInit), a.key0, a.key1);
    const float f = (float)(u.x >> 8) * 0x1p-24f;
    V = a.E[q] + (a.Vth[q] - a.E[q]) * f;
  }
  a.V[i] = V;
  a.c[i] = 0.f;
  a.ref[i] = 0;
}

// ------------------------------------------------------------------------
// Fixed-point helpers

// Input sum in mV: one rounding of I * 2^-Q to binary32 (an int64 sum below
// 2^53 converts to binary64 exactly first).
__device__ __forceinline__ float fix_to_f32(int32_t v) { return (float)v; }
__device__ __forceinline__ float fix_to_f32(int64_t v) { return (float)(double)v; }

template <typename Acc>
__device__ __forceinline__ void atomic_add_fix(Acc* p, Acc v);
template <>
__device__ __forceinline__ void atomic_add_fix<int32_t>(int32_t* p, int32_t v) {
  atomicAdd(p, v);
}
template <>
__device__ __forceinline__ void atomic_add_fix<int64_t>(int64_t* p, int64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}

template <typename Acc>
__device__ __forceinline__ void lds_add(Acc* p, Acc v);
template <>
__device__ __forceinline__ void lds_add<int32_t>(int32_t* p, int32_t v) {
  atomicAdd(p, v);
}
template <>
__device__ __forceinline__ void lds_add<int64_t>(int64_t* p, int64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}

// Fixed-point efficacy of a code entry, computed as delivery computes it
// from the stored code (same conversions, same int8 scale).
template <typename Acc>
struct CodeDec {
  float two_q;
  int f16;
  Acc sc[kMaxPops];  // int8 scale of each source population of the network
  __device__ __forceinline__ Acc operator()(uint32_t e) const {
    const uint32_t code = e >> kCodeShift;
    if (f16) {
      __half_raw r;
      r.x = (unsigned short)code;
      return (Acc)__builtin_rintf(__half2float(__half(r)) * two_q);
    }
    const Acc q = (Acc)(int8_t)(uint8_t)(code & 0xFFu);
    const uint32_t pop = (code >> 8) & 3u;
    const Acc s = pop == 0u ? sc[0] : pop == 1u ? sc[1] : pop == 2u ? sc[2] : sc[3];
    return q * s;
  }
};

// Decoder for the entries of tile `tile` (uniform loads).
template <typename Acc>
__device__ __forceinline__ CodeDec<Acc> code_dec(const StepArgs& a, int tile) {
  CodeDec<Acc> d;
  d.two_q = a.two_q;
  d.f16 = a.q_code == kCodeF16;
#pragma unroll
  for (int q = 0; q < kMaxPops; ++q) d.sc[q] = 0;
  if (a.q_code == kCodeI8) {
    const int64_t b = (int64_t)a.P * a.nets[a.tile_net[tile]].mbase;
#pragma unroll
    for (int q = 0; q < kMaxPops; ++q)
      if (q < a.P) d.sc[q] = (Acc)a.sfix[b + q];
  }
  return d;
}

// Entry views: the in-tile index | delay index << 10 (x) and the
// fixed-point efficacy (w) of each format.  Packed queue entries carry no
// delay index.
struct PackedEntry {
  uint32_t v;
};
struct CodeEntry {
  uint32_t v;
};
template <typename Acc>
__device__ __forceinline__ uint32_t ent_x(const QEntry<Acc>& e) { return e.x(); }
__device__ __forceinline__ uint32_t ent_x(PackedEntry e) { return e.v & 1023u; }
__device__ __forceinline__ uint32_t ent_x(CodeEntry e) { return e.v & 0xFFFFu; }
template <typename Acc>
__device__ __forceinline__ Acc ent_w(const QEntry<Acc>& e, const CodeDec<Acc>&) {
  return e.w();
}
template <typename Acc>
__device__ __forceinline__ Acc ent_w(PackedEntry e, const CodeDec<Acc>&) {
  return (Acc)((int32_t)e.v >> 10);
}
template <typename Acc>
__device__ __forceinline__ Acc ent_w(CodeEntry e, const CodeDec<Acc>& d) {
  return d(e.v);
}

// Event queues of one tile.  At step t the tile sums the queue of slot
// t mod D and the events of its inbox of step t-1 that arrive now
// (gather_now, before the neuron update); the other events of that inbox are
// moved into the tile's per-slot queues (route_inbox), off the update's
// path: in the delivery kernel of the same step for the split schedule.
// Entries are loaded kQBatch per thread at a time before any is used, so
// that their memory latency is paid once per batch.
constexpr int kQBatch = 8;

// Packed queue entry (int32 inputs whose efficacies all fit 21 bits):
// fixed-point efficacy << 10 | in-tile index.
__device__ __forceinline__ uint32_t pack_entry(int32_t w, uint32_t idx) {
  return ((uint32_t)w << 10) | idx;
}

// The batches of gather_now: the current queue (entries CE) and the inbox
// of step t-1 (entries IE), kQBatch entries per thread at a time.
template <typename Acc, typename CE, typename IE>
__device__ __forceinline__ void gather_batches(const CE* cq, const IE* iq, uint32_t n_cur,
                                               uint32_t n_in, Acc* s_in,
                                               const CodeDec<Acc>& dec) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const uint32_t n_max = n_cur > n_in ? n_cur : n_in;
  for (uint32_t r0 = 0; r0 < n_max; r0 += (uint32_t)nth * kQBatch) {
    CE ce[kQBatch];
    IE ie[kQBatch];
#pragma unroll
    for (int u = 0; u < kQBatch; ++u) {
      const uint32_t e = r0 + (uint32_t)(u * nth + tid);
      if (e < n_cur) ce[u] = cq[e];
      if (e < n_in) ie[u] = iq[e];
    }
#pragma unroll
    for (int u = 0; u < kQBatch; ++u) {
      const uint32_t e = r0 + (uint32_t)(u * nth + tid);
      if (e < n_cur) lds_add<Acc>(&s_in[ent_x(ce[u]) & 1023u], ent_w<Acc>(ce[u], dec));
      if (e < n_in && (ent_x(ie[u]) >> 10) == 0u)  // delay d_min = 1
        lds_add<Acc>(&s_in[ent_x(ie[u]) & 1023u], ent_w<Acc>(ie[u], dec));
    }
  }
}

// Entry formats of queues and inboxes, fixed per kernel instance: QEntry in
// both; packed queue entries with QEntry inboxes; code entries in both.
constexpr int kFmtWide = 0;
constexpr int kFmtPacked = 1;
constexpr int kFmtCode = 2;

template <typename Acc, int FMT>
__device__ __forceinline__ void gather_now(const StepArgs& a, int tile, const StepTime& T,
                                           Acc* s_in) {
  const int D = a.D;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int cur = (int)T.slot;
  const uint32_t par = (T.t - 1u) & 1u;
  const uint32_t qn = a.q_cnt[(int64_t)tile * D + cur];
  const uint32_t n_cur = qn < (uint32_t)a.q_cap ? qn : (uint32_t)a.q_cap;
  uint32_t n_in = 0;
  if (a.d_min == 1) {  // only then can an event of step t-1 arrive at t
    const uint32_t got = a.in_cnt[((int64_t)par * a.n_tiles + tile) * kInboxStride];
    n_in = got < (uint32_t)a.in_cap ? got : (uint32_t)a.in_cap;
  }
  for (int k = tid; k < 1024; k += nth) s_in[k] = 0;
  lds_barrier();
  const int64_t qo = ((int64_t)tile * D + cur) * a.q_cap;
  const int64_t io = ((int64_t)par * a.n_tiles + tile) * a.in_cap;
  if constexpr (FMT == kFmtCode) {
    const CodeDec<Acc> dec = code_dec<Acc>(a, tile);
    gather_batches<Acc>(static_cast<const CodeEntry*>(a.q_q) + qo,
                        static_cast<const CodeEntry*>(a.in_q) + io, n_cur, n_in, s_in, dec);
  } else {
    const CodeDec<Acc> none{};
    if constexpr (FMT == kFmtPacked)
      gather_batches<Acc>(static_cast<const PackedEntry*>(a.q_q) + qo,
                          static_cast<const QEntry<Acc>*>(a.in_q) + io, n_cur, n_in, s_in, none);
    else
      gather_batches<Acc>(static_cast<const QEntry<Acc>*>(a.q_q) + qo,
                          static_cast<const QEntry<Acc>*>(a.in_q) + io, n_cur, n_in, s_in, none);
  }
  lds_barrier();
  // every thread has used the count and the slot mark: the current queue
  // is empty and the slot cleared now
  if (tid == 0) {
    a.q_cnt[(int64_t)tile * D + cur] = 0;
    a.s_dirty[(int64_t)tile * D + cur] = 0u;
  }
}

// Dynamic LDS of the delivery blocks: the prefix of the tile counts
// (per-tile spike lists), then the staging of the inbox entries, 256 per
// wavefront.
constexpr size_t kStageBytes = 4 * 256 * 8;
// Block-merged reservations: an LDS hash of the target tiles of the four
// chunks a delivery block handles at once (key, events, inbox base).
constexpr int kHashBits = 10;
constexpr int kHash = 1 << kHashBits;      // >= the runs of 4 chunks (4 x 256)
constexpr uint32_t kHashEmpty = 0xFFFFFFFFu;
constexpr size_t kHashBytes = 3 * kHash * 4;
static_assert(kHash == 4 * 256, "one uint4 of hash keys per thread of a 256-thread block");
__host__ __device__ inline uint32_t stage_offset_words(const StepArgs& a) {
  return a.spk_lists ? 0u : ((uint32_t)a.n_tiles + 3u) / 4u * 4u;
}

// LDS of route_inbox.
template <typename Acc>
struct RouteLds {
  Acc sw[kStage];                 // routed events, grouped by slot
  uint16_t sx[kStage];
  uint8_t ss[kStage];
  uint32_t qc[kQueueMaxSlots];    // queue counts before this step
  uint32_t cnew[kQueueMaxSlots];  // events routed to each slot now
  uint32_t off[kQueueMaxSlots];   // their first staging position
};

// Moves the events of the inbox of step t-1 that arrive after t into the
// tile's per-slot queues, one contiguous run per slot (past the staging
// space or a full queue they are added into the slot), and empties the
// inbox.  The queue of slot t mod D is neither read nor written.
template <typename Acc, typename IE>
__device__ __forceinline__ void route_entries(const StepArgs& a, int tile, const StepTime& T,
                                              RouteLds<Acc>& L) {
  constexpr bool CODE = std::is_same<IE, CodeEntry>::value;
  const int D = a.D;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int cur = (int)T.slot;
  const uint32_t par = (T.t - 1u) & 1u;
  const int64_t ic = ((int64_t)par * a.n_tiles + tile) * kInboxStride;
  const uint32_t got = a.in_cnt[ic];
  const uint32_t n_in = got < (uint32_t)a.in_cap ? got : (uint32_t)a.in_cap;
  for (int k = tid; k < D; k += nth) {
    L.qc[k] = a.q_cnt[(int64_t)tile * D + k];
    L.cnew[k] = 0;
  }
  lds_barrier();
  Acc* slots = static_cast<Acc*>(a.slots);
  const IE* iq = static_cast<const IE*>(a.in_q) + ((int64_t)par * a.n_tiles + tile) * a.in_cap;
  QEntry<Acc>* qw = static_cast<QEntry<Acc>*>(a.q_q);
  const int64_t qb = (int64_t)tile * D * a.q_cap;
  const CodeDec<Acc> dec = code_dec<Acc>(a, tile);
  for (uint32_t r0 = 0; r0 < n_in; r0 += (uint32_t)nth * kQBatch) {
    IE ie[kQBatch];
    int sl[kQBatch];
    uint32_t rk[kQBatch];
#pragma unroll
    for (int u = 0; u < kQBatch; ++u) {
      const uint32_t e = r0 + (uint32_t)(u * nth + tid);
      if (e < n_in) ie[u] = iq[e];
    }
#pragma unroll
    for (int u = 0; u < kQBatch; ++u) {
      sl[u] = -1;
      if (r0 + (uint32_t)(u * nth + tid) < n_in) {
        const uint32_t x = ent_x(ie[u]);
        const int dk = (int)(x >> 10) < a.n_del ? (int)(x >> 10) : a.n_del - 1;
        const int off = a.d_min + dk - 1;  // arrival in off steps: 0 .. D - 2
        if (off > 0) {
          int s2 = cur + off;
          if (s2 >= D) s2 -= D;
          sl[u] = s2;
          rk[u] = atomicAdd(&L.cnew[s2], 1u);
        }
      }
    }
    lds_barrier();
    if (tid < 64) {  // exclusive scan of the per-slot counts (D <= 128)
      const uint32_t c0 = 2 * tid < D ? L.cnew[2 * tid] : 0u;
      const uint32_t c1 = 2 * tid + 1 < D ? L.cnew[2 * tid + 1] : 0u;
      uint32_t v = c0 + c1;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t w = __shfl_up(v, o);
        if (tid >= o) v += w;
      }
      const uint32_t ex = v - c0 - c1;
      if (2 * tid < D) L.off[2 * tid] = ex;
      if (2 * tid + 1 < D) L.off[2 * tid + 1] = ex + c0;
    }
    lds_barrier();
#pragma unroll
    for (int u = 0; u < kQBatch; ++u) {
      if (sl[u] < 0) continue;
      const uint32_t sp = L.off[sl[u]] + rk[u];
      const uint32_t idx = ent_x(ie[u]) & 1023u;
      if (sp < (uint32_t)kStage) {
        L.sx[sp] = (uint16_t)idx;
        L.ss[sp] = (uint8_t)sl[u];
        if constexpr (CODE)
          L.sw[sp] = (Acc)ie[u].v;  // the entry itself, moved unchanged
        else
          L.sw[sp] = ie[u].w();
      } else {
        atomic_add_fix<Acc>(slots + (int64_t)sl[u] * a.N_pad + (int64_t)tile * 1024 + idx,
                            ent_w<Acc>(ie[u], dec));
        a.s_dirty[(int64_t)tile * D + sl[u]] = 1u;
      }
    }
    lds_barrier();
    const uint32_t total = L.off[D - 1] + L.cnew[D - 1];
    const uint32_t staged = total < (uint32_t)kStage ? total : (uint32_t)kStage;
    for (uint32_t e = tid; e < staged; e += nth) {
      const int s2 = L.ss[e];
      const uint32_t gpos = L.qc[s2] + (e - L.off[s2]);
      if (gpos < (uint32_t)a.q_cap) {
        if (CODE) {
          static_cast<uint32_t*>(a.q_q)[qb + (int64_t)s2 * a.q_cap + gpos] = (uint32_t)L.sw[e];
        } else if (sizeof(Acc) == 4 && a.q_packed) {
          static_cast<uint32_t*>(a.q_q)[qb + (int64_t)s2 * a.q_cap + gpos] =
              pack_entry((int32_t)L.sw[e], L.sx[e]);
        } else {
          qw[qb + (int64_t)s2 * a.q_cap + gpos] = QEntry<Acc>::make(L.sx[e], L.sw[e]);
        }
      } else {
        const Acc w = CODE ? dec((uint32_t)L.sw[e]) : L.sw[e];
        atomic_add_fix<Acc>(slots + (int64_t)s2 * a.N_pad + (int64_t)tile * 1024 + L.sx[e], w);
        a.s_dirty[(int64_t)tile * D + s2] = 1u;
      }
    }
    lds_barrier();
    // queue counts after this round: staged events only (the rest went to
    // the slots)
    for (int k = tid; k < D; k += nth) {
      const uint32_t o = L.off[k], c = L.cnew[k];
      const uint32_t st = o >= (uint32_t)kStage ? 0u : (o + c <= (uint32_t)kStage ? c : kStage - o);
      L.qc[k] += st;
      L.cnew[k] = 0;
    }
    lds_barrier();
  }
  // every thread has used the inbox count by now
  if (tid == 0) a.in_cnt[ic] = 0;
  for (int k = tid; k < D; k += nth)
    if (k != cur) a.q_cnt[(int64_t)tile * D + k] = L.qc[k];
}

// CODE: code entries (binary16 and int8 efficacies), else QEntry inboxes.
template <typename Acc, bool CODE>
__device__ __forceinline__ void route_inbox(const StepArgs& a, int tile, const StepTime& T,
                                            RouteLds<Acc>& L) {
  if constexpr (CODE)
    route_entries<Acc, CodeEntry>(a, tile, T, L);
  else
    route_entries<Acc, QEntry<Acc>>(a, tile, T, L);
}

// Entry q of a four-entry array of uniform values, without indexing; the
// update is compiled for NP = 2 populations (q in 0..1) or up to 4.
template <int NP, typename T>
__device__ __forceinline__ T sel(const T (&v)[kMaxPops], int q) {
  if (NP == 2) return q ? v[1] : v[0];
  return q == 0 ? v[0] : q == 1 ? v[1] : q == 2 ? v[2] : v[3];
}

// Population of module-local index l from the ends h[0..2] of the first
// three populations.
template <int NP>
__device__ __forceinline__ int pop_index(int l, int h0, int h1, int h2) {
  if (NP == 2) return l >= h0 ? 1 : 0;
  return (l >= h0) + (l >= h1) + (l >= h2);
}

// ------------------------------------------------------------------------
// Neuron update of the 4 neurons i0..i0+3 (global indices) of one thread at
// step t; nd is the tile's network.  neuron_load reads and clears the input
// slot, reads the state and adds the external drive; neuron_finish adds the
// queued inputs (s_in, may be null), integrates Eq. 2 and returns the
// spiking neurons as a mask (compact_spikes lists them).  Counters of the random draws
// use the network's own neuron indices, so a network in a batch draws what
// it draws alone.
template <typename Acc>
struct NeuronRegs {
  Acc I[4];
  float V[4], c[4];
  uint32_t r4;
};

// Where the four neurons of a thread sit: global index i0 of the first,
// its network-local index il0 (a multiple of 4), and the module and
// module-local index of il0.
struct NeuronPos {
  uint32_t i0, il0, m0;
  int l0;
};

__device__ __forceinline__ NeuronPos neuron_pos(const NetDev& nd, int tile, int tid) {
  NeuronPos P;
  P.i0 = ((uint32_t)tile * 256u + (uint32_t)tid) * 4u;
  P.il0 = P.i0 - (uint32_t)nd.base;
  P.m0 = module_of(nd, P.il0);
  P.l0 = (int)(P.il0 - P.m0 * (uint32_t)nd.K);
  return P;
}

template <typename Acc, int NP>
__device__ __forceinline__ void neuron_load(const StepArgs& a, const NetDev& nd, int net,
                                            const NeuronPos& P, const StepTime& T,
                                            NeuronRegs<Acc>& R) {
  const uint32_t i0 = P.i0, t = T.t;
  Acc* sl = static_cast<Acc*>(a.slots) + ((size_t)T.slot * (size_t)a.N_pad + i0);
  // with queues the slot holds input only where an event found its queue
  // full (marked per tile and slot); gather_now clears the mark
  const bool marked = a.q_cap == 0 || a.s_dirty[(i0 >> 10) * (uint32_t)a.D + T.slot] != 0u;
  if (!marked) {
#pragma unroll
    for (int j = 0; j < 4; ++j) R.I[j] = 0;
  } else if (sizeof(Acc) == 4) {
    const int4 v = *reinterpret_cast<const int4*>(sl);
    R.I[0] = v.x; R.I[1] = v.y; R.I[2] = v.z; R.I[3] = v.w;
    *reinterpret_cast<int4*>(sl) = make_int4(0, 0, 0, 0);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      R.I[j] = sl[j];
      sl[j] = 0;
    }
  }
  // the state streams through once per step: non-temporal loads and
  // stores keep it from displacing the tables and entries in L2
  const NtF4 V4 = __builtin_nontemporal_load(reinterpret_cast<const NtF4*>(a.V + i0));
  const NtF4 c4 = __builtin_nontemporal_load(reinterpret_cast<const NtF4*>(a.c + i0));
  R.r4 = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(a.ref + i0));
  R.V[0] = V4.x; R.V[1] = V4.y; R.V[2] = V4.z; R.V[3] = V4.w;
  R.c[0] = c4.x; R.c[1] = c4.y; R.c[2] = c4.z; R.c[3] = c4.w;

  // external Poisson drive generated on the fly: counts from word j of
  // (il0/4, t, EXT); efficacies 2b and 2b+1 of neuron j from word j of
  // (il0/4, t, EXTJ | b << 8), high half then low half
  const uint32_t g = P.il0 >> 2;
  const uint4 u = philox10(make_uint4(g, t, 0u, kTagExt), nd.key0, nd.key1);
  const uint32_t uu[4] = {u.x, u.y, u.z, u.w};
  int q[4], k[4], npj[4];
  const int h0 = nd.pop_hi[0], h1 = nd.pop_hi[1], h2 = nd.pop_hi[2];
  const int np[kMaxPops] = {nd.n_pois[0], nd.n_pois[1], NP > 2 ? nd.n_pois[2] : 0,
                            NP > 2 ? nd.n_pois[3] : 0};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int lj = P.l0 + j;
    if (lj >= nd.K) lj -= nd.K;
    q[j] = pop_index<NP>(lj, h0, h1, h2);
    k[j] = 0;
    npj[j] = sel<NP>(np, q[j]);
  }
  // Poisson counts: the number of thresholds (increasing, uniform over the
  // block) not above the draw; the scan of a neuron stops at its first
  // threshold above the draw, the wavefront's once no lane goes on (most
  // counts are 0 or 1)
  bool on[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) on[j] = true;
  for (int x = 0; x < kMaxPois; ++x) {
    const uint32_t th[kMaxPops] = {nd.pois[0][x], nd.pois[1][x],
                                   NP > 2 ? nd.pois[2][x] : 0u, NP > 2 ? nd.pois[3][x] : 0u};
    bool any = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      on[j] = on[j] && x < npj[j] && uu[j] >= sel<NP>(th, q[j]);
      k[j] += on[j] ? 1 : 0;
      any |= on[j];
    }
    if (!__any(any)) break;
  }
  int kmax = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) kmax = k[j] > kmax ? k[j] : kmax;
  const Acc* jx = static_cast<const Acc*>(a.jx) + (size_t)net * kMaxPops * kQuantN;
  for (int b = 0; 2 * b < kmax; ++b) {
    const uint4 v = philox10(make_uint4(g, t, 0u, kTagExtJ | ((uint32_t)b << 8)), nd.key0, nd.key1);
    const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
    Acc e0[4], e1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {  // issue the table loads before any is used
      e0[j] = 2 * b < k[j] ? jx[q[j] * kQuantN + (vv[j] >> 16)] : (Acc)0;
      e1[j] = 2 * b + 1 < k[j] ? jx[q[j] * kQuantN + (vv[j] & 0xFFFFu)] : (Acc)0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) R.I[j] += e0[j] + e1[j];
  }
}

template <typename Acc, int NP>
__device__ __forceinline__ uint32_t neuron_finish(const StepArgs& a, const NetDev& nd,
                                                  const NeuronPos& P, const StepTime& T,
                                                  NeuronRegs<Acc>& R, const Acc* s_in) {
  if (s_in) {  // this thread's four entries of the tile's queue sums
#pragma unroll
    for (int j = 0; j < 4; ++j) R.I[j] += s_in[4 * threadIdx.x + j];
  }
  const uint32_t i0 = P.i0;
  const int l0 = P.l0;
  // per-population constants: uniform loads, selected per lane.  NP = 3:
  // up to four populations whose constants form two classes (entry 1 holds
  // those of population cls_rep, where class 1 begins), selected two-way
  constexpr int NS = NP == 3 ? 2 : NP;
  const int r1 = NP == 3 ? nd.cls_rep : 1;
  const float Pm[kMaxPops] = {nd.Pm[0], nd.Pm[r1], nd.Pm[2], nd.Pm[3]};
  const float Pc[kMaxPops] = {nd.Pc[0], nd.Pc[r1], nd.Pc[2], nd.Pc[3]};
  const float PVc[kMaxPops] = {nd.PVc[0], nd.PVc[r1], nd.PVc[2], nd.PVc[3]};
  const float It[kMaxPops] = {nd.Iterm[0], nd.Iterm[r1], nd.Iterm[2], nd.Iterm[3]};
  const float E[kMaxPops] = {nd.E[0], nd.E[r1], nd.E[2], nd.E[3]};
  const float Vth[kMaxPops] = {nd.Vth[0], nd.Vth[r1], nd.Vth[2], nd.Vth[3]};
  const float Vr[kMaxPops] = {nd.Vr[0], nd.Vr[r1], nd.Vr[2], nd.Vr[3]};
  const float al[kMaxPops] = {nd.alpha[0], nd.alpha[r1], nd.alpha[2], nd.alpha[3]};
  const int na[kMaxPops] = {nd.n_arp[0], nd.n_arp[r1], nd.n_arp[2], nd.n_arp[3]};
  const int h0 = nd.pop_hi[0], h1 = nd.pop_hi[1], h2 = nd.pop_hi[2];
  const int c_hi = NP == 3 ? nd.cls_hi : 0;
  uint32_t r_out = 0, mask = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int lj = l0 + j;
    if (lj >= nd.K) lj -= nd.K;
    const int qq = pop_index<NP>(lj, h0, h1, h2);
    const int qs = NP == 3 ? (lj >= c_hi ? 1 : 0) : qq;  // constants' entry
    uint32_t rj = (R.r4 >> (8 * j)) & 0xFFu;
    if ((int64_t)P.il0 + j < nd.N) {
      const float dv = fix_to_f32(R.I[j]) * a.inv2q;
      float Vj = R.V[j], cj = R.c[j];
      const float Pcq = sel<NS>(Pc, qs), Eq = sel<NS>(E, qs);
      bool spk = false;
      if (rj > 0) {
        rj -= 1;
        cj = cj * Pcq;
      } else {
        float vv = Vj - Eq;
        vv = vv * sel<NS>(Pm, qs);
        vv = Eq + vv;
        const float cc = cj * sel<NS>(PVc, qs);
        vv = vv - cc;
        vv = vv + sel<NS>(It, qs);
        vv = vv + dv;
        cj = cj * Pcq;
        if (vv > sel<NS>(Vth, qs)) {
          spk = true;
          vv = sel<NS>(Vr, qs);
          cj = cj + sel<NS>(al, qs);
          rj = (uint32_t)sel<NS>(na, qs);
        }
        Vj = vv;
      }
      R.V[j] = Vj;
      R.c[j] = cj;
      if (spk) {
        mask |= 1u << j;
        if (a.t_post) a.t_post[i0 + j] = (int32_t)T.t;  // plastic networks
        // population count of the rate bin (Sec. 2.3)
        const uint32_t mod = (uint32_t)nd.mbase + P.m0 + (l0 + j >= nd.K ? 1u : 0u);
        atomicAdd(&a.rates[((size_t)T.bin * (uint32_t)a.M + mod) * (uint32_t)a.P + qq], 1u);
      }
    }
    r_out |= rj << (8 * j);
  }
  __builtin_nontemporal_store(NtF4{R.V[0], R.V[1], R.V[2], R.V[3]},
                              reinterpret_cast<NtF4*>(a.V + i0));
  __builtin_nontemporal_store(NtF4{R.c[0], R.c[1], R.c[2], R.c[3]},
                              reinterpret_cast<NtF4*>(a.c + i0));
  __builtin_nontemporal_store(r_out, reinterpret_cast<uint32_t*>(a.ref + i0));
  return mask;
}

// Spikes of a block in neuron order: each thread holds up to four (bit j of
// mask: neuron i0 + j); the prefix within a wavefront comes from three
// ballots of the per-thread counts, the wavefront totals are exchanged in
// LDS (s_wt, one per wavefront).  Writes the ids in increasing order to
// s_spk and returns the block's count (the same in every thread); s_spk is
// read by other threads only after the next barrier.
__device__ __forceinline__ int compact_spikes(uint32_t mask, uint32_t i0, int32_t* s_spk,
                                              int* s_wt) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t c = (uint32_t)__popc(mask);
  const unsigned long long b0 = __ballot(c & 1u), b1 = __ballot(c & 2u), b2 = __ballot(c & 4u);
  const unsigned long long lt = (1ull << lane) - 1ull;
  const int pre = __popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt);
  if (lane == 0) s_wt[wave] = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
  lds_barrier();
  int base = 0, total = 0;
  const int nw = (int)(blockDim.x >> 6);
  for (int w = 0; w < nw; ++w) {
    const int v = s_wt[w];
    base += w < wave ? v : 0;
    total += v;
  }
  int k = base + pre;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if ((mask >> j) & 1u) s_spk[k++] = (int32_t)(i0 + j);
  return total;
}

// Plasticity event of one synapse (Sec. 2.1): source spike at step ta,
// target's last spike tp; t_act and y are the synapse's state (the rule is
// documented with dpsnn_params; binary32, no contraction).
__device__ __forceinline__ void stdp_event(const StepArgs& a, int32_t ta, int32_t tp,
                                           int32_t& t_act, float& y) {
  const int32_t L = a.stdp_L;
  const float* Ep = a.stdp_tab;
  const float* Em = Ep + L;
  const float* Dy = Em + L;
  const int32_t tl = t_act;
  y = (tl >= 0 && ta - tl < L) ? y * Dy[ta - tl] : 0.0f;
  if (tl >= 0 && tp > tl && tp - tl < L && ta - tp < L) y = y + Ep[tp - tl] * Dy[ta - tp];
  if (tp >= 0 && ta - tp < L) y = y - Em[ta - tp];
  t_act = ta;
}

// One chunk of a row: 256 synapses (4 per lane) of row s from p0 = chunk *
// 256; targets, and the fixed-point efficacies (binary32 rows) or the
// stored codes (binary16 and int8 rows, decoded where a fixed-point value
// is needed, with the int8 scale of the source population), so that a
// code chunk holds no more registers than it needs.
template <typename Acc>
struct Chunk {
  int32_t s, p0;
  int tv[4];
  Acc wv[4];
  uint32_t cv[4];
  Acc scale;
};

// Fixed-point efficacy j of a loaded chunk.
template <typename Acc, int WDT>
__device__ __forceinline__ Acc chunk_fix(const StepArgs& a, const Chunk<Acc>& c, int j) {
  if constexpr (WDT == DPSNN_W_F32)
    return c.wv[j];
  else if constexpr (WDT == DPSNN_W_F16)
    return (Acc)__builtin_rintf(__half2float(__ushort_as_half((unsigned short)c.cv[j])) *
                                a.two_q);
  else
    return (Acc)(int8_t)(uint8_t)c.cv[j] * c.scale;
}

// Loads of a chunk (issued, not waited for: the values are used later).
template <typename Acc, int WDT>
__device__ __forceinline__ void chunk_load(const StepArgs& a, int32_t s, int p0, int lane,
                                           Chunk<Acc>& c) {
  c.s = s;
  c.p0 = p0;
  const int64_t rb = (int64_t)s * a.row_stride;
  int64_t scale = 0;
  int q_src = 0;  // source population (int8 codes)
  if (WDT == DPSNN_W_I8) {
    int32_t ms;
    module_pop(a, s, &ms, &q_src);
    scale = a.sfix[(int64_t)a.P * ms + q_src];
  }
  const int p = p0 + lane * 4;
  c.scale = (Acc)scale;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    c.tv[j] = 0;
    if (WDT == DPSNN_W_F32)
      c.wv[j] = 0;
    else
      c.cv[j] = 0;
  }
  if (p < a.K_out) {  // rows are padded to a multiple of 4 words
    // a row is read once per spike: non-temporal loads, so that the
    // inboxes and queues written now and read in the next step stay cached
    const NtI4 tg = __builtin_nontemporal_load(reinterpret_cast<const NtI4*>(a.tgt + rb + p));
    c.tv[0] = tg.x; c.tv[1] = tg.y; c.tv[2] = tg.z; c.tv[3] = tg.w;
    if (WDT == DPSNN_W_F32) {
      const NtF4 w4 = __builtin_nontemporal_load(
          reinterpret_cast<const NtF4*>(static_cast<const float*>(a.w) + rb + p));
      c.wv[0] = (Acc)__builtin_rintf(w4.x * a.two_q);
      c.wv[1] = (Acc)__builtin_rintf(w4.y * a.two_q);
      c.wv[2] = (Acc)__builtin_rintf(w4.z * a.two_q);
      c.wv[3] = (Acc)__builtin_rintf(w4.w * a.two_q);
    } else if (WDT == DPSNN_W_F16) {
      const NtU16x4 h4 = __builtin_nontemporal_load(
          reinterpret_cast<const NtU16x4*>(static_cast<const uint16_t*>(a.w) + rb + p));
      const uint32_t hv[4] = {h4.x, h4.y, h4.z, h4.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) c.cv[j] = hv[j];
    } else {
      const uint32_t b4 = __builtin_nontemporal_load(
          reinterpret_cast<const uint32_t*>(static_cast<const int8_t*>(a.w) + rb + p));
#pragma unroll
      for (int j = 0; j < 4; ++j)  // element p + j is byte j
        c.cv[j] = (b4 >> (8 * j) & 0xFFu) | (uint32_t)q_src << 8;
    }
  }
}

// Plasticity events of a loaded chunk: when the source is excitatory its
// synapses register the activation (before the events are delivered).
template <typename Acc>
__device__ __forceinline__ void chunk_plasticity(const StepArgs& a, const Chunk<Acc>& c,
                                                 uint32_t t, int lane) {
  const int64_t rb = (int64_t)c.s * a.row_stride;
  const int p = c.p0 + lane * 4;
  int32_t ms;
  int q;
  module_pop(a, c.s, &ms, &q);
  if (a.nets[a.tile_net[c.s >> 10]].exc[q] && p < a.K_out) {
    int4 ta4 = *reinterpret_cast<const int4*>(a.syn_t + rb + p);
    float4 y4 = *reinterpret_cast<const float4*>(a.syn_y + rb + p);
    int32_t tav[4] = {ta4.x, ta4.y, ta4.z, ta4.w};
    float yv[4] = {y4.x, y4.y, y4.z, y4.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (p + j < a.K_out)
        stdp_event(a, (int32_t)t, a.t_post[c.tv[j] & kTargetMask], tav[j], yv[j]);
    *reinterpret_cast<int4*>(a.syn_t + rb + p) = make_int4(tav[0], tav[1], tav[2], tav[3]);
    *reinterpret_cast<float4*>(a.syn_y + rb + p) = make_float4(yv[0], yv[1], yv[2], yv[3]);
  }
}

// Delivery of a loaded chunk.  s_b is the wavefront's 256-entry LDS
// scratch, s_e (or null: entries stored from the lanes that hold them) its
// 256-entry staging of the inbox entries.  Every lane of the wavefront takes
// part, also past the end of the row.
template <typename Acc, int WDT>
__device__ __forceinline__ void chunk_deliver(const StepArgs& a, const Chunk<Acc>& c,
                                              const StepTime& T, int lane, uint32_t* s_b,
                                              unsigned long long* s_e,
                                              uint32_t* s_hash = nullptr, bool valid = true) {
  const int p0 = c.p0;
  const int p = p0 + lane * 4;
  const int* tv = c.tv;
  const uint32_t* cv = c.cv;
  const uint32_t t = T.t;
  int slot0 = (int)T.slot + a.d_min;  // slot of arrival at t + d_min
  if (slot0 >= a.D) slot0 -= a.D;
  Acc* slots = static_cast<Acc*>(a.slots);
  if (a.q_cap == 0) {
    if (!valid) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (p + j < a.K_out) {
        int sl = slot0 + (int)((uint32_t)tv[j] >> kDelayShift);
        if (sl >= a.D) sl -= a.D;
        const int32_t target = tv[j] & kTargetMask;
        atomic_add_fix<Acc>(slots + (int64_t)sl * a.N_pad + target, chunk_fix<Acc, WDT>(a, c, j));
      }
    }
    return;
  }
  // Rows are sorted by target, so the events to one tile form runs.  The
  // first event of a run reserves room for the whole run in that tile's
  // inbox; the others take the following entries.
  const int end = p0 + 256 < a.K_out ? p0 + 256 : a.K_out;
  int tl[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) tl[j] = valid && p + j < end ? (tv[j] & kTargetMask) >> 10 : -1;
  int prev = __shfl_up(tl[3], 1);
  if (lane == 0) prev = -2;
  bool f[4];
  f[0] = tl[0] >= 0 && tl[0] != prev;
#pragma unroll
  for (int j = 1; j < 4; ++j) f[j] = tl[j] >= 0 && tl[j] != tl[j - 1];
  // start of the run of each event: the last start at or before it
  int last = -1, first = 1 << 30;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (f[j]) {
      last = p + j;
      first = first < p + j ? first : p + j;
    }
  }
  // Run starts increase with the lane, so the last start before this lane
  // is the last start of the nearest lower lane that has one, and the
  // first start after it the first start of the nearest higher such lane:
  // one ballot and two lane reads.
  const uint64_t heads = __ballot(last >= 0);  // uniform
  const uint32_t h_lo = (uint32_t)heads, h_hi = (uint32_t)(heads >> 32);
  const uint32_t l5 = (uint32_t)lane & 31u;
  const uint32_t m_lt = (1u << l5) - 1u, m_gt = ~((2u << l5) - 1u);  // l5 = 31: 2 << 31 = 0
  // nearest lower lane with a start (-1: none)
  const uint32_t b_own = (lane < 32 ? h_lo : h_hi) & m_lt;
  const int lo_lane = b_own ? (lane & 32) + 31 - __clz(b_own)
                            : (lane >= 32 && h_lo ? 31 - __clz(h_lo) : -1);
  // nearest higher lane with a start (64: none)
  const uint32_t a_own = (lane < 32 ? h_lo : h_hi) & (l5 == 31u ? 0u : m_gt);
  const int hi_lane = a_own ? (lane & 32) + __ffs(a_own) - 1
                            : (lane < 32 && h_hi ? 32 + __ffs(h_hi) - 1 : 64);
  const int lo_last = __shfl(last, lo_lane < 0 ? lane : lo_lane);
  const int hi_first = __shfl(first, hi_lane > 63 ? lane : hi_lane);
  const int carry = lo_lane < 0 ? -1 : lo_last;
  const int nxt = hi_lane > 63 ? 1 << 30 : hi_first;
  int rs[4];
  {
    int c = carry;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (f[j]) c = p + j;
      rs[j] = c;
    }
  }
  const uint32_t par = t & 1u;
  uint32_t len[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    len[j] = 0;
    if (f[j]) {
      int ne = nxt;
#pragma unroll
      for (int k = 3; k > j; --k)
        if (f[k]) ne = p + k;
      if (ne > end) ne = end;
      len[j] = (uint32_t)(ne - (p + j));
    }
  }
  if (s_hash) {
    // Reservations merged over the block's four chunks (the same chunk of
    // four spikes in a row of the spike list, whose rows share target
    // tiles): each run enters its tile in the LDS hash and takes its rank
    // among the block's events to that tile; one returning atomic per tile
    // then reserves them all, and each run's base is that reservation plus
    // its rank.  Every wavefront of the block passes both barriers.
    uint32_t* s_hk = s_hash;
    uint32_t* s_hc = s_hash + kHash;
    uint32_t* s_hb = s_hash + 2 * kHash;
    // each run's hash entry and rank (< 2^11) wait in the wavefront's
    // scratch across the barriers, not in registers
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (f[j]) {
        const uint32_t key = (uint32_t)tl[j];
        uint32_t h = (key * 2654435761u) >> (32 - kHashBits);
        // at most kHash distinct tiles per round: a free or matching
        // entry is always found
        for (;;) {
          const uint32_t old = atomicCAS(&s_hk[h], kHashEmpty, key);
          if (old == kHashEmpty || old == key) break;
          h = (h + 1) & (uint32_t)(kHash - 1);
        }
        s_b[p + j - p0] = h << 16 | atomicAdd(&s_hc[h], len[j]);
      }
    }
    lds_barrier();
    {
      const int h0 = (int)threadIdx.x * 4;  // kHash == 4 * blockDim.x
      const uint4 k4 = *reinterpret_cast<const uint4*>(s_hk + h0);
      const uint32_t kk[4] = {k4.x, k4.y, k4.z, k4.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (kk[u] != kHashEmpty) {
          s_hb[h0 + u] = atomicAdd(&a.in_cnt[((int64_t)par * a.n_tiles + kk[u]) * kInboxStride],
                                   s_hc[h0 + u]);
          s_hk[h0 + u] = kHashEmpty;
          s_hc[h0 + u] = 0;
        }
      }
    }
    lds_barrier();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (f[j]) {
        const uint32_t v = s_b[p + j - p0];
        s_b[p + j - p0] = s_hb[v >> 16] + (v & 0xFFFFu);
      }
    }
  } else {
    // reservations: one returning atomic per run
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (f[j])
        s_b[p + j - p0] =
            atomicAdd(&a.in_cnt[((int64_t)par * a.n_tiles + tl[j]) * kInboxStride], len[j]);
  }
  wave_lds_sync();
  if (s_e) {
    // Entries are staged in LDS and stored with lane l writing chunk
    // positions l, l + 64, l + 128, l + 192: consecutive lanes then write
    // consecutive entries of a run, so the stores coalesce.  Inbox index of
    // each entry (~0: none, an event past the inbox goes to its slot here).
    uint32_t off[4];
    unsigned long long ev[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      off[j] = ~0u;
      ev[j] = 0ull;
      if (tl[j] >= 0) {
        const uint32_t pos = s_b[rs[j] - p0] + (uint32_t)(p + j - rs[j]);
        const int32_t target = tv[j] & kTargetMask;
        const uint32_t dk = (uint32_t)tv[j] >> kDelayShift;
        const uint32_t x = (uint32_t)(target & 1023) | (dk << 10);
        if (pos < (uint32_t)a.in_cap) {
          off[j] = ((uint32_t)par * (uint32_t)a.n_tiles + (uint32_t)tl[j]) * (uint32_t)a.in_cap +
                   pos;
          if (WDT != DPSNN_W_F32 && a.q_code) {
            ev[j] = code_entry(cv[j], x);
          } else {
            const QEntry<Acc> e = QEntry<Acc>::make(x, chunk_fix<Acc, WDT>(a, c, j));
            ev[j] = *reinterpret_cast<const unsigned long long*>(&e);
          }
        } else {
          int sl = slot0 + (int)dk;
          if (sl >= a.D) sl -= a.D;
          atomic_add_fix<Acc>(slots + (int64_t)sl * a.N_pad + target, chunk_fix<Acc, WDT>(a, c, j));
          a.s_dirty[(int64_t)tl[j] * a.D + sl] = 1u;
        }
      }
    }
    wave_lds_sync();  // every lane has read its run bases
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      s_b[4 * lane + j] = off[j];
      s_e[4 * lane + j] = ev[j];
    }
    wave_lds_sync();
    const bool code = WDT != DPSNN_W_F32 && a.q_code;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t o = s_b[lane + 64 * j];
      if (o != ~0u) {
        const unsigned long long e = s_e[lane + 64 * j];
        if (code)
          static_cast<uint32_t*>(a.in_q)[o] = (uint32_t)e;
        else
          static_cast<unsigned long long*>(a.in_q)[o] = e;
      }
    }
    wave_lds_sync();  // s_b and s_e are written again by the next chunk
    return;
  }
  QEntry<Acc>* iq = static_cast<QEntry<Acc>*>(a.in_q);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (tl[j] >= 0) {
      const uint32_t pos = s_b[rs[j] - p0] + (uint32_t)(p + j - rs[j]);
      const int32_t target = tv[j] & kTargetMask;
      const uint32_t dk = (uint32_t)tv[j] >> kDelayShift;
      const uint32_t x = (uint32_t)(target & 1023) | (dk << 10);
      if (pos < (uint32_t)a.in_cap) {
        const int64_t o = ((int64_t)par * a.n_tiles + tl[j]) * a.in_cap + pos;
        if (WDT != DPSNN_W_F32 && a.q_code)
          static_cast<uint32_t*>(a.in_q)[o] = code_entry(cv[j], x);
        else
          iq[o] = QEntry<Acc>::make(x, chunk_fix<Acc, WDT>(a, c, j));
      } else {
        int sl = slot0 + (int)dk;
        if (sl >= a.D) sl -= a.D;
        atomic_add_fix<Acc>(slots + (int64_t)sl * a.N_pad + target, chunk_fix<Acc, WDT>(a, c, j));
        a.s_dirty[(int64_t)tl[j] * a.D + sl] = 1u;
      }
    }
  }
  wave_lds_sync();  // s_b is written again by the wavefront's next chunk
}

__device__ __forceinline__ void record_spike(const StepArgs& a, int32_t id, uint32_t t,
                                             unsigned long long pos) {
  if (pos < (unsigned long long)a.spike_log_cap) a.log[pos] = make_int2((int)t, id);
}

// ------------------------------------------------------------------------
// Split schedule: neuron kernel, then the delivery kernel.
// Update of one tile of 1024 neurons by one block, and the tile's spike
// list (its own, or appended to one of the kSpkLists lists of the step).
template <typename Acc, int NP, int FMT>
__device__ __forceinline__ void update_tile(const StepArgs& a, const StepTime& T, int tile,
                                            int32_t* s_spk, Acc* s_in, int* s_wt,
                                            uint32_t* s_base) {
  const int tid = threadIdx.x;
  const uint32_t t = T.t;
  const int net = __builtin_amdgcn_readfirstlane(a.tile_net[tile]);
  const NetDev& nd = a.nets[net];
  const NeuronPos P = neuron_pos(nd, tile, tid);
  NeuronRegs<Acc> R;
  neuron_load<Acc, NP>(a, nd, net, P, T, R);
  if (a.q_cap)
    gather_now<Acc, FMT>(a, tile, T, s_in);
  else
    lds_barrier();
  const uint32_t mask = neuron_finish<Acc, NP>(a, nd, P, T, R, a.q_cap ? s_in : nullptr);
  const int n = compact_spikes(mask, P.i0, s_spk, s_wt);
  lds_barrier();
  if (!a.spk_lists) {  // the tile's own list and count
    int32_t* out = a.spk + (int64_t)tile * 1024;
    for (int k = tid; k < n; k += 256) out[k] = s_spk[k];
    if (tid == 0) a.blk_cnt[tile] = n;
    return;
  }
  if (n == 0) return;
  // append the tile's spikes to spike list g = (tile >> kSpkListShift) mod
  // kSpkLists of the step: the counters share the appends, and neighbouring
  // tiles, whose rows reach the same target tiles, follow each other in a
  // list (the merged reservations of delivery gain from that)
  const int g = (tile >> kSpkListShift) % kSpkLists;
  if (tid == 0)
    *s_base = atomicAdd(&a.spk_n[((t & 1u) * kSpkLists + g) * kSpkStride], (uint32_t)n);
  lds_barrier();
  // (a list holds every neuron of its tiles: the bound only guards)
  const uint32_t base = *s_base;
  const int64_t room = a.spk_cap - (int64_t)base;
  const int n_w = (int64_t)n < room ? n : (room > 0 ? (int)room : 0);
  int32_t* out = a.spk + (int64_t)g * a.spk_cap + base;
  for (int k = tid; k < n_w; k += 256) out[k] = s_spk[k];
}

template <typename Acc, int NP, int FMT>
__global__ void __launch_bounds__(256) k_neuron(StepArgs a, StepOff o) {
  __shared__ int32_t s_spk[1024];
  __shared__ Acc s_in[1024];
  __shared__ int s_wt[4];
  __shared__ uint32_t s_base;
  update_tile<Acc, NP, FMT>(a, step_time(a, o), blockIdx.x, s_spk, s_in, s_wt, &s_base);
}

// Spike number sidx of the step: per-tile lists, the tile found by binary
// search in the LDS prefix of the tile counts; or appended lists, found by
// the wavefront's prefix of the list counts (lane g: list g).
__device__ __forceinline__ int32_t spike_at(const StepArgs& a, int sidx, const int32_t* s_pref,
                                            uint32_t incl, uint32_t excl) {
  if (!a.spk_lists) {
    int l = 0, h = a.n_tiles - 1;  // first tile with s_pref[tile] > sidx
    while (l < h) {
      const int mid = (l + h) >> 1;
      if (s_pref[mid] > sidx)
        h = mid;
      else
        l = mid + 1;
    }
    const int first = l ? s_pref[l - 1] : 0;
    return __builtin_amdgcn_readfirstlane(a.spk[(int64_t)l * 1024 + (sidx - first)]);
  }
  // the first list whose inclusive prefix exceeds sidx
  const int g = (int)__popcll(__ballot(incl <= (uint32_t)sidx));
  const uint32_t first = __shfl(excl, g);
  return __builtin_amdgcn_readfirstlane(
      a.spk[(int64_t)g * a.spk_cap + ((uint32_t)sidx - first)]);
}

// Delivery of the step's spikes by one block (every thread takes part):
// wavefront wid of nw delivery wavefronts takes work items wid, wid + nw,
// ...  s_dyn: the dynamic LDS (tile-count prefix and entry staging), s_part
// and s_b: the block's small LDS arrays.  Block `lead` also advances the
// spike-log bases and clears the spike-list counters of the next step.
template <typename Acc, int WDT, bool PLAST, bool MERGE = false>
__device__ __forceinline__ void deliver_spikes(const StepArgs& a, const StepTime& T,
                                               int64_t wid, int64_t nw, bool lead,
                                               int32_t* s_dyn, int32_t* s_part,
                                               uint32_t (*s_b)[256],
                                               uint32_t* s_hash = nullptr) {
  const int tid = threadIdx.x;
  const int nb = a.n_tiles;
  const uint32_t t = T.t;
  const int lane = tid & 63;
  int32_t* s_pref = s_dyn;
  unsigned long long* s_stage =
      reinterpret_cast<unsigned long long*>(s_dyn + stage_offset_words(a));
  uint32_t incl = 0, excl = 0;
  int n_spk;
  if (!a.spk_lists) {
    // block-wide inclusive scan of the tile counts: a coalesced copy into
    // LDS, each thread scans a contiguous run, wavefront shuffles and one
    // exchange of the four wavefront totals
    for (int b = tid; b < nb; b += 256) s_pref[b] = a.blk_cnt[b];
    lds_barrier();
    const int per = (nb + 255) / 256;
    const int lo = tid * per;
    const int hi = lo + per < nb ? lo + per : nb;
    int run = 0;
    for (int b = lo; b < hi; ++b) run += s_pref[b];
    int inc = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(inc, off);
      if (lane >= off) inc += v;
    }
    if (lane == 63) s_part[tid >> 6] = inc;
    lds_barrier();
    int acc = inc - run;
    for (int w = 0; w < (tid >> 6); ++w) acc += s_part[w];
    for (int b = lo; b < hi; ++b) {
      acc += s_pref[b];
      s_pref[b] = acc;
    }
    if (tid == 255) s_part[4] = acc;
    lds_barrier();
    n_spk = s_part[4];
  } else {
    // the appended lists, one per lane: inclusive and exclusive prefix of
    // their counts
    uint32_t cnt = a.spk_n[((t & 1u) * kSpkLists + lane) * kSpkStride];
    if (cnt > (uint64_t)a.spk_cap) cnt = (uint32_t)a.spk_cap;
    incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t v = __shfl_up(incl, off);
      if (lane >= off) incl += v;
    }
    excl = incl - cnt;
    n_spk = (int)__shfl(incl, 63);
  }
  const unsigned long long log0 = a.log_base[t & 1];
  if (lead && tid == 0) {
    a.log_base[(t + 1) & 1] = log0 + (unsigned long long)n_spk;
    a.n_spikes[0] += (unsigned long long)n_spk;
  }
  // the list counters of the next step start from zero (nothing else reads
  // them in this step)
  if (a.spk_lists && lead && tid < kSpkLists)
    a.spk_n[(((t + 1u) & 1u) * kSpkLists + tid) * kSpkStride] = 0u;
  const int cpr = (a.K_out + 255) / 256;  // chunks per row
  if constexpr (MERGE) {
    // (with queues and appended spike lists only)
    // Block items: chunk bi mod cpr of the four spikes 4 (bi / cpr) + w,
    // wavefront w taking one; the block's wavefronts run the same rounds.
    const int wave = tid >> 6;
    const int64_t b = wid >> 2, nb = nw >> 2;
    const int64_t bitems = ((int64_t)n_spk + 3) / 4 * cpr;
    for (int h = tid; h < kHash; h += 256) {
      s_hash[h] = kHashEmpty;
      s_hash[kHash + h] = 0u;
    }
    lds_barrier();
    auto load_block_item = [&](int64_t bi, Chunk<Acc>& c) -> bool {
      const int64_t g = bi / cpr;
      const int chunk = (int)(bi - g * cpr);
      const int64_t sidx = 4 * g + wave;
      if (sidx >= n_spk) {
        c.s = 0;
        c.p0 = 0;
        return false;
      }
      const int32_t s = spike_at(a, (int)sidx, s_pref, incl, excl);
      if (chunk == 0 && lane == 0) record_spike(a, s, t, log0 + (unsigned long long)sidx);
      chunk_load<Acc, WDT>(a, s, chunk * 256, lane, c);
      return true;
    };
    Chunk<Acc> cur;
    bool v_cur = false;
    if (b < bitems) v_cur = load_block_item(b, cur);
    for (int64_t bi = b; bi < bitems; bi += nb) {
      Chunk<Acc> nxt;
      bool v_nxt = false;
      const bool more = bi + nb < bitems;
      if (more) v_nxt = load_block_item(bi + nb, nxt);
      if (PLAST && v_cur) chunk_plasticity<Acc>(a, cur, t, lane);
      chunk_deliver<Acc, WDT>(a, cur, T, lane, s_b[wave], s_stage + wave * 256, s_hash, v_cur);
      if (!more) break;
      cur = nxt;
      v_cur = v_nxt;
    }
  } else {
  const int64_t items = (int64_t)n_spk * cpr;
  // item it: chunk it mod cpr of spike number it / cpr.  The next item's
  // loads are issued before the current item is delivered.
  auto load_item = [&](int64_t it, Chunk<Acc>& c) {
    const int sidx = (int)(it / cpr);
    const int chunk = (int)(it - (int64_t)sidx * cpr);
    const int32_t s = spike_at(a, sidx, s_pref, incl, excl);
    if (chunk == 0 && lane == 0) record_spike(a, s, t, log0 + (unsigned long long)sidx);
    chunk_load<Acc, WDT>(a, s, chunk * 256, lane, c);
  };
  Chunk<Acc> cur;
  if (wid < items) load_item(wid, cur);
  for (int64_t it = wid; it < items; it += nw) {
    Chunk<Acc> nxt;
    const bool more = it + nw < items;
    if (more) load_item(it + nw, nxt);
    if (PLAST) chunk_plasticity<Acc>(a, cur, t, lane);
    chunk_deliver<Acc, WDT>(a, cur, T, lane, s_b[tid >> 6], s_stage + (tid >> 6) * 256);
    if (!more) break;
    cur = nxt;
  }
  }
}

template <typename Acc, int WDT, bool PLAST = false, bool MERGE = false>
__global__ void __launch_bounds__(256) k_deliver(StepArgs a, StepOff o) {
  // delivery blocks: inclusive prefix of the tile counts (per-tile lists)
  // and entry staging; routing blocks: their RouteLds
  extern __shared__ __align__(16) int32_t s_dyn[];
  __shared__ int32_t s_part[8];
  __shared__ uint32_t s_b[4][256];
  const StepTime T = step_time(a, o);
  if ((int)blockIdx.x >= a.deliver_blocks) {
    // routing of the inboxes of step t-1, one tile at a time
    RouteLds<Acc>& L = *reinterpret_cast<RouteLds<Acc>*>(s_dyn);
    const int nr = (int)gridDim.x - a.deliver_blocks;
    for (int tile = (int)blockIdx.x - a.deliver_blocks; tile < a.n_tiles; tile += nr)
      route_inbox<Acc, WDT != DPSNN_W_F32>(a, tile, T, L);
    return;
  }
  deliver_spikes<Acc, WDT, PLAST, MERGE>(
      a, T, (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), (int64_t)a.deliver_blocks * 4,
      blockIdx.x == 0, s_dyn, s_part, s_b,
      MERGE ? reinterpret_cast<uint32_t*>(s_dyn + stage_offset_words(a) + kStageBytes / 4)
            : nullptr);
}

// Fused schedule (small networks): the tile's own spikes are delivered by
// its four wavefronts right after the update.
template <typename Acc, int WDT, int NP>
__global__ void __launch_bounds__(256) k_step(StepArgs a, StepOff o) {
  __shared__ int32_t s_spk[1024];
  __shared__ Acc s_in[1024];
  __shared__ RouteLds<Acc> s_route;
  __shared__ uint32_t s_b[4][256];
  __shared__ int s_wt[4];
  __shared__ unsigned long long s_logbase;
  const int tid = threadIdx.x;
  const StepTime T = step_time(a, o);
  const uint32_t t = T.t;
  const int net = __builtin_amdgcn_readfirstlane(a.tile_net[blockIdx.x]);
  const NetDev& nd = a.nets[net];
  const NeuronPos P = neuron_pos(nd, blockIdx.x, tid);
  NeuronRegs<Acc> R;
  neuron_load<Acc, NP>(a, nd, net, P, T, R);
  if (!a.q_cap)
    lds_barrier();
  else if constexpr (WDT != DPSNN_W_F32)
    gather_now<Acc, kFmtCode>(a, blockIdx.x, T, s_in);
  else if (sizeof(Acc) == 4 && a.q_packed)
    gather_now<Acc, kFmtPacked>(a, blockIdx.x, T, s_in);
  else
    gather_now<Acc, kFmtWide>(a, blockIdx.x, T, s_in);
  const uint32_t mask = neuron_finish<Acc, NP>(a, nd, P, T, R, a.q_cap ? s_in : nullptr);
  const int n = compact_spikes(mask, P.i0, s_spk, s_wt);
  if (a.q_cap) route_inbox<Acc, WDT != DPSNN_W_F32>(a, blockIdx.x, T, s_route);  // barriers
  lds_barrier();
  if (n == 0) return;
  if (tid == 0) {
    // both log bases advance together in this schedule
    s_logbase = atomicAdd(&a.log_base[t & 1], (unsigned long long)n);
    atomicAdd(&a.log_base[(t + 1) & 1], (unsigned long long)n);
    atomicAdd(a.n_spikes, (unsigned long long)n);
  }
  lds_barrier();
  for (int k = tid; k < n; k += 256)
    record_spike(a, s_spk[k], t, s_logbase + (unsigned long long)k);
  const int lane = tid & 63, wave = tid >> 6;
  const int cpr = (a.K_out + 255) / 256;
  for (int it = wave; it < n * cpr; it += 4) {
    const int k = it / cpr;
    const int32_t s = __builtin_amdgcn_readfirstlane(s_spk[k]);
    Chunk<Acc> c;
    chunk_load<Acc, WDT>(a, s, (it - k * cpr) * 256, lane, c);
    chunk_deliver<Acc, WDT>(a, c, T, lane, s_b[wave], nullptr);
  }
}

// Residues of step t_base + t_off computed on the device (the persistent
// schedule's steps inside one launch).
__device__ __forceinline__ StepOff step_off_dev(const StepArgs& a, uint32_t t_off) {
  StepOff o;
  o.t_off = t_off;
  o.d_slot = t_off % (uint32_t)a.D;
  o.d_phase = t_off % (uint32_t)a.rate_bin_steps;
  o.d_bin = (t_off / (uint32_t)a.rate_bin_steps) % (uint32_t)a.rate_bins_cap;
  return o;
}

// Persistent schedule: n_steps steps in one cooperative launch of blocks
// that are all resident at once (G of them).  Each step: block b updates
// tiles b, b + G, ...; the grid synchronises; every block delivers (its
// wavefronts take delivery items over all 4 G wavefronts) and then routes
// the previous step's inboxes of tiles b, b + G, ...; the grid
// synchronises.  This is the split schedule's sequence of work, so the
// results are the same.
template <typename Acc, int WDT, int NP, int FMT>
__global__ void __launch_bounds__(256) k_persist(StepArgs a, StepOff o, uint32_t n_steps) {
  extern __shared__ __align__(16) int32_t s_dyn[];
  __shared__ int32_t s_spk[1024];
  __shared__ Acc s_in[1024];
  __shared__ int s_wt[4];
  __shared__ uint32_t s_base;
  __shared__ int32_t s_part[8];
  __shared__ uint32_t s_b[4][256];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int G = (int)gridDim.x;
  for (uint32_t k = 0; k < n_steps; ++k) {
    const StepTime T = step_time(a, step_off_dev(a, o.t_off + k));
    for (int tile = (int)blockIdx.x; tile < a.n_tiles; tile += G) {
      update_tile<Acc, NP, FMT>(a, T, tile, s_spk, s_in, s_wt, &s_base);
      lds_barrier();  // the tile's LDS is reused by the next one
    }
    grid.sync();
    deliver_spikes<Acc, WDT, false>(a, T, (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6),
                                    (int64_t)G * 4, blockIdx.x == 0, s_dyn, s_part, s_b);
    if (a.q_cap) {
      lds_barrier();  // the dynamic LDS holds the routing stage from here
      RouteLds<Acc>& L = *reinterpret_cast<RouteLds<Acc>*>(s_dyn);
      for (int tile = (int)blockIdx.x; tile < a.n_tiles; tile += G)
        route_inbox<Acc, WDT != DPSNN_W_F32>(a, tile, T, L);
    }
    grid.sync();
  }
}

// Advance the device step counter after `n` steps; on a switch from the
// split to the fused schedule, make both spike-log bases current.
__global__ void k_tick(uint32_t* t_base, uint32_t n, unsigned long long* log_base,
                       int sync_logs, uint32_t* spk_n, uint32_t D, uint32_t rbs, uint32_t cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const uint32_t t = t_base[0];
    if (sync_logs) log_base[(t + 1) & 1] = log_base[t & 1];
    const uint32_t t1 = t + n;
    // the counter and the residues the step kernels start from
    t_base[0] = t1;
    t_base[1] = t1 % D;
    t_base[2] = t1 % rbs;
    t_base[3] = (t1 / rbs) % cap;
  }
  // spike-list counters of the next step start from zero
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < 2 * kSpkLists; k += blockDim.x) spk_n[k * kSpkStride] = 0u;
}

// k_drain for one entry format (IE: inbox entries, CE: queue entries).
template <typename Acc, typename IE, typename CE>
__device__ __forceinline__ void drain_tile(const StepArgs& a, int tile, uint32_t t,
                                           const CodeDec<Acc>& dec) {
  const int D = a.D;
  Acc* slots = static_cast<Acc*>(a.slots);
  const uint32_t par = (t - 1u) & 1u;
  const int64_t ic = ((int64_t)par * a.n_tiles + tile) * kInboxStride;
  const uint32_t got = a.in_cnt[ic];
  const uint32_t n_in = got < (uint32_t)a.in_cap ? got : (uint32_t)a.in_cap;
  const IE* iq = static_cast<const IE*>(a.in_q) + ((int64_t)par * a.n_tiles + tile) * a.in_cap;
  for (uint32_t e = threadIdx.x; e < n_in; e += blockDim.x) {
    const uint32_t x = ent_x(iq[e]);
    const int dk = (int)(x >> 10) < a.n_del ? (int)(x >> 10) : a.n_del - 1;
    // emitted at t - 1, arrives at t - 1 + d_min + dk
    const int sl = (int)(((uint64_t)t + (uint64_t)(a.d_min + dk) - 1u) % (uint64_t)D);
    atomic_add_fix<Acc>(slots + (int64_t)sl * a.N_pad + (int64_t)tile * 1024 + (x & 1023u),
                        ent_w<Acc>(iq[e], dec));
  }
  const CE* qq = static_cast<const CE*>(a.q_q) + (int64_t)tile * D * a.q_cap;
  for (int k = 0; k < D; ++k) {
    const uint32_t qn = a.q_cnt[(int64_t)tile * D + k];
    const uint32_t n = qn < (uint32_t)a.q_cap ? qn : (uint32_t)a.q_cap;
    for (uint32_t e = threadIdx.x; e < n; e += blockDim.x) {
      const CE q = qq[(int64_t)k * a.q_cap + e];
      atomic_add_fix<Acc>(slots + (int64_t)k * a.N_pad + (int64_t)tile * 1024 + (ent_x(q) & 1023u),
                          ent_w<Acc>(q, dec));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) a.in_cnt[ic] = 0;
  for (int k = threadIdx.x; k < D; k += blockDim.x) {
    a.q_cnt[(int64_t)tile * D + k] = 0;
    a.s_dirty[(int64_t)tile * D + k] = 1u;
  }
}

// Pending queue entries of tile blockIdx.x after t steps added into the
// slots: the inbox of step t-1 and every per-slot queue; all left empty.
template <typename Acc>
__global__ void __launch_bounds__(256) k_drain(StepArgs a, uint32_t t) {
  const int tile = blockIdx.x;
  const CodeDec<Acc> dec = code_dec<Acc>(a, tile);
  if (a.q_code)
    drain_tile<Acc, CodeEntry, CodeEntry>(a, tile, t, dec);
  else if (sizeof(Acc) == 4 && a.q_packed)
    drain_tile<Acc, QEntry<Acc>, PackedEntry>(a, tile, t, dec);
  else
    drain_tile<Acc, QEntry<Acc>, QEntry<Acc>>(a, tile, t, dec);
}

// ------------------------------------------------------------------------
// The launch for step t_base + t_off: t_off and its residues.
static StepOff step_off(const StepArgs& a, uint32_t t_off) {
  StepOff o;
  o.t_off = t_off;
  o.d_slot = t_off % (uint32_t)a.D;
  o.d_phase = t_off % (uint32_t)a.rate_bin_steps;
  o.d_bin = (t_off / (uint32_t)a.rate_bin_steps) % (uint32_t)a.rate_bins_cap;
  return o;
}

hipError_t launch_gen(const GenArgs& a, int wdt, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  const int per_wave = gen_stage_bytes(a.K_out);
  int wpb = 60000 / per_wave;
  wpb = wpb < 1 ? 1 : (wpb > 4 ? 4 : wpb);
  const int64_t blocks = (a.N + wpb - 1) / wpb;
  const size_t lds = (size_t)wpb * per_wave;
  if (wdt == DPSNN_W_F32)
    hipLaunchKernelGGL(k_gen<DPSNN_W_F32>, dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a);
  else if (wdt == DPSNN_W_F16)
    hipLaunchKernelGGL(k_gen<DPSNN_W_F16>, dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a);
  else
    hipLaunchKernelGGL(k_gen<DPSNN_W_I8>, dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_absum_max(const unsigned long long* absum, int64_t n,
                            unsigned long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_absum_max, dim3(1024), dim3(256), 0, st, absum, n, out);
  return hipGetLastError();
}

hipError_t launch_init(const InitArgs& a, hipStream_t st) {
  const int64_t blocks = (a.N_pad + 255) / 256;
  hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Merged reservations in the delivery kernel: spike lists of kind 2 (the
// appended lists) with queues.
static bool merge_reserve(const StepArgs& a) { return a.q_cap && a.spk_lists == 2; }

// Dynamic LDS of the delivery kernel: the larger of the tile-count prefix
// (per-tile spike lists) and the routing blocks' RouteLds.
template <typename Acc>
static size_t deliver_lds(const StepArgs& a) {
  // (the merged reservations' hash only with appended spike lists, whose
  // blocks keep no tile-count prefix)
  const size_t pref =
      (size_t)stage_offset_words(a) * 4 + kStageBytes + (merge_reserve(a) ? kHashBytes : 0);
  const size_t route = a.route_blocks ? sizeof(RouteLds<Acc>) : 0;
  return pref > route ? pref : route;
}

template <typename Acc, int FMT>
static void launch_neuron_fmt(const StepArgs& a, uint32_t t_off, hipStream_t st) {
  const dim3 tiles((unsigned)a.n_tiles), block(256);
  if (a.P <= 2)
    hipLaunchKernelGGL((k_neuron<Acc, 2, FMT>), tiles, block, 0, st, a, step_off(a, t_off));
  else if (a.two_cls)
    hipLaunchKernelGGL((k_neuron<Acc, 3, FMT>), tiles, block, 0, st, a, step_off(a, t_off));
  else
    hipLaunchKernelGGL((k_neuron<Acc, 4, FMT>), tiles, block, 0, st, a, step_off(a, t_off));
}

template <typename Acc>
static void launch_neuron(const StepArgs& a, uint32_t t_off, hipStream_t st) {
  if (a.q_code) {
    launch_neuron_fmt<Acc, kFmtCode>(a, t_off, st);
    return;
  }
  if constexpr (sizeof(Acc) == 4) {
    if (a.q_packed) {
      launch_neuron_fmt<Acc, kFmtPacked>(a, t_off, st);
      return;
    }
  }
  launch_neuron_fmt<Acc, kFmtWide>(a, t_off, st);
}

template <typename Acc, bool MERGE>
static void launch_deliver(const StepArgs& a, int wdt, dim3 grid, size_t lds, uint32_t t_off,
                           hipStream_t st) {
  const dim3 block(256);
  if (a.plastic)
    hipLaunchKernelGGL((k_deliver<Acc, DPSNN_W_F32, true, MERGE>), grid, block, lds, st, a,
                       step_off(a, t_off));
  else if (wdt == DPSNN_W_F32)
    hipLaunchKernelGGL((k_deliver<Acc, DPSNN_W_F32, false, MERGE>), grid, block, lds, st, a,
                       step_off(a, t_off));
  else if (wdt == DPSNN_W_F16)
    hipLaunchKernelGGL((k_deliver<Acc, DPSNN_W_F16, false, MERGE>), grid, block, lds, st, a,
                       step_off(a, t_off));
  else
    hipLaunchKernelGGL((k_deliver<Acc, DPSNN_W_I8, false, MERGE>), grid, block, lds, st, a,
                       step_off(a, t_off));
}

template <typename Acc>
static void launch_split(const StepArgs& a, int wdt, uint32_t t_off, hipStream_t st) {
  launch_neuron<Acc>(a, t_off, st);
  const size_t lds = deliver_lds<Acc>(a);
  const dim3 grid((unsigned)(a.deliver_blocks + a.route_blocks));
  if (merge_reserve(a))
    launch_deliver<Acc, true>(a, wdt, grid, lds, t_off, st);
  else
    launch_deliver<Acc, false>(a, wdt, grid, lds, t_off, st);
}

template <typename Acc, int NP>
static void launch_fused_np(const StepArgs& a, int wdt, uint32_t t_off, hipStream_t st) {
  const dim3 tiles((unsigned)a.n_tiles), block(256);
  if (wdt == DPSNN_W_F32)
    hipLaunchKernelGGL((k_step<Acc, DPSNN_W_F32, NP>), tiles, block, 0, st, a, step_off(a, t_off));
  else if (wdt == DPSNN_W_F16)
    hipLaunchKernelGGL((k_step<Acc, DPSNN_W_F16, NP>), tiles, block, 0, st, a, step_off(a, t_off));
  else
    hipLaunchKernelGGL((k_step<Acc, DPSNN_W_I8, NP>), tiles, block, 0, st, a, step_off(a, t_off));
}

template <typename Acc>
static void launch_fused(const StepArgs& a, int wdt, uint32_t t_off, hipStream_t st) {
  if (a.P <= 2)
    launch_fused_np<Acc, 2>(a, wdt, t_off, st);
  else
    launch_fused_np<Acc, 4>(a, wdt, t_off, st);
}

template <typename Acc, int WDT, int NP, int FMT>
static hipError_t launch_persist_t(const StepArgs& a, uint32_t t_off, uint32_t n,
                                   hipStream_t st) {
  const void* fn = reinterpret_cast<const void*>(&k_persist<Acc, WDT, NP, FMT>);
  const size_t pref = (size_t)stage_offset_words(a) * 4 + kStageBytes;
  const size_t route = a.q_cap ? sizeof(RouteLds<Acc>) : 0;
  const size_t lds = pref > route ? pref : route;
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, &k_persist<Acc, WDT, NP, FMT>, 256, lds);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (per_cu < 1 || cus < 1) return hipErrorLaunchFailure;
  StepArgs aa = a;
  StepOff o = step_off(a, t_off);
  uint32_t nn = n;
  void* args[] = {&aa, &o, &nn};
  return hipLaunchCooperativeKernel(fn, dim3((unsigned)(per_cu * cus)), dim3(256), args,
                                    (unsigned)lds, st);
}

template <typename Acc, int NP>
static hipError_t launch_persist_np(const StepArgs& a, int wdt, uint32_t t_off, uint32_t n,
                                    hipStream_t st) {
  if (wdt == DPSNN_W_F16) return launch_persist_t<Acc, DPSNN_W_F16, NP, kFmtCode>(a, t_off, n, st);
  if (wdt == DPSNN_W_I8) return launch_persist_t<Acc, DPSNN_W_I8, NP, kFmtCode>(a, t_off, n, st);
  if constexpr (sizeof(Acc) == 4)
    if (a.q_packed) return launch_persist_t<Acc, DPSNN_W_F32, NP, kFmtPacked>(a, t_off, n, st);
  return launch_persist_t<Acc, DPSNN_W_F32, NP, kFmtWide>(a, t_off, n, st);
}

hipError_t launch_persist(const StepArgs& a, int wdt, int acc_bits, uint32_t t_off, uint32_t n,
                          hipStream_t st) {
  if (acc_bits == 32)
    return a.P <= 2 ? launch_persist_np<int32_t, 2>(a, wdt, t_off, n, st)
                    : launch_persist_np<int32_t, 4>(a, wdt, t_off, n, st);
  return a.P <= 2 ? launch_persist_np<int64_t, 2>(a, wdt, t_off, n, st)
                  : launch_persist_np<int64_t, 4>(a, wdt, t_off, n, st);
}

hipError_t launch_step(const StepArgs& a, int wdt, int acc_bits, int sched, uint32_t t_off,
                       hipStream_t st) {
  if (sched == DPSNN_SCHED_PERSIST) return launch_persist(a, wdt, acc_bits, t_off, 1, st);
  if (sched == DPSNN_SCHED_SPLIT) {
    if (acc_bits == 32)
      launch_split<int32_t>(a, wdt, t_off, st);
    else
      launch_split<int64_t>(a, wdt, t_off, st);
  } else {
    if (acc_bits == 32)
      launch_fused<int32_t>(a, wdt, t_off, st);
    else
      launch_fused<int64_t>(a, wdt, t_off, st);
  }
  return hipGetLastError();
}

// One phase of the split schedule on its own (0 = neuron update, 1 = delivery).
hipError_t launch_phase(const StepArgs& a, int wdt, int acc_bits, int phase, uint32_t t_off,
                        hipStream_t st) {
  const dim3 grid((unsigned)(a.deliver_blocks + a.route_blocks));
  const size_t lds = acc_bits == 32 ? deliver_lds<int32_t>(a) : deliver_lds<int64_t>(a);
  if (phase == 0) {
    if (acc_bits == 32)
      launch_neuron<int32_t>(a, t_off, st);
    else
      launch_neuron<int64_t>(a, t_off, st);
  } else {
    // the delivery launch of the split schedule, as launch_split makes it
    const bool m = merge_reserve(a);
    if (acc_bits == 32) {
      if (m)
        launch_deliver<int32_t, true>(a, wdt, grid, lds, t_off, st);
      else
        launch_deliver<int32_t, false>(a, wdt, grid, lds, t_off, st);
    } else {
      if (m)
        launch_deliver<int64_t, true>(a, wdt, grid, lds, t_off, st);
      else
        launch_deliver<int64_t, false>(a, wdt, grid, lds, t_off, st);
    }
  }
  return hipGetLastError();
}

size_t deliver_lds_bytes(const StepArgs& a, int acc_bits) {
  // dynamic part, plus the wavefront scratch s_b and s_part
  return (acc_bits == 32 ? deliver_lds<int32_t>(a) : deliver_lds<int64_t>(a)) +
         sizeof(uint32_t) * 4 * 256 + sizeof(int32_t) * 8;
}

hipError_t launch_drain(const StepArgs& a, int acc_bits, uint32_t t, hipStream_t st) {
  if (a.q_cap == 0 || a.n_tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)a.n_tiles);
  if (acc_bits == 32)
    hipLaunchKernelGGL(k_drain<int32_t>, grid, dim3(256), 0, st, a, t);
  else
    hipLaunchKernelGGL(k_drain<int64_t>, grid, dim3(256), 0, st, a, t);
  return hipGetLastError();
}

// Periodic efficacy update of every plastic synapse after T steps (Sec. 2.1:
// the synapses apply their integrated plasticity signal once per period):
// w = clip(w + eta (y Dy(T - t_act)), 0, w_max), y = 0.
__global__ void __launch_bounds__(256) k_stdp_update(StepArgs a, int32_t T) {
  const int64_t total = a.N_pad * a.row_stride;
  const int32_t L = a.stdp_L;
  const float* Dy = a.stdp_tab + 2 * L;
  float* w = static_cast<float*>(const_cast<void*>(a.w));  // plastic efficacies
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = x / a.row_stride;
    const int j = (int)(x - s * a.row_stride);
    if (j >= a.K_out) continue;
    const NetDev& nd = a.nets[a.tile_net[s >> 10]];
    const int64_t il = s - nd.base;
    if (il >= nd.N) continue;  // padding
    const int l = (int)((uint32_t)il - module_of(nd, (uint32_t)il) * (uint32_t)nd.K);
    const int q = (l >= nd.pop_hi[0]) + (l >= nd.pop_hi[1]) + (l >= nd.pop_hi[2]);
    if (!nd.exc[q]) continue;
    const int32_t tl = a.syn_t[x];
    if (tl >= 0 && T - tl < L) {
      float v = w[x] + a.stdp_eta * (a.syn_y[x] * Dy[T - tl]);
      v = v < 0.0f ? 0.0f : (v > a.stdp_wmax ? a.stdp_wmax : v);
      w[x] = v;
    }
    a.syn_y[x] = 0.0f;
  }
}

hipError_t launch_stdp_update(const StepArgs& a, int32_t T, hipStream_t st) {
  const int64_t total = a.N_pad * a.row_stride;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_stdp_update, dim3((unsigned)blocks), dim3(256), 0, st, a, T);
  return hipGetLastError();
}

hipError_t launch_tick(const StepArgs& a, uint32_t n, int sync_logs, hipStream_t st) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, a.t_base, n, a.log_base, sync_logs,
                     a.spk_n, (uint32_t)a.D, (uint32_t)a.rate_bin_steps,
                     (uint32_t)a.rate_bins_cap);
  return hipGetLastError();
}

}  // namespace dpsnn
