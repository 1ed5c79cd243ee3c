// HIP kernels of libdpsnn for gfx950 (64-lane wavefronts).
//
//  k_gen      one wavefront per source row: draws the K_out synapses of the
//             source from Philox (Eq. 1 targets, uniform delay, quantile-table
//             efficacy), ranks them stably by delay with wavefront ballots and
//             writes the delay-sorted row plus its delay offsets.  The delay
//             index also rides in the top 6 bits of each target word, so that
//             delivery needs no lookup.
//  k_init     initial membrane potentials, fatigue and refractory counters.
//  k_neuron   one step of dt for a tile of 1024 neurons (4 per thread):
//             input slot read-and-clear, external Poisson drive, Eq. 2 update,
//             threshold; the tile's spikes go to its own segment of the spike
//             list (no global counter).
//  k_deliver  the tile counts are scanned in LDS by every block; then every
//             wavefront of the grid takes chunks of 256 synapses of spiking
//             rows (16-byte loads) and adds the fixed-point efficacies into the
//             target slots with atomics.  Spreading the chunks over the whole
//             chip keeps every CU issuing atomics.  Also appends the spike log
//             and the 5 ms population counts.
//  k_step     fused schedule for small networks: k_neuron followed by the
//             delivery of the tile's own spikes by its four wavefronts.
//
// A step reads only slot t mod D and delivery writes only slots t+d_min ..
// t+d_max, so update and delivery of one step need no grid-wide ordering;
// the kernel boundary orders consecutive steps.  The step index is read on
// the device (t = *t_base + t_off) so that launches can be captured in a graph.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "dpsnn_internal.h"
#include "philox.h"

namespace dpsnn {

// ------------------------------------------------------------------------
// Connectivity generation
__host__ __device__ inline int gen_stage_bytes(int Ko) {
  // tgt (4) + efficacy index (2) + rank (2) + delay index (1) per synapse
  return ((9 * Ko + 15) / 16) * 16 + 64 * 4;
}

template <int WDT>
__global__ void __launch_bounds__(256) k_gen(GenArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int64_t s = (int64_t)blockIdx.x * wpb + wave;
  const bool active = s < a.N;
  const int Ko = a.K_out;

  unsigned char* base = smem + (size_t)wave * gen_stage_bytes(Ko);
  int32_t* st_tgt = reinterpret_cast<int32_t*>(base);
  uint16_t* st_w = reinterpret_cast<uint16_t*>(st_tgt + Ko);
  uint16_t* st_rank = st_w + Ko;
  uint8_t* st_del = reinterpret_cast<uint8_t*>(st_rank + Ko);
  uint32_t* st_off = reinterpret_cast<uint32_t*>(base + ((9 * Ko + 15) / 16) * 16);

  const int32_t ls = active ? (int32_t)(s % a.K) : 0;
  const int32_t ms = active ? (int32_t)(s / a.K) : 0;
  const int pop = ls < a.K_exc ? 0 : 1;
  const int xs = ms % a.W, ys = ms / a.W;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;

  uint32_t cnt = 0;  // lane x: synapses with delay index x seen so far
  if (active) {
    for (int j0 = 0; j0 < Ko; j0 += 64) {
      const int j = j0 + lane;
      int k = -1;
      int32_t tg = 0;
      uint16_t wi = 0;
      if (j < Ko) {
        const uint4 u = philox10(make_uint4((uint32_t)s, (uint32_t)j, 0u, kTagSyn),
                                 a.key0, a.key1);
        if (j < a.n_local[pop]) {
          const uint32_t r = scale32(u.x, (uint32_t)(a.K - 1));
          tg = ms * a.K + (int32_t)(r + (r >= (uint32_t)ls ? 1u : 0u));
        } else {
          int lo = 0, hi = a.n_off - 1;  // first threshold above u.x
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a.off_thr[mid] <= u.x)
              lo = mid + 1;
            else
              hi = mid;
          }
          int xt = xs + a.off_xy[2 * lo];
          int yt = ys + a.off_xy[2 * lo + 1];
          if (xt >= a.W) xt -= a.W;
          if (yt >= a.H) yt -= a.H;
          tg = (yt * a.W + xt) * a.K + (int32_t)scale32(u.y, (uint32_t)a.K);
        }
        k = (int)scale32(u.z, (uint32_t)a.n_del);
        wi = (uint16_t)(u.w >> 16);
      }
      // stable rank among equal delays: earlier chunks, then lower lanes
      const uint32_t before = cnt;
      uint32_t in_chunk = 0;
      for (int x = 0; x < a.n_del; ++x) {
        const uint64_t m = __ballot(k == x);
        if (lane == x) cnt += (uint32_t)__popcll(m);
        if (k == x) in_chunk = (uint32_t)__popcll(m & below);
      }
      const uint32_t prev = __shfl(before, k < 0 ? 0 : k);
      if (j < Ko) {
        st_tgt[j] = tg;
        st_w[j] = wi;
        st_del[j] = (uint8_t)k;
        st_rank[j] = (uint16_t)(prev + in_chunk);
      }
    }
    // exclusive scan of the per-delay counts across lanes
    uint32_t incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t v = __shfl_up(incl, off);
      if (lane >= off) incl += v;
    }
    const uint32_t excl = incl - cnt;
    if (lane < a.n_del) {
      st_off[lane] = excl;
      a.doff[s * a.doff_stride + lane] = (uint16_t)excl;
    }
    if (lane == 0) a.doff[s * a.doff_stride + a.n_del] = (uint16_t)Ko;
    for (int x = a.n_del + 1 + lane; x < a.doff_stride; x += 64)
      a.doff[s * a.doff_stride + x] = 0;
  }
  __syncthreads();
  if (!active) return;
  const int64_t rb = s * a.row_stride;
  for (int j = lane; j < Ko; j += 64) {
    const int k = st_del[j];
    const uint32_t pos = st_off[k] + st_rank[j];
    if (pos >= (uint32_t)Ko) continue;  // unreachable: ranks stay inside the row
    const int64_t o = rb + pos;
    const int32_t tg = st_tgt[j];
    const uint16_t wi = st_w[j];
    const int32_t gt = tg + (int32_t)a.tgt_base;  // global target index
    a.tgt[o] = gt | (k << kDelayShift);
    if (WDT == DPSNN_W_F32)
      static_cast<float*>(a.w)[o] = static_cast<const float*>(a.wtab[pop])[wi];
    else if (WDT == DPSNN_W_F16)
      static_cast<uint16_t*>(a.w)[o] = static_cast<const uint16_t*>(a.wtab[pop])[wi];
    else
      static_cast<int8_t*>(a.w)[o] = static_cast<const int8_t*>(a.wtab[pop])[wi];
    if (a.absum) {
      const int64_t f = a.wfix_tab[pop][wi];
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
    const int q = (int)(i % a.K) < a.K_exc ? 0 : 1;
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

template <typename Acc, int WDT>
__device__ __forceinline__ Acc stored_to_fix(const void* w, int64_t o, float two_q,
                                             int64_t scale) {
  if (WDT == DPSNN_W_F32) {
    return (Acc)__builtin_rintf(static_cast<const float*>(w)[o] * two_q);
  } else if (WDT == DPSNN_W_F16) {
    const __half h = static_cast<const __half*>(w)[o];
    return (Acc)__builtin_rintf(__half2float(h) * two_q);
  } else {
    return (Acc)static_cast<const int8_t*>(w)[o] * (Acc)scale;
  }
}

// ------------------------------------------------------------------------
// Neuron update of the 4 neurons i0..i0+3 (global indices) of one thread at
// step t; nd is the tile's network.  Spiking neurons are appended to the LDS
// list s_spk (count s_n).  Counters of the random draws use the network's
// own neuron indices, so a network in a batch draws what it draws alone.
template <typename Acc>
__device__ __forceinline__ void update4(const StepArgs& a, const NetDev& nd, int64_t i0,
                                        uint32_t t, int32_t* s_spk, int* s_n) {
  const int slot = (int)(t % (uint32_t)a.D);
  Acc* sl = static_cast<Acc*>(a.slots) + (int64_t)slot * a.N_pad + i0;
  Acc I[4];
  if (sizeof(Acc) == 4) {
    const int4 v = *reinterpret_cast<const int4*>(sl);
    I[0] = v.x; I[1] = v.y; I[2] = v.z; I[3] = v.w;
    *reinterpret_cast<int4*>(sl) = make_int4(0, 0, 0, 0);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      I[j] = sl[j];
      sl[j] = 0;
    }
  }
  const float4 V4 = *reinterpret_cast<const float4*>(a.V + i0);
  const float4 c4 = *reinterpret_cast<const float4*>(a.c + i0);
  const uint32_t r4 = *reinterpret_cast<const uint32_t*>(a.ref + i0);
  float Vv[4] = {V4.x, V4.y, V4.z, V4.w};
  float cv[4] = {c4.x, c4.y, c4.z, c4.w};

  // external Poisson drive generated on the fly: counts from word j of
  // (il0/4, t, EXT); efficacies 2b and 2b+1 of neuron j from word j of
  // (il0/4, t, EXTJ | b << 8), high half then low half
  const int64_t il0 = i0 - nd.base;  // network-local index, a multiple of 4
  const uint32_t g = (uint32_t)(il0 >> 2);
  const uint4 u = philox10(make_uint4(g, t, 0u, kTagExt), nd.key0, nd.key1);
  const uint32_t uu[4] = {u.x, u.y, u.z, u.w};
  const int64_t m0 = il0 / nd.K;
  const int l0 = (int)(il0 - m0 * nd.K);
  int q[4], k[4];
  int kmax = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int lj = l0 + j;
    if (lj >= nd.K) lj -= nd.K;
    q[j] = lj < nd.K_exc ? 0 : 1;
    int kk = 0;
    for (int x = 0; x < nd.n_pois[q[j]]; ++x) kk += uu[j] >= nd.pois[q[j]][x] ? 1 : 0;
    k[j] = kk;
    kmax = kk > kmax ? kk : kmax;
  }
  const Acc* jx = static_cast<const Acc*>(nd.jxfix);
  for (int b = 0; 2 * b < kmax; ++b) {
    const uint4 v = philox10(make_uint4(g, t, 0u, kTagExtJ | ((uint32_t)b << 8)), nd.key0, nd.key1);
    const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (2 * b < k[j]) I[j] += jx[q[j] * kQuantN + (vv[j] >> 16)];
      if (2 * b + 1 < k[j]) I[j] += jx[q[j] * kQuantN + (vv[j] & 0xFFFFu)];
    }
  }

  uint32_t r_out = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int qq = q[j];
    uint32_t rj = (r4 >> (8 * j)) & 0xFFu;
    if (il0 + j < nd.N) {
      const float dv = fix_to_f32(I[j]) * a.inv2q;
      float Vj = Vv[j], cj = cv[j];
      bool spk = false;
      if (rj > 0) {
        rj -= 1;
        cj = cj * nd.Pc[qq];
      } else {
        float vv = Vj - nd.E[qq];
        vv = vv * nd.Pm[qq];
        vv = nd.E[qq] + vv;
        const float cc = cj * nd.PVc[qq];
        vv = vv - cc;
        vv = vv + nd.Iterm[qq];
        vv = vv + dv;
        cj = cj * nd.Pc[qq];
        if (vv > nd.Vth[qq]) {
          spk = true;
          vv = nd.Vr[qq];
          cj = cj + nd.alpha[qq];
          rj = (uint32_t)nd.n_arp[qq];
        }
        Vj = vv;
      }
      Vv[j] = Vj;
      cv[j] = cj;
      if (spk) {
        const int pos = atomicAdd(s_n, 1);
        s_spk[pos] = (int32_t)(i0 + j);
      }
    }
    r_out |= rj << (8 * j);
  }
  *reinterpret_cast<float4*>(a.V + i0) = make_float4(Vv[0], Vv[1], Vv[2], Vv[3]);
  *reinterpret_cast<float4*>(a.c + i0) = make_float4(cv[0], cv[1], cv[2], cv[3]);
  *reinterpret_cast<uint32_t*>(a.ref + i0) = r_out;
}

// Global module and population of a (global) neuron id.
__device__ __forceinline__ void module_pop(const StepArgs& a, int32_t id, int32_t* mod,
                                           int* pop) {
  const NetDev& nd = a.nets[a.tile_net[id >> 10]];
  const int32_t local = id - (int32_t)nd.base;
  const int32_t m = local / nd.K;
  *mod = nd.mbase + m;
  *pop = (local - m * nd.K) < nd.K_exc ? 0 : 1;
}

// 256 synapses (4 per lane) of row s starting at p0 = chunk * 256.
template <typename Acc, int WDT>
__device__ __forceinline__ void deliver_chunk(const StepArgs& a, int32_t s, int p0,
                                              uint32_t t, int lane) {
  const int64_t rb = (int64_t)s * a.row_stride;
  int64_t scale = 0;
  if (WDT == DPSNN_W_I8) {
    int32_t ms;
    int q;
    module_pop(a, s, &ms, &q);
    scale = a.sfix[2 * ms + q];
  }
  const int p = p0 + lane * 4;
  if (p >= a.K_out) return;
  const int4 tg = *reinterpret_cast<const int4*>(a.tgt + rb + p);
  const int tv[4] = {tg.x, tg.y, tg.z, tg.w};
  Acc wv[4];
  if (WDT == DPSNN_W_F32) {
    const float4 w4 = *reinterpret_cast<const float4*>(static_cast<const float*>(a.w) + rb + p);
    wv[0] = (Acc)__builtin_rintf(w4.x * a.two_q);
    wv[1] = (Acc)__builtin_rintf(w4.y * a.two_q);
    wv[2] = (Acc)__builtin_rintf(w4.z * a.two_q);
    wv[3] = (Acc)__builtin_rintf(w4.w * a.two_q);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) wv[j] = stored_to_fix<Acc, WDT>(a.w, rb + p + j, a.two_q, scale);
  }
  const int slot0 = (int)((t + (uint32_t)a.d_min) % (uint32_t)a.D);
  Acc* slots = static_cast<Acc*>(a.slots);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (p + j < a.K_out) {
      int sl = slot0 + (int)((uint32_t)tv[j] >> kDelayShift);
      if (sl >= a.D) sl -= a.D;
      const int32_t target = tv[j] & kTargetMask;
      atomic_add_fix<Acc>(slots + (int64_t)sl * a.N_pad + target, wv[j]);
    }
  }
}

__device__ __forceinline__ void record_spike(const StepArgs& a, int32_t id, uint32_t t,
                                             unsigned long long pos) {
  if (pos < (unsigned long long)a.spike_log_cap) a.log[pos] = make_int2((int)t, id);
  const uint32_t bin = (t / (uint32_t)a.rate_bin_steps) % (uint32_t)a.rate_bins_cap;
  int32_t mod;
  int q;
  module_pop(a, id, &mod, &q);
  atomicAdd(&a.rates[((int64_t)bin * a.M + mod) * 2 + q], 1u);
}

// ------------------------------------------------------------------------
// Split schedule: neuron kernel, then the delivery kernel.
template <typename Acc>
__global__ void __launch_bounds__(256) k_neuron(StepArgs a, uint32_t t_off) {
  __shared__ int32_t s_spk[1024];
  __shared__ int s_n;
  const int tid = threadIdx.x;
  if (tid == 0) s_n = 0;
  __syncthreads();
  const uint32_t t = a.t_base[0] + t_off;
  const int64_t i0 = ((int64_t)blockIdx.x * 256 + tid) * 4;
  const NetDev& nd = a.nets[a.tile_net[blockIdx.x]];
  update4<Acc>(a, nd, i0, t, s_spk, &s_n);
  __syncthreads();
  const int n = s_n;
  int32_t* out = a.spk + (int64_t)blockIdx.x * 1024;
  for (int k = tid; k < n; k += 256) out[k] = s_spk[k];
  if (tid == 0) a.blk_cnt[blockIdx.x] = n;
}

template <typename Acc, int WDT>
__global__ void __launch_bounds__(256) k_deliver(StepArgs a, uint32_t t_off) {
  extern __shared__ int32_t s_pref[];  // inclusive prefix of the tile counts
  __shared__ int32_t s_part[256];
  const int tid = threadIdx.x;
  const int nb = a.n_tiles;
  const uint32_t t = a.t_base[0] + t_off;
  // block-wide scan: each thread sums a contiguous run of tile counts
  const int per = (nb + 255) / 256;
  const int lo = tid * per;
  const int hi = lo + per < nb ? lo + per : nb;
  int run = 0;
  for (int b = lo; b < hi; ++b) run += a.blk_cnt[b];
  s_part[tid] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int v = tid >= off ? s_part[tid - off] : 0;
    __syncthreads();
    s_part[tid] += v;
    __syncthreads();
  }
  int acc = s_part[tid] - run;
  for (int b = lo; b < hi; ++b) {
    acc += a.blk_cnt[b];
    s_pref[b] = acc;
  }
  __syncthreads();
  const int n_spk = s_part[255];
  const unsigned long long log0 = a.log_base[t & 1];
  if (blockIdx.x == 0 && tid == 0) {
    a.log_base[(t + 1) & 1] = log0 + (unsigned long long)n_spk;
    a.n_spikes[0] += (unsigned long long)n_spk;
  }
  const int cpr = (a.K_out + 255) / 256;  // chunks per row
  const int64_t items = (int64_t)n_spk * cpr;
  const int lane = tid & 63;
  const int64_t wid = (int64_t)blockIdx.x * 4 + (tid >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t it = wid; it < items; it += nw) {
    const int sidx = (int)(it / cpr);
    const int chunk = (int)(it - (int64_t)sidx * cpr);
    // tile holding spike number sidx: first b with s_pref[b] > sidx
    int l = 0, h = nb - 1;
    while (l < h) {
      const int mid = (l + h) >> 1;
      if (s_pref[mid] > sidx)
        h = mid;
      else
        l = mid + 1;
    }
    const int first = l ? s_pref[l - 1] : 0;
    const int32_t s = __builtin_amdgcn_readfirstlane(a.spk[(int64_t)l * 1024 + (sidx - first)]);
    if (chunk == 0 && lane == 0) record_spike(a, s, t, log0 + (unsigned long long)sidx);
    deliver_chunk<Acc, WDT>(a, s, chunk * 256, t, lane);
  }
}

// Fused schedule (small networks): the tile's own spikes are delivered by
// its four wavefronts right after the update.
template <typename Acc, int WDT>
__global__ void __launch_bounds__(256) k_step(StepArgs a, uint32_t t_off) {
  __shared__ int32_t s_spk[1024];
  __shared__ int s_n;
  __shared__ unsigned long long s_logbase;
  const int tid = threadIdx.x;
  if (tid == 0) s_n = 0;
  __syncthreads();
  const uint32_t t = a.t_base[0] + t_off;
  const int64_t i0 = ((int64_t)blockIdx.x * 256 + tid) * 4;
  const NetDev& nd = a.nets[a.tile_net[blockIdx.x]];
  update4<Acc>(a, nd, i0, t, s_spk, &s_n);
  __syncthreads();
  const int n = s_n;
  if (n == 0) return;
  if (tid == 0) {
    // both log bases advance together in this schedule
    s_logbase = atomicAdd(&a.log_base[t & 1], (unsigned long long)n);
    atomicAdd(&a.log_base[(t + 1) & 1], (unsigned long long)n);
    atomicAdd(a.n_spikes, (unsigned long long)n);
  }
  __syncthreads();
  for (int k = tid; k < n; k += 256)
    record_spike(a, s_spk[k], t, s_logbase + (unsigned long long)k);
  const int lane = tid & 63, wave = tid >> 6;
  const int cpr = (a.K_out + 255) / 256;
  for (int it = wave; it < n * cpr; it += 4) {
    const int k = it / cpr;
    const int32_t s = __builtin_amdgcn_readfirstlane(s_spk[k]);
    deliver_chunk<Acc, WDT>(a, s, (it - k * cpr) * 256, t, lane);
  }
}

// Advance the device step counter after `n` steps; on a switch from the
// split to the fused schedule, make both spike-log bases current.
__global__ void k_tick(uint32_t* t_base, uint32_t n, unsigned long long* log_base,
                       int sync_logs) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const uint32_t t = t_base[0];
    if (sync_logs) log_base[(t + 1) & 1] = log_base[t & 1];
    t_base[0] = t + n;
  }
}

// ------------------------------------------------------------------------
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

template <typename Acc>
static void launch_split(const StepArgs& a, int wdt, uint32_t t_off, hipStream_t st) {
  const dim3 tiles((unsigned)a.n_tiles), block(256);
  hipLaunchKernelGGL(k_neuron<Acc>, tiles, block, 0, st, a, t_off);
  const size_t lds = (size_t)a.n_tiles * 4;
  const dim3 grid((unsigned)a.deliver_blocks);
  if (wdt == DPSNN_W_F32)
    hipLaunchKernelGGL((k_deliver<Acc, DPSNN_W_F32>), grid, block, lds, st, a, t_off);
  else if (wdt == DPSNN_W_F16)
    hipLaunchKernelGGL((k_deliver<Acc, DPSNN_W_F16>), grid, block, lds, st, a, t_off);
  else
    hipLaunchKernelGGL((k_deliver<Acc, DPSNN_W_I8>), grid, block, lds, st, a, t_off);
}

template <typename Acc>
static void launch_fused(const StepArgs& a, int wdt, uint32_t t_off, hipStream_t st) {
  const dim3 tiles((unsigned)a.n_tiles), block(256);
  if (wdt == DPSNN_W_F32)
    hipLaunchKernelGGL((k_step<Acc, DPSNN_W_F32>), tiles, block, 0, st, a, t_off);
  else if (wdt == DPSNN_W_F16)
    hipLaunchKernelGGL((k_step<Acc, DPSNN_W_F16>), tiles, block, 0, st, a, t_off);
  else
    hipLaunchKernelGGL((k_step<Acc, DPSNN_W_I8>), tiles, block, 0, st, a, t_off);
}

hipError_t launch_step(const StepArgs& a, int wdt, int acc_bits, int sched, uint32_t t_off,
                       hipStream_t st) {
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
  const dim3 tiles((unsigned)a.n_tiles), block(256);
  const dim3 grid((unsigned)a.deliver_blocks);
  const size_t lds = (size_t)a.n_tiles * 4;
  if (phase == 0) {
    if (acc_bits == 32)
      hipLaunchKernelGGL(k_neuron<int32_t>, tiles, block, 0, st, a, t_off);
    else
      hipLaunchKernelGGL(k_neuron<int64_t>, tiles, block, 0, st, a, t_off);
  } else if (acc_bits == 32) {
    if (wdt == DPSNN_W_F32)
      hipLaunchKernelGGL((k_deliver<int32_t, DPSNN_W_F32>), grid, block, lds, st, a, t_off);
    else if (wdt == DPSNN_W_F16)
      hipLaunchKernelGGL((k_deliver<int32_t, DPSNN_W_F16>), grid, block, lds, st, a, t_off);
    else
      hipLaunchKernelGGL((k_deliver<int32_t, DPSNN_W_I8>), grid, block, lds, st, a, t_off);
  } else {
    if (wdt == DPSNN_W_F32)
      hipLaunchKernelGGL((k_deliver<int64_t, DPSNN_W_F32>), grid, block, lds, st, a, t_off);
    else if (wdt == DPSNN_W_F16)
      hipLaunchKernelGGL((k_deliver<int64_t, DPSNN_W_F16>), grid, block, lds, st, a, t_off);
    else
      hipLaunchKernelGGL((k_deliver<int64_t, DPSNN_W_I8>), grid, block, lds, st, a, t_off);
  }
  return hipGetLastError();
}

hipError_t launch_tick(const StepArgs& a, uint32_t n, int sync_logs, hipStream_t st) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, a.t_base, n, a.log_base, sync_logs);
  return hipGetLastError();
}

}  // namespace dpsnn
