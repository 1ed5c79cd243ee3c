// HIP kernels of libdpsnn for gfx950 (64-lane wavefronts).
//
//  k_gen   one wavefront per source row: draws the K_out synapses of the
//          source from Philox (Eq. 1 targets, uniform delay, quantile-table
//          efficacy), ranks them stably by delay with wavefront ballots and
//          writes the delay-sorted row plus its delay offsets.
//  k_init  initial membrane potentials, fatigue and refractory counters.
//  k_step  one step of dt for a tile of 1024 neurons (4 per thread): input
//          slot read-and-clear, external Poisson drive, Eq. 2 update,
//          threshold, spike compaction in LDS, then the tile's own spikes are
//          delivered by its four wavefronts, each walking a whole row with
//          16-byte loads and fixed-point atomics into the target slots.
//          The step reads only slot t mod D and delivery writes only slots
//          t+d_min .. t+d_max, so the two phases need no grid-wide sync
//          inside a step; the kernel boundary orders consecutive steps.
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
    a.tgt[o] = tg;
    if (WDT == DPSNN_W_F32)
      static_cast<float*>(a.w)[o] = static_cast<const float*>(a.wtab[pop])[wi];
    else if (WDT == DPSNN_W_F16)
      static_cast<uint16_t*>(a.w)[o] = static_cast<const uint16_t*>(a.wtab[pop])[wi];
    else
      static_cast<int8_t*>(a.w)[o] = static_cast<const int8_t*>(a.wtab[pop])[wi];
    if (a.absum) {
      const int64_t f = a.wfix_tab[pop][wi];
      atomicAdd(&a.absum[tg], (unsigned long long)(f < 0 ? -f : f));
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
// One step.

// Fixed-point input sum in mV: one rounding of I * 2^-Q to binary32 (an
// int64 sum below 2^53 converts to binary64 exactly first).
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

template <typename Acc, int WDT>
__device__ __forceinline__ void deliver_row(const StepArgs& a, int32_t s, uint32_t t,
                                            int lane) {
  const int64_t rb = (int64_t)s * a.row_stride;
  const int32_t* trow = a.tgt + rb;
  const uint16_t* drow = a.doff + (int64_t)s * a.doff_stride;
  int64_t scale = 0;
  if (WDT == DPSNN_W_I8) {
    const int32_t ms = s / a.K;
    const int q = (s - ms * a.K) < a.K_exc ? 0 : 1;
    scale = a.sfix[2 * ms + q];
  }
  const int slot0 = (int)((t + (uint32_t)a.d_min) % (uint32_t)a.D);
  Acc* slots = static_cast<Acc*>(a.slots);
  for (int p0 = lane * 4; p0 < a.K_out; p0 += 256) {
    const int4 tg = *reinterpret_cast<const int4*>(trow + p0);
    const int tv[4] = {tg.x, tg.y, tg.z, tg.w};
    int kd[4] = {0, 0, 0, 0};
    for (int x = 1; x < a.n_del; ++x) {
      const int b = drow[x];
#pragma unroll
      for (int q = 0; q < 4; ++q) kd[q] += (p0 + q >= b) ? 1 : 0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (p0 + q < a.K_out) {
        int sl = slot0 + kd[q];
        if (sl >= a.D) sl -= a.D;
        const Acc v = stored_to_fix<Acc, WDT>(a.w, rb + p0 + q, a.two_q, scale);
        atomic_add_fix<Acc>(slots + (int64_t)sl * a.N_pad + tv[q], v);
      }
    }
  }
}

template <typename Acc, int WDT>
__global__ void __launch_bounds__(256) k_step(StepArgs a, uint32_t t) {
  __shared__ int32_t s_spk[1024];
  __shared__ int s_n;
  __shared__ unsigned long long s_logbase;
  const int tid = threadIdx.x;
  if (tid == 0) s_n = 0;
  __syncthreads();

  const int64_t i0 = ((int64_t)blockIdx.x * 256 + tid) * 4;
  const int slot = (int)(t % (uint32_t)a.D);
  if (i0 < a.N) {
    Acc* sl = static_cast<Acc*>(a.slots) + (int64_t)slot * a.N_pad + i0;
    Acc I[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      I[j] = sl[j];
      sl[j] = 0;
    }
    float4 V4 = *reinterpret_cast<const float4*>(a.V + i0);
    float4 c4 = *reinterpret_cast<const float4*>(a.c + i0);
    uint32_t r4 = *reinterpret_cast<const uint32_t*>(a.ref + i0);
    float Vv[4] = {V4.x, V4.y, V4.z, V4.w};
    float cv[4] = {c4.x, c4.y, c4.z, c4.w};
    const uint4 u = philox10(make_uint4((uint32_t)(i0 >> 2), t, 0u, kTagExt), a.key0, a.key1);
    const uint32_t uu[4] = {u.x, u.y, u.z, u.w};
    const int64_t m0 = i0 / a.K;
    const int l0 = (int)(i0 - m0 * a.K);
    uint32_t r_out = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = i0 + j;
      int lj = l0 + j;
      if (lj >= a.K) lj -= a.K;
      const int q = lj < a.K_exc ? 0 : 1;
      uint32_t rj = (r4 >> (8 * j)) & 0xFFu;
      if (i < a.N) {
        // external Poisson drive generated on the fly
        int k = 0;
        for (int x = 0; x < a.n_pois[q]; ++x) k += uu[j] >= a.pois[q][x] ? 1 : 0;
        Acc sum = I[j];
        if (k > 0) {
          uint4 v = make_uint4(0, 0, 0, 0);
          for (int e = 0; e < k; ++e) {
            if ((e & 7) == 0)
              v = philox10(make_uint4((uint32_t)i, t, 0u, kTagExtJ | ((uint32_t)(e >> 3) << 8)),
                           a.key0, a.key1);
            const int wsel = (e & 7) >> 1;
            const uint32_t word = wsel == 0 ? v.x : wsel == 1 ? v.y : wsel == 2 ? v.z : v.w;
            const uint32_t idx = (e & 1) ? (word & 0xFFFFu) : (word >> 16);
            sum += static_cast<const Acc*>(a.jxfix)[q * kQuantN + idx];
          }
        }
        const float dv = fix_to_f32(sum) * a.inv2q;
        float Vj = Vv[j], cj = cv[j];
        bool spk = false;
        if (rj > 0) {
          rj -= 1;
          cj = cj * a.Pc[q];
        } else {
          float vv = Vj - a.E[q];
          vv = vv * a.Pm[q];
          vv = a.E[q] + vv;
          const float cc = cj * a.PVc[q];
          vv = vv - cc;
          vv = vv + a.Iterm[q];
          vv = vv + dv;
          cj = cj * a.Pc[q];
          if (vv > a.Vth[q]) {
            spk = true;
            vv = a.Vr[q];
            cj = cj + a.alpha[q];
            rj = (uint32_t)a.n_arp[q];
          }
          Vj = vv;
        }
        Vv[j] = Vj;
        cv[j] = cj;
        if (spk) {
          const int pos = atomicAdd(&s_n, 1);
          s_spk[pos] = (int32_t)i;
        }
      }
      r_out |= rj << (8 * j);
    }
    *reinterpret_cast<float4*>(a.V + i0) = make_float4(Vv[0], Vv[1], Vv[2], Vv[3]);
    *reinterpret_cast<float4*>(a.c + i0) = make_float4(cv[0], cv[1], cv[2], cv[3]);
    *reinterpret_cast<uint32_t*>(a.ref + i0) = r_out;
  }
  __syncthreads();
  const int n = s_n;
  if (n == 0) return;
  if (tid == 0) {
    s_logbase = atomicAdd(a.log_count, (unsigned long long)n);
    atomicAdd(a.n_spikes, (unsigned long long)n);
  }
  __syncthreads();
  const uint32_t bin = (t / (uint32_t)a.rate_bin_steps) % (uint32_t)a.rate_bins_cap;
  for (int k = tid; k < n; k += 256) {
    const int32_t id = s_spk[k];
    const unsigned long long pos = s_logbase + (unsigned long long)k;
    if (pos < (unsigned long long)a.spike_log_cap) a.log[pos] = make_int2((int)t, id);
    const int32_t mod = id / a.K;
    const int q = (id - mod * a.K) < a.K_exc ? 0 : 1;
    atomicAdd(&a.rates[((int64_t)bin * a.M + mod) * 2 + q], 1u);
  }
  const int lane = tid & 63, wave = tid >> 6;
  for (int k = wave; k < n; k += 4) {
    const int32_t s = __builtin_amdgcn_readfirstlane(s_spk[k]);
    deliver_row<Acc, WDT>(a, s, t, lane);
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

hipError_t launch_step(const StepArgs& a, int wdt, int acc_bits, uint32_t t, hipStream_t st) {
  const dim3 grid((unsigned)(a.N_pad / 1024)), block(256);
  if (acc_bits == 32) {
    if (wdt == DPSNN_W_F32)
      hipLaunchKernelGGL((k_step<int32_t, DPSNN_W_F32>), grid, block, 0, st, a, t);
    else if (wdt == DPSNN_W_F16)
      hipLaunchKernelGGL((k_step<int32_t, DPSNN_W_F16>), grid, block, 0, st, a, t);
    else
      hipLaunchKernelGGL((k_step<int32_t, DPSNN_W_I8>), grid, block, 0, st, a, t);
  } else {
    if (wdt == DPSNN_W_F32)
      hipLaunchKernelGGL((k_step<int64_t, DPSNN_W_F32>), grid, block, 0, st, a, t);
    else if (wdt == DPSNN_W_F16)
      hipLaunchKernelGGL((k_step<int64_t, DPSNN_W_F16>), grid, block, 0, st, a, t);
    else
      hipLaunchKernelGGL((k_step<int64_t, DPSNN_W_I8>), grid, block, 0, st, a, t);
  }
  return hipGetLastError();
}

}  // namespace dpsnn
