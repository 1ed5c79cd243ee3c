// Slow-wave analysis of module rates (Sec. 2.3, Eq. 4), on the rate bins
// held on the device.
//
// Per module, the signal is L(k) = log(c(k) + 1) - log(c_down + 1) + eta(k)
// with c(k) the module's spikes in bin k (all populations), c_down / c_up
// the rounded mean counts of the bins at or below / above the lower median
// of the window, and eta white noise of the given variance (Philox word 0
// of (module, bin, bin >> 32, WAVE) keyed by the seed, through the 65536
// standard normal quantiles).  The threshold is halfway between the levels
// in log units; a Down-to-Up transition at bin k needs min_down bins at or
// below the threshold before k and min_up bins above it from k on, and its
// time is the linear interpolation of L between the centres of bins k-1 and
// k.  Transitions of all modules are ordered by (k, interpolation fraction
// in 32-bit fixed point, module) and grouped greedily into waves (a module
// entering the current wave a second time starts the next).  Eq. 4 gives
// V = 1 / |grad T| from central differences of T over the modules of the
// wave (one-sided at the wave's edge, no wrap-around); the wave speed is
// the mean V.  Logarithms of integers come from a table built on the host,
// so that every threshold decision is the same binary64 comparison on any
// machine.
#include <algorithm>

#include "dpsnn_internal.h"
#include "philox.h"

namespace dpsnn {

constexpr uint32_t kTagWave = 5;  // analysis noise of module m, bin b: (m, b, b >> 32, WAVE)

// Count of module m in window bin k: sum over the populations.
__device__ __forceinline__ uint32_t wave_count(const WaveArgs& a, int m, int k) {
  const int64_t b = (a.slot0 + k) % a.ring;
  const uint32_t* p = a.counts + (b * a.M_stride + a.mbase + m) * a.P;
  uint32_t s = 0;
  for (int q = 0; q < a.P; ++q) s += p[q];
  return s;
}

// Largest count of the window (for the size of the log table).
__global__ void __launch_bounds__(256) k_wave_max(WaveArgs a, uint32_t* out) {
  const int m = blockIdx.x;
  uint32_t mx = 0;
  for (int k = threadIdx.x; k < a.nb; k += blockDim.x) {
    const uint32_t c = wave_count(a, m, k);
    mx = c > mx ? c : mx;
  }
  atomicMax(out, mx);
}

// One block per module: levels, threshold, signal, transitions (in bin
// order) into the module's list.
__global__ void __launch_bounds__(256) k_wave_levels(WaveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nb = a.nb, m = blockIdx.x, tid = threadIdx.x;
  int np2 = 1;
  while (np2 < nb) np2 <<= 1;
  uint32_t* c = reinterpret_cast<uint32_t*>(smem);             // [nb]
  double* L = reinterpret_cast<double*>(smem + ((nb * 4 + 15) & ~15));  // [nb]
  uint32_t* srt = reinterpret_cast<uint32_t*>(L);              // [np2], before L
  __shared__ unsigned long long s_sum[4];
  for (int k = tid; k < np2; k += blockDim.x) {
    const uint32_t v = k < nb ? wave_count(a, m, k) : 0xFFFFFFFFu;
    if (k < nb) c[k] = v;
    srt[k] = v;
  }
  if (tid < 4) s_sum[tid] = 0;
  __syncthreads();
  // bitonic sort of the counts, padded with the largest value
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < np2; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const uint32_t x = srt[i], y = srt[j];
          if ((x > y) == up) {
            srt[i] = y;
            srt[j] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  const uint32_t med = srt[(nb - 1) / 2];
  unsigned long long slo = 0, nlo = 0, shi = 0, nhi = 0;
  for (int k = tid; k < nb; k += blockDim.x) {
    const uint32_t v = c[k];
    if (v <= med) {
      slo += v;
      nlo += 1;
    } else {
      shi += v;
      nhi += 1;
    }
  }
  atomicAdd(&s_sum[0], slo);
  atomicAdd(&s_sum[1], nlo);
  atomicAdd(&s_sum[2], shi);
  atomicAdd(&s_sum[3], nhi);
  __syncthreads();  // the sorted copy is no longer needed: L overwrites it
  const unsigned long long Slo = s_sum[0], Nlo = s_sum[1], Shi = s_sum[2], Nhi = s_sum[3];
  if (Nhi == 0) {  // no Up bins: no transitions
    if (tid == 0) a.cnt[m] = 0;
    return;
  }
  const unsigned long long cd = (2 * Slo + Nlo) / (2 * Nlo);
  const unsigned long long cu = (2 * Shi + Nhi) / (2 * Nhi);
  const double ld = a.lnt[cd + 1];
  const double theta = 0.5 * (a.lnt[cu + 1] - ld);
  for (int k = tid; k < nb; k += blockDim.x) {
    const uint64_t bin = (uint64_t)(a.bin0 + k);
    const uint4 u = philox10(make_uint4((uint32_t)m, (uint32_t)bin, (uint32_t)(bin >> 32), kTagWave),
                             a.key0, a.key1);
    const double eta = a.sd * a.z[u.x >> 16];
    L[k] = (a.lnt[c[k] + 1] - ld) + eta;
  }
  __syncthreads();
  // transitions, written in bin order: block-wide ordered compaction
  __shared__ uint32_t s_wc[4];
  const int lane = tid & 63, wv = tid >> 6;
  uint32_t base = 0;
  for (int k0 = 0; k0 < nb; k0 += blockDim.x) {
    const int k = k0 + tid;
    bool hit = k >= a.min_down && k + a.min_up <= nb;
    for (int j = k - a.min_down; hit && j < k; ++j) hit = L[j] <= theta;
    for (int j = k; hit && j < k + a.min_up; ++j) hit = L[j] > theta;
    const unsigned long long bal = __ballot(hit);
    if (lane == 0) s_wc[wv] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = base;
    for (int w = 0; w < wv; ++w) before += s_wc[w];
    before += (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
    if (hit && before < (uint32_t)a.cap_pm) {
      const double frac = (theta - L[k - 1]) / (L[k] - L[k - 1]);
      const double fq = frac * 4294967296.0;
      const int64_t o = (int64_t)m * a.cap_pm + before;
      a.tr_k[o] = (uint32_t)k;
      a.tr_q[o] = fq < 4294967295.0 ? (uint32_t)fq : 4294967295u;
      a.tr_T[o] = ((double)(a.bin0 + k) - 0.5 + frac) * a.dbin;
    }
    base += s_wc[0] + s_wc[1] + s_wc[2] + s_wc[3];
    __syncthreads();
  }
  if (tid == 0) a.cnt[m] = base < (uint32_t)a.cap_pm ? base : (uint32_t)a.cap_pm;
}

// Histogram of the transitions over their bins.
__global__ void __launch_bounds__(256) k_wave_hist(WaveArgs a) {
  const int m = blockIdx.x;
  for (uint32_t j = threadIdx.x; j < a.cnt[m]; j += blockDim.x)
    atomicAdd(&a.hist[a.tr_k[(int64_t)m * a.cap_pm + j]], 1u);
}

// Exclusive prefix of the histogram (one block): bucket offsets.
__global__ void __launch_bounds__(1024) k_wave_scan(WaveArgs a) {
  __shared__ uint32_t s[1024];
  const int tid = threadIdx.x;
  const int per = (a.nb + 1023) / 1024;
  const int lo = tid * per, hi = lo + per < a.nb ? lo + per : a.nb;
  uint32_t run = 0;
  for (int k = lo; k < hi; ++k) run += a.hist[k];
  s[tid] = run;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t v = tid >= o ? s[tid - o] : 0u;
    __syncthreads();
    s[tid] += v;
    __syncthreads();
  }
  uint32_t acc = s[tid] - run;
  for (int k = lo; k < hi; ++k) {
    a.off[k] = acc;
    acc += a.hist[k];
  }
  if (tid == 1023) a.off[a.nb] = s[1023];
}

// Scatter into the buckets (order inside a bucket: arbitrary, sorted next).
__global__ void __launch_bounds__(256) k_wave_scatter(WaveArgs a) {
  const int m = blockIdx.x;
  for (uint32_t j = threadIdx.x; j < a.cnt[m]; j += blockDim.x) {
    const int64_t o = (int64_t)m * a.cap_pm + j;
    const uint32_t k = a.tr_k[o];
    const uint32_t pos = a.off[k] + atomicAdd(&a.fill[k], 1u);
    a.keys[pos] = ((unsigned long long)a.tr_q[o] << 32) |
                  ((unsigned long long)m << 12) | (unsigned long long)j;
  }
}

// One block per bucket: bitonic sort of its keys (fraction, module) in LDS.
__global__ void __launch_bounds__(256) k_wave_bsort(WaveArgs a) {
  extern __shared__ __align__(16) unsigned long long sk[];
  const int b = blockIdx.x;
  const uint32_t o0 = a.off[b], n = a.off[b + 1] - o0;
  if (n < 2) return;
  uint32_t np2 = 1;
  while (np2 < n) np2 <<= 1;
  for (uint32_t i = threadIdx.x; i < np2; i += blockDim.x)
    sk[i] = i < n ? a.keys[o0 + i] : ~0ull;
  __syncthreads();
  for (uint32_t size = 2; size <= np2; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < np2; i += blockDim.x) {
        const uint32_t j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const unsigned long long x = sk[i], y = sk[j];
          if ((x > y) == up) {
            sk[i] = y;
            sk[j] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) a.keys[o0 + i] = sk[i];
}

// Greedy grouping over the ordered transitions.  A wave that starts at
// position s ends just before the first position whose module already
// occurred at or after s: nxt(s) = min over s' >= s of next(s'), next(s')
// being the following position of the module at s'.  So the wave starts
// are the chain 0, nxt(0), nxt(nxt(0)), ...: the next positions and their
// suffix minimum are computed in parallel, the chain is walked once per
// wave, and every position then finds its wave by bisection.

// Position of every transition in the order: pos[m][j] = i.
__global__ void __launch_bounds__(256) k_wave_inv(WaveArgs a) {
  const uint32_t total = a.off[a.nb];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += gridDim.x * blockDim.x) {
    const unsigned long long key = a.keys[i];
    const int m = (int)((key >> 12) & 0xFFFFFu);
    const uint32_t j = (uint32_t)(key & 0xFFFu);
    a.pos[(int64_t)m * a.cap_pm + j] = i;
  }
}

// next(i): the position of the same module's following transition, or
// total.
__global__ void __launch_bounds__(256) k_wave_next(WaveArgs a) {
  const uint32_t total = a.off[a.nb];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += gridDim.x * blockDim.x) {
    const unsigned long long key = a.keys[i];
    const int m = (int)((key >> 12) & 0xFFFFFu);
    const uint32_t j = (uint32_t)(key & 0xFFFu);
    a.nxt[i] = j + 1 < a.cnt[m] ? a.pos[(int64_t)m * a.cap_pm + j + 1] : total;
  }
}

// Suffix minimum of next() in place (one block): nxt(s).
__global__ void __launch_bounds__(1024) k_wave_sufmin(WaveArgs a) {
  __shared__ uint32_t s[1024];
  const int tid = threadIdx.x;
  const uint32_t total = a.off[a.nb];
  const uint32_t per = (total + 1023) / 1024;
  const uint32_t lo = tid * per < total ? tid * per : total;
  const uint32_t hi = lo + per < total ? lo + per : total;
  uint32_t run = total;
  for (uint32_t i = hi; i > lo; --i) {
    const uint32_t v = a.nxt[i - 1];
    run = v < run ? v : run;
    a.nxt[i - 1] = run;
  }
  s[tid] = run;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // suffix minimum of the chunk minima
    const uint32_t v = tid + o < 1024 ? s[tid + o] : total;
    __syncthreads();
    s[tid] = v < s[tid] ? v : s[tid];
    __syncthreads();
  }
  const uint32_t later = tid + 1 < 1024 ? s[tid + 1] : total;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t v = a.nxt[i];
    a.nxt[i] = later < v ? later : v;
  }
}

// The chain of wave starts (one thread).
__global__ void k_wave_chain(WaveArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t total = a.off[a.nb];
  int32_t w = 0;
  for (uint32_t st = 0; st < total; st = a.nxt[st]) a.wave_first[w++] = (int32_t)st;
  a.wave_first[w] = (int32_t)total;
  a.n_waves[0] = w;
}

// Module, time and wave of every position.
__global__ void __launch_bounds__(256) k_wave_assign(WaveArgs a) {
  const uint32_t total = a.off[a.nb];
  const int32_t nw = a.n_waves[0];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += gridDim.x * blockDim.x) {
    const unsigned long long key = a.keys[i];
    const int m = (int)((key >> 12) & 0xFFFFFu);
    const uint32_t j = (uint32_t)(key & 0xFFFu);
    int32_t l = 0, h = nw - 1;  // last wave whose first position is <= i
    while (l < h) {
      const int32_t mid = (l + h + 1) >> 1;
      if ((uint32_t)a.wave_first[mid] <= i)
        l = mid;
      else
        h = mid - 1;
    }
    a.out_module[i] = m;
    a.out_T[i] = a.tr_T[(int64_t)m * a.cap_pm + j];
    a.out_wave[i] = l;
  }
}

// One block per wave of the batch starting at wave w0: Eq. 4 over the
// wave's modules; the batch's transition-time grids are a.grid[batch][M].
__global__ void __launch_bounds__(256) k_wave_speed(WaveArgs a, int32_t w0) {
  __shared__ double s_sum[4], s_min[4];
  __shared__ int32_t s_cnt[4];
  const int w = w0 + (int)blockIdx.x, tid = threadIdx.x;
  double* g = a.grid + (int64_t)blockIdx.x * a.M;
  const int32_t i0 = a.wave_first[w], i1 = a.wave_first[w + 1];
  for (int m = tid; m < a.M; m += blockDim.x) g[m] = __builtin_nan("");
  __syncthreads();
  for (int32_t i = i0 + tid; i < i1; i += blockDim.x) g[a.out_module[i]] = a.out_T[i];
  __threadfence_block();
  __syncthreads();
  double sum = 0.0, tmin = __builtin_inf();
  int32_t cnt = 0;
  const bool measured = i1 - i0 >= a.min_modules;
  for (int32_t i = i0 + tid; i < i1; i += blockDim.x) {
    const int m = a.out_module[i];
    const double Tm = g[m];
    tmin = Tm < tmin ? Tm : tmin;
    if (!measured) continue;
    const int x = m % a.W, y = m / a.W;
    const double tl = x > 0 ? g[m - 1] : __builtin_nan("");
    const double tr = x + 1 < a.W ? g[m + 1] : __builtin_nan("");
    const double td = y > 0 ? g[m - a.W] : __builtin_nan("");
    const double tu = y + 1 < a.H ? g[m + a.W] : __builtin_nan("");
    double gx, gy;
    if (!__builtin_isnan(tl) && !__builtin_isnan(tr)) gx = 0.5 * (tr - tl);
    else if (!__builtin_isnan(tr)) gx = tr - Tm;
    else if (!__builtin_isnan(tl)) gx = Tm - tl;
    else continue;
    if (!__builtin_isnan(td) && !__builtin_isnan(tu)) gy = 0.5 * (tu - td);
    else if (!__builtin_isnan(tu)) gy = tu - Tm;
    else if (!__builtin_isnan(td)) gy = Tm - td;
    else continue;
    const double g2 = gx * gx + gy * gy;
    if (g2 == 0.0) continue;
    sum += 1000.0 / __builtin_sqrt(g2);
    cnt += 1;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_down(sum, o);
    cnt += __shfl_down(cnt, o);
    const double v = __shfl_down(tmin, o);
    tmin = v < tmin ? v : tmin;
  }
  if ((tid & 63) == 0) {
    s_sum[tid >> 6] = sum;
    s_cnt[tid >> 6] = cnt;
    s_min[tid >> 6] = tmin;
  }
  __syncthreads();
  if (tid == 0) {
    double S = 0.0, T0 = __builtin_inf();
    int32_t N = 0;
    for (int k = 0; k < 4; ++k) {
      S += s_sum[k];
      N += s_cnt[k];
      T0 = s_min[k] < T0 ? s_min[k] : T0;
    }
    a.wave_speed[w] = N > 0 ? S / (double)N : __builtin_nan("");
    a.wave_t0[w] = T0;
    a.wave_n[w] = i1 - i0;
  }
}

// Mean of the measured wave speeds, summed in wave order (one thread).
__global__ void k_wave_mean(WaveArgs a, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  int64_t n = 0;
  for (int32_t w = 0; w < a.n_waves[0]; ++w) {
    const double v = a.wave_speed[w];
    if (!__builtin_isnan(v)) {
      s += v;
      n += 1;
    }
  }
  out[0] = n > 0 ? s / (double)n : __builtin_nan("");
}

hipError_t launch_wave_mean(const WaveArgs& a, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_wave_mean, dim3(1), dim3(64), 0, st, a, out);
  return hipGetLastError();
}

hipError_t launch_wave_max(const WaveArgs& a, uint32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_wave_max, dim3((unsigned)a.M), dim3(256), 0, st, a, out);
  return hipGetLastError();
}

hipError_t launch_wave_transitions(const WaveArgs& a, hipStream_t st) {
  const size_t lds = (size_t)((a.nb * 4 + 15) & ~15) + (size_t)a.nb * 8;
  int np2 = 1;
  while (np2 < a.nb) np2 <<= 1;
  const size_t lds_sort = (size_t)((a.nb * 4 + 15) & ~15) + (size_t)np2 * 4;
  hipLaunchKernelGGL(k_wave_levels, dim3((unsigned)a.M), dim3(256),
                     lds > lds_sort ? lds : lds_sort, st, a);
  hipLaunchKernelGGL(k_wave_hist, dim3((unsigned)a.M), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_wave_scan, dim3(1), dim3(1024), 0, st, a);
  hipLaunchKernelGGL(k_wave_scatter, dim3((unsigned)a.M), dim3(256), 0, st, a);
  int mp2 = 1;
  while (mp2 < a.M) mp2 <<= 1;
  hipLaunchKernelGGL(k_wave_bsort, dim3((unsigned)a.nb), dim3(256), (size_t)mp2 * 8, st, a);
  const unsigned gb = (unsigned)std::min<int64_t>(4096, ((int64_t)a.M * a.cap_pm + 255) / 256);
  hipLaunchKernelGGL(k_wave_inv, dim3(gb), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_wave_next, dim3(gb), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_wave_sufmin, dim3(1), dim3(1024), 0, st, a);
  hipLaunchKernelGGL(k_wave_chain, dim3(1), dim3(64), 0, st, a);
  hipLaunchKernelGGL(k_wave_assign, dim3(gb), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_wave_speed(const WaveArgs& a, int32_t w0, int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wave_speed, dim3((unsigned)n), dim3(256), 0, st, a, w0);
  return hipGetLastError();
}

}  // namespace dpsnn
