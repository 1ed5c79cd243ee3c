// Host-side tables of libdpsnn, computed once per build in binary64 and
// rounded once to the width the device uses.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "dpsnn_internal.h"

namespace dpsnn {

namespace {

// Standard normal quantile.  Table entries are defined as the result of a
// bisection on Phi(x) = erfc(-x / sqrt 2) / 2 over [-40, 40] run until the
// midpoint no longer moves, taking the upper end, with the lower tail used
// for p > 1/2 through Phi^-1(p) = -Phi^-1(1 - p).  Fixing the procedure
// (not just the accuracy) fixes every binary64 bit of the table.
double quantile(double p) {
  if (p > 0.5) return -quantile(1.0 - p);
  double a = -40.0, b = 40.0;
  while (true) {
    const double m = 0.5 * (a + b);
    if (!(m > a && m < b)) break;
    if (0.5 * erfc(-m / sqrt(2.0)) < p)
      a = m;
    else
      b = m;
  }
  return b;
}

const std::vector<double>& normal_grid() {
  static std::vector<double> z;
  static std::once_flag once;
  std::call_once(once, [] {
    z.resize(kQuantN);
    for (int i = 0; i < kQuantN; ++i) z[i] = quantile((i + 0.5) / kQuantN);
  });
  return z;
}

// binary64 -> binary16, round to nearest even, from the bit fields.
uint16_t to_half(double x) {
  uint64_t b;
  memcpy(&b, &x, 8);
  const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
  const int ex = (int)((b >> 52) & 0x7FF);
  const uint64_t man = b & ((1ull << 52) - 1);
  if (ex == 0x7FF) return sign | (man ? 0x7E00 : 0x7C00);
  if (ex == 0) return sign;                 // binary64 subnormal -> 0
  const int e = ex - 1023;
  if (e > 15) return sign | 0x7C00;
  const uint64_t sig = (1ull << 52) | man;  // value = sig * 2^(e - 52)
  const int drop = e >= -14 ? 42 : 28 - e;  // bits below the half's unit
  if (drop > 62) return sign;
  uint64_t kept = sig >> drop;
  const uint64_t rest = sig & ((1ull << drop) - 1);
  const uint64_t halfway = 1ull << (drop - 1);
  if (rest > halfway || (rest == halfway && (kept & 1))) ++kept;
  if (e < -14) return sign | (uint16_t)kept;  // 1024 -> smallest normal
  const uint32_t v = ((uint32_t)(e + 15) << 10) + (uint32_t)(kept - 1024);
  return v >= 0x7C00 ? (uint16_t)(sign | 0x7C00) : (uint16_t)(sign | v);
}

double from_half(uint16_t h) {
  const int e = (h >> 10) & 31, m = h & 1023;
  double v = e == 0 ? ldexp((double)m, -24) : ldexp((double)(1024 + m), e - 25);
  return (h & 0x8000) ? -v : v;
}

}  // namespace

int validate(const dpsnn_params& p) {
  if (p.abi_version != DPSNN_ABI_VERSION) return DPSNN_E_INVAL;
  if (p.grid_w < 1 || p.grid_h < 1 || p.K < 4 || p.K_out < 0 || p.K_out > kMaxKout)
    return DPSNN_E_INVAL;
  const int64_t N = (int64_t)p.grid_w * p.grid_h * p.K;
  if (N > (int64_t)kTargetMask) return DPSNN_E_INVAL;  // target field of a row word
  if (!(p.frac_exc >= 0 && p.frac_exc <= 1)) return DPSNN_E_INVAL;
  for (int q = 0; q < 2; ++q) {
    if (!(p.frac_local[q] >= 0 && p.frac_local[q] <= 1)) return DPSNN_E_INVAL;
    if (!(p.tau_m[q] > 0) || !(p.tau_c[q] > 0) || !(p.tau_arp[q] >= 0))
      return DPSNN_E_INVAL;
    if (!(p.nu_ext_hz[q] >= 0) || !(p.J_sd[q] >= 0) || !(p.Jext_sd[q] >= 0))
      return DPSNN_E_INVAL;
    if (llround(p.tau_arp[q] / p.dt_ms) > 255) return DPSNN_E_INVAL;
  }
  if (!(p.lambda > 0) || !(p.dt_ms > 0)) return DPSNN_E_INVAL;
  if (p.torus != 1) return DPSNN_E_INVAL;
  if (p.d_min < 1 || p.d_max < p.d_min || p.d_max - p.d_min + 1 > kMaxDelays)
    return DPSNN_E_INVAL;
  if (p.weight_dtype < DPSNN_W_F32 || p.weight_dtype > DPSNN_W_I8) return DPSNN_E_INVAL;
  if (p.acc_bits != 32 && p.acc_bits != 64) return DPSNN_E_INVAL;
  if (p.q_frac_bits < 0 || p.q_frac_bits > (p.acc_bits == 32 ? 30 : 40))
    return DPSNN_E_INVAL;
  if (p.rate_bin_steps < 1 || p.rate_bins_cap < 1 || p.spike_log_cap < 0)
    return DPSNN_E_INVAL;
  if (p.queue_cap < -1 || p.queue_cap > (1 << 20)) return DPSNN_E_INVAL;
  const int M = p.grid_w * p.grid_h;
  for (int q = 0; q < 2; ++q) {
    const long nloc = llround(p.frac_local[q] * p.K_out);
    if (M == 1 && nloc < p.K_out) return DPSNN_E_INVAL;  // nowhere remote
  }
  return DPSNN_OK;
}

int compute_tables(const dpsnn_params& p, HostTables& T) {
  const int rc = validate(p);
  if (rc != DPSNN_OK) return rc;
  T.M = p.grid_w * p.grid_h;
  T.N = (int64_t)T.M * p.K;
  T.N_pad = (T.N + 1023) / 1024 * 1024;
  T.K_exc = (int32_t)llround(p.frac_exc * p.K);
  for (int q = 0; q < 2; ++q) T.n_local[q] = (int32_t)llround(p.frac_local[q] * p.K_out);
  T.D = p.d_max + 1;
  T.n_del = p.d_max - p.d_min + 1;
  T.row_stride = (p.K_out + 3) / 4 * 4;
  const double two_q = ldexp(1.0, p.q_frac_bits);

  for (int q = 0; q < 2; ++q) {
    // Eq. 2 over one step dt, exactly: c' = c Pc and
    // V' = E + (V - E) Pm - c gc (Pc - Pm) / (1/tau_m - 1/tau_c) + I tau_m (1 - Pm).
    const double Pm = exp(-p.dt_ms / p.tau_m[q]);
    const double Pc = exp(-p.dt_ms / p.tau_c[q]);
    const double rm = 1.0 / p.tau_m[q], rc_ = 1.0 / p.tau_c[q];
    const double PVc = rm != rc_ ? p.gc[q] * (Pc - Pm) / (rm - rc_)
                                 : p.gc[q] * p.dt_ms * Pm;
    const double It = p.I_const[q] * p.tau_m[q] * (1.0 - Pm);
    const double v[4] = {Pm, Pc, PVc, It};
    for (int k = 0; k < 4; ++k) {
      T.prop64[q][k] = v[k];
      T.prop32[q][k] = (float)v[k];
    }
    T.n_arp[q] = (int32_t)llround(p.tau_arp[q] / p.dt_ms);

    // Poisson counts of the external drive: threshold j is floor(F(j) 2^32)
    // for the Poisson CDF F of mean nu dt, kept while below 2^32 - 1.
    T.n_pois[q] = 0;
    const double mean = p.nu_ext_hz[q] * p.dt_ms * 1e-3;
    if (mean > 0) {
      double term = exp(-mean);
      double cdf = term;
      for (int j = 0; j < kMaxPois; ++j) {
        if (j) {
          term = term * mean / (double)j;
          cdf = cdf + term;
        }
        const double thr = floor(cdf * 4294967296.0);
        if (thr >= 4294967295.0) break;
        T.pois[q][T.n_pois[q]++] = (uint32_t)thr;
      }
    }
  }

  // Eq. 1 on the torus: offsets (ox, oy) enumerated row-major without
  // (0, 0); weight exp(-d / lambda) with d the Euclidean length of the
  // shortest periodic image; thresholds floor(cum / Z * 2^32) of the
  // running sums, the last offset taking the remainder.
  const int W = p.grid_w, H = p.grid_h;
  std::vector<double> wt;
  T.off_xy.clear();
  for (int oy = 0; oy < H; ++oy)
    for (int ox = 0; ox < W; ++ox) {
      if (!ox && !oy) continue;
      const int dx = std::min(ox, W - ox), dy = std::min(oy, H - oy);
      wt.push_back(exp(-sqrt((double)(dx * dx + dy * dy)) / p.lambda));
      T.off_xy.push_back(ox);
      T.off_xy.push_back(oy);
    }
  double Z = 0.0;
  for (double x : wt) Z += x;
  T.off_thr.clear();
  double run = 0.0;
  for (size_t k = 0; k + 1 < wt.size(); ++k) {
    run += wt[k];
    const double thr = floor(run / Z * 4294967296.0);
    T.off_thr.push_back(thr >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)thr);
  }

  // Efficacies (Sec. 2.2: Gaussian with mean J and SD Delta J): midpoint
  // quantile tables mu + sigma Phi^-1((i + 1/2) / 65536).
  const std::vector<double>& z = normal_grid();
  T.ext_bound = 0;
  for (int q = 0; q < 2; ++q) {
    T.wt64[q].resize(kQuantN);
    T.wt32[q].resize(kQuantN);
    T.wt16[q].resize(kQuantN);
    T.wq8[q].resize(kQuantN);
    T.jx64[q].resize(kQuantN);
    T.jx32[q].resize(kQuantN);
    T.jxfix[q].resize(kQuantN);
    double amax = 0.0;
    int64_t jmax = 0;
    for (int i = 0; i < kQuantN; ++i) {
      const double w = p.J_mean[q] + p.J_sd[q] * z[i];
      T.wt64[q][i] = w;
      T.wt32[q][i] = (float)w;
      T.wt16[q][i] = to_half(w);
      amax = std::max(amax, fabs(w));
      const double je = p.Jext_mean[q] + p.Jext_sd[q] * z[i];
      T.jx64[q][i] = je;
      T.jx32[q][i] = (float)je;
      T.jxfix[q][i] = (int64_t)rint((double)T.jx32[q][i] * two_q);
      jmax = std::max<int64_t>(jmax, std::llabs(T.jxfix[q][i]));
    }
    // int8 codes: scale s = max|w| / 127 held in binary32, code
    // rint(w / s) clipped to +-127, contribution code * rint(s 2^Q).
    T.s8[q] = (float)(amax > 0 ? amax / 127.0 : 1.0);
    T.s8fix[q] = (int64_t)rint((double)T.s8[q] * two_q);
    for (int i = 0; i < kQuantN; ++i) {
      double code = rint(T.wt64[q][i] / (double)T.s8[q]);
      code = std::min(127.0, std::max(-127.0, code));
      T.wq8[q][i] = (int8_t)code;
    }
    const int64_t b = (int64_t)(T.n_pois[q] + 1) * jmax;
    T.ext_bound = std::max(T.ext_bound, b);
  }
  return DPSNN_OK;
}

// Fixed-point value of a stored efficacy, as the device computes it.
static int64_t stored_fix(const dpsnn_params& p, const HostTables& T, int q, int i) {
  const double two_q = ldexp(1.0, p.q_frac_bits);
  if (p.weight_dtype == DPSNN_W_F32) return (int64_t)rint((double)T.wt32[q][i] * two_q);
  if (p.weight_dtype == DPSNN_W_F16) return (int64_t)rint(from_half(T.wt16[q][i]) * two_q);
  return (int64_t)T.wq8[q][i] * T.s8fix[q];
}

int64_t host_table(const HostTables& T, const char* name, void* out, int64_t cap) {
  auto put = [&](const void* src, int64_t bytes) -> int64_t {
    if (out && cap >= bytes) memcpy(out, src, (size_t)bytes);
    return bytes;
  };
  if (!strcmp(name, "prop_f64")) return put(T.prop64, sizeof(T.prop64));
  if (!strcmp(name, "prop_f32")) return put(T.prop32, sizeof(T.prop32));
  if (!strcmp(name, "n_arp")) return put(T.n_arp, sizeof(T.n_arp));
  if (!strcmp(name, "pois_thr_0")) return put(T.pois[0], 4 * (int64_t)T.n_pois[0]);
  if (!strcmp(name, "pois_thr_1")) return put(T.pois[1], 4 * (int64_t)T.n_pois[1]);
  if (!strcmp(name, "off_thr")) return put(T.off_thr.data(), 4 * (int64_t)T.off_thr.size());
  if (!strcmp(name, "off_xy")) return put(T.off_xy.data(), 4 * (int64_t)T.off_xy.size());
  if (!strcmp(name, "s8")) return put(T.s8, sizeof(T.s8));
  if (!strcmp(name, "s8fix")) return put(T.s8fix, sizeof(T.s8fix));
  for (int q = 0; q < 2; ++q) {
    const char d = (char)('0' + q);
    auto is = [&](const char* stem) {
      const size_t n = strlen(stem);
      return !strncmp(name, stem, n) && name[n] == d && name[n + 1] == 0;
    };
    if (is("wt64_")) return put(T.wt64[q].data(), 8 * (int64_t)kQuantN);
    if (is("wt32_")) return put(T.wt32[q].data(), 4 * (int64_t)kQuantN);
    if (is("wt16_")) return put(T.wt16[q].data(), 2 * (int64_t)kQuantN);
    if (is("wq8_")) return put(T.wq8[q].data(), (int64_t)kQuantN);
    if (is("jx64_")) return put(T.jx64[q].data(), 8 * (int64_t)kQuantN);
    if (is("jx32_")) return put(T.jx32[q].data(), 4 * (int64_t)kQuantN);
    if (is("jxfix_")) return put(T.jxfix[q].data(), 8 * (int64_t)kQuantN);
  }
  return DPSNN_E_INVAL;
}

// Fixed-point efficacy table by source pop for the stored format (host
// copy used by the build-time range check).
std::vector<int64_t> fix_table(const dpsnn_params& p, const HostTables& T, int q) {
  std::vector<int64_t> v(kQuantN);
  for (int i = 0; i < kQuantN; ++i) v[i] = stored_fix(p, T, q, i);
  return v;
}

}  // namespace dpsnn
