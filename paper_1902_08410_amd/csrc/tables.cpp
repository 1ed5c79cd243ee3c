// Host-side tables of libdpsnn, computed once per build in binary64 and
// rounded once to the width the device uses.
#include <math.h>

#include <cmath>
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
  if (!(p.lambda > 0) || !(p.dt_ms > 0)) return DPSNN_E_INVAL;
  if (p.d_min < 1 || p.d_max < p.d_min || p.d_max - p.d_min + 1 > kMaxDelays)
    return DPSNN_E_INVAL;
  if (p.weight_dtype < DPSNN_W_F32 || p.weight_dtype > DPSNN_W_I8) return DPSNN_E_INVAL;
  if (p.acc_bits != 32 && p.acc_bits != 64) return DPSNN_E_INVAL;
  if (p.plastic != 0 && p.plastic != 1) return DPSNN_E_INVAL;
  if (p.plastic) {
    if (p.weight_dtype != DPSNN_W_F32 || p.stdp_update_steps < 1 ||
        p.stdp_update_steps > (1 << 24))
      return DPSNN_E_INVAL;
    if (!(p.stdp_A_plus >= 0) || !(p.stdp_A_minus >= 0) || !(p.stdp_tau_plus > 0) ||
        !(p.stdp_tau_minus > 0) || !(p.stdp_tau_y > 0) || !std::isfinite(p.stdp_eta) ||
        !(p.stdp_w_max > 0) || !std::isfinite(p.stdp_w_max))
      return DPSNN_E_INVAL;
  }
  if (p.q_frac_bits < 0 || p.q_frac_bits > (p.acc_bits == 32 ? 30 : 40))
    return DPSNN_E_INVAL;
  if (p.rate_bin_steps < 1 || p.rate_bins_cap < 1 || p.spike_log_cap < 0)
    return DPSNN_E_INVAL;
  if (p.queue_cap < -1 || p.queue_cap > (1 << 20)) return DPSNN_E_INVAL;
  const int M = p.grid_w * p.grid_h;
  if (p.n_pops == 0) {
    if (!(p.frac_exc >= 0 && p.frac_exc <= 1)) return DPSNN_E_INVAL;
    for (int q = 0; q < 2; ++q) {
      if (!(p.frac_local[q] >= 0 && p.frac_local[q] <= 1)) return DPSNN_E_INVAL;
      if (!(p.tau_m[q] > 0) || !(p.tau_c[q] > 0) || !(p.tau_arp[q] >= 0))
        return DPSNN_E_INVAL;
      if (!(p.nu_ext_hz[q] >= 0) || !(p.J_sd[q] >= 0) || !(p.Jext_sd[q] >= 0))
        return DPSNN_E_INVAL;
      if (llround(p.tau_arp[q] / p.dt_ms) > 255) return DPSNN_E_INVAL;
      const long nloc = llround(p.frac_local[q] * p.K_out);
      if (M == 1 && nloc < p.K_out) return DPSNN_E_INVAL;  // nowhere remote
    }
    if (p.torus != 0 && p.torus != 1) return DPSNN_E_INVAL;
    return DPSNN_OK;
  }
  if (p.n_pops < 2 || p.n_pops > kMaxPops) return DPSNN_E_INVAL;
  if (p.open_boundary != 0 && p.open_boundary != 1) return DPSNN_E_INVAL;
  int64_t sum = 0;
  for (int q = 0; q < p.n_pops; ++q) {
    if (p.pop_size[q] < 1) return DPSNN_E_INVAL;
    sum += p.pop_size[q];
    if (!(p.p_tau_m[q] > 0) || !(p.p_tau_c[q] > 0) || !(p.p_tau_arp[q] >= 0))
      return DPSNN_E_INVAL;
    if (!(p.p_nu_ext_hz[q] >= 0) || !(p.p_Jext_sd[q] >= 0)) return DPSNN_E_INVAL;
    if (llround(p.p_tau_arp[q] / p.dt_ms) > 255) return DPSNN_E_INVAL;
  }
  if (sum != p.K) return DPSNN_E_INVAL;
  for (int s = 0; s < p.n_pops; ++s) {
    int64_t deg = 0;
    for (int t = 0; t < p.n_pops; ++t) {
      if (p.n_syn[t][s] < 0 || !(p.J_sd_ts[t][s] >= 0)) return DPSNN_E_INVAL;
      deg += p.n_syn[t][s];
      if (t == s && p.n_syn[t][s] > 0 && p.pop_size[t] < 2) return DPSNN_E_INVAL;
    }
    if (deg != p.K_out) return DPSNN_E_INVAL;  // rows of one length
  }
  return DPSNN_OK;
}

namespace {

// Populations, their parameters and the synapse blocks of every source
// population, from either parameter model.
struct PopParams {
  double tau_m, E, V_th, V_r, tau_arp, alpha_c, tau_c, gc, I_const;
  double nu_ext, Jx_mean, Jx_sd;
};

void population_model(const dpsnn_params& p, HostTables& T, PopParams* pp) {
  if (p.n_pops == 0) {
    // two populations; a source's first round(frac_local K_out) synapses
    // stay in its module, the others go to other modules (Eq. 1); a target
    // is any neuron of the module; both blocks share the source's table
    const int K_exc = (int)llround(p.frac_exc * p.K);
    T.P = 2;
    T.pop_lo[0] = 0;
    T.pop_hi[0] = K_exc;
    T.pop_lo[1] = K_exc;
    T.pop_hi[1] = p.K;
    for (int q = 0; q < 2; ++q) {
      pp[q] = {p.tau_m[q], p.E[q], p.V_th[q], p.V_r[q], p.tau_arp[q], p.alpha_c[q],
               p.tau_c[q], p.gc[q], p.I_const[q], p.nu_ext_hz[q], p.Jext_mean[q],
               p.Jext_sd[q]};
      const int nl = (int)llround(p.frac_local[q] * p.K_out);
      int b = 0;
      if (nl > 0) {
        T.blk_n[q][b] = nl;
        T.blk_rule[q][b++] = kRuleOwn;
      }
      if (p.K_out - nl > 0) {
        T.blk_n[q][b] = p.K_out - nl;
        T.blk_rule[q][b++] = kRuleOthers;
      }
      for (int k = 0; k < 2; ++k) {
        T.blk_lo[q][k] = 0;
        T.blk_hi[q][k] = p.K;
        T.blk_J[q][k] = p.J_mean[q];
        T.blk_sd[q][k] = p.J_sd[q];
      }
      T.n_blk[q] = b;
    }
    T.open = p.torus ? 0 : 1;  // torus = 0: the grid has edges
    return;
  }
  T.P = p.n_pops;
  int lo = 0;
  for (int q = 0; q < T.P; ++q) {
    T.pop_lo[q] = lo;
    lo += p.pop_size[q];
    T.pop_hi[q] = lo;
    pp[q] = {p.p_tau_m[q], p.p_E[q], p.p_V_th[q], p.p_V_r[q], p.p_tau_arp[q],
             p.p_alpha_c[q], p.p_tau_c[q], p.p_gc[q], p.p_I_const[q], p.p_nu_ext_hz[q],
             p.p_Jext_mean[q], p.p_Jext_sd[q]};
  }
  for (int s = 0; s < T.P; ++s) {
    int b = 0;
    for (int t = 0; t < T.P; ++t) {
      if (!p.n_syn[t][s]) continue;
      T.blk_n[s][b] = p.n_syn[t][s];
      T.blk_lo[s][b] = T.pop_lo[t];
      T.blk_hi[s][b] = T.pop_hi[t];
      T.blk_rule[s][b] = p.pop_exc[s] ? kRuleAll : kRuleOwn;
      T.blk_J[s][b] = p.J_mean_ts[t][s];
      T.blk_sd[s][b] = p.J_sd_ts[t][s];
      ++b;
    }
    T.n_blk[s] = b;
  }
  T.open = p.open_boundary;
}

}  // namespace

static int64_t stored_fix(const dpsnn_params& p, const HostTables& T, int q, int b, int i);

// int32 input slots: the parts of the fixed-point range bound that the
// parameters alone decide (the per-neuron sum over incoming synapses needs
// the rows and is checked at build): every single efficacy, the largest
// external sum of one step, and a plastic efficacy's upper clip w_max must
// each be below 2^31.
static int range_check(const dpsnn_params& p, const HostTables& T) {
  if (p.acc_bits != 32) return DPSNN_OK;
  const int64_t lim = (int64_t)1 << 31;
  if (T.ext_bound >= lim) return DPSNN_E_RANGE;
  if (p.plastic && ldexp(p.stdp_w_max, p.q_frac_bits) >= 2147483647.5) return DPSNN_E_RANGE;
  for (int q = 0; q < T.P; ++q)
    for (int b = 0; b < T.tables(q); ++b)
      for (int i = 0; i < kQuantN; ++i) {
        const int64_t v = stored_fix(p, T, q, b, i);
        if (v >= lim || v <= -lim) return DPSNN_E_RANGE;
      }
  return DPSNN_OK;
}

int compute_tables(const dpsnn_params& p, HostTables& T) {
  const int rc = validate(p);
  if (rc != DPSNN_OK) return rc;
  T.M = p.grid_w * p.grid_h;
  T.N = (int64_t)T.M * p.K;
  T.N_pad = (T.N + 1023) / 1024 * 1024;
  T.D = p.d_max + 1;
  T.n_del = p.d_max - p.d_min + 1;
  T.row_stride = (p.K_out + 3) / 4 * 4;
  const double two_q = ldexp(1.0, p.q_frac_bits);
  PopParams pp[kMaxPops];
  population_model(p, T, pp);

  bool others = false, all = false;
  for (int q = 0; q < T.P; ++q) {
    for (int b = 0; b < T.n_blk[q]; ++b) {
      others |= T.blk_rule[q][b] == kRuleOthers;
      all |= T.blk_rule[q][b] == kRuleAll;
    }
    // Eq. 2 over one step dt, exactly: c' = c Pc and
    // V' = E + (V - E) Pm - c gc (Pc - Pm) / (1/tau_m - 1/tau_c) + I tau_m (1 - Pm).
    const PopParams& a = pp[q];
    const double Pm = exp(-p.dt_ms / a.tau_m);
    const double Pc = exp(-p.dt_ms / a.tau_c);
    const double rm = 1.0 / a.tau_m, rc_ = 1.0 / a.tau_c;
    const double PVc = rm != rc_ ? a.gc * (Pc - Pm) / (rm - rc_) : a.gc * p.dt_ms * Pm;
    const double It = a.I_const * a.tau_m * (1.0 - Pm);
    const double v[4] = {Pm, Pc, PVc, It};
    for (int k = 0; k < 4; ++k) {
      T.prop64[q][k] = v[k];
      T.prop32[q][k] = (float)v[k];
    }
    T.n_arp[q] = (int32_t)llround(a.tau_arp / p.dt_ms);
    T.E[q] = a.E;
    T.Vth[q] = a.V_th;
    T.Vr[q] = a.V_r;
    T.alpha[q] = a.alpha_c;

    // Poisson counts of the external drive: threshold j is floor(F(j) 2^32)
    // for the Poisson CDF F of mean nu dt, kept while below 2^32 - 1.
    T.n_pois[q] = 0;
    const double mean = a.nu_ext * p.dt_ms * 1e-3;
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
  if (others && all) return DPSNN_E_INVAL;  // one offset table per network

  // Eq. 1: weight exp(-d / lambda) per offset; thresholds floor(cum / Z 2^32)
  // of the running sums, the last offset taking the remainder.  Offsets:
  //  - to other modules on the torus: (ox, oy) row-major over [0,W) x [0,H)
  //    without (0, 0), d the length of the shortest periodic image;
  //  - to any module on the torus: the same with (0, 0);
  //  - with open edges: (dx, dy) row-major over [-(W-1), W-1] x
  //    [-(H-1), H-1], d = |(dx, dy)|, without (0, 0) to other modules; the
  //    device repeats a draw that leaves the grid.
  const int W = p.grid_w, H = p.grid_h;
  std::vector<double> wt;
  T.off_xy.clear();
  if (!T.open) {
    for (int oy = 0; oy < H; ++oy)
      for (int ox = 0; ox < W; ++ox) {
        if (!ox && !oy && !all) continue;
        const int dx = std::min(ox, W - ox), dy = std::min(oy, H - oy);
        wt.push_back(exp(-sqrt((double)(dx * dx + dy * dy)) / p.lambda));
        T.off_xy.push_back(ox);
        T.off_xy.push_back(oy);
      }
  } else {
    for (int dy = 1 - H; dy < H; ++dy)
      for (int dx = 1 - W; dx < W; ++dx) {
        if (!dx && !dy && !all) continue;
        wt.push_back(exp(-sqrt((double)(dx * dx + dy * dy)) / p.lambda));
        T.off_xy.push_back(dx);
        T.off_xy.push_back(dy);
      }
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
  // quantile tables mu + sigma Phi^-1((i + 1/2) / 65536), one per (source
  // pop, block); external ones per target pop.
  const std::vector<double>& z = normal_grid();
  T.ext_bound = 0;
  for (int q = 0; q < T.P; ++q) {
    double amax = 0.0;
    for (int b = 0; b < T.tables(q); ++b) {
      T.wt64[q][b].resize(kQuantN);
      T.wt32[q][b].resize(kQuantN);
      T.wt16[q][b].resize(kQuantN);
      T.wq8[q][b].resize(kQuantN);
      for (int i = 0; i < kQuantN; ++i) {
        const double w = T.blk_J[q][b] + T.blk_sd[q][b] * z[i];
        T.wt64[q][b][i] = w;
        T.wt32[q][b][i] = (float)w;
        T.wt16[q][b][i] = to_half(w);
        amax = std::max(amax, fabs(w));
      }
    }
    // int8 codes: one scale per source pop, s = max|w| / 127 held in
    // binary32, code rint(w / s) clipped to +-127, contribution
    // code * rint(s 2^Q).
    T.s8[q] = (float)(amax > 0 ? amax / 127.0 : 1.0);
    T.s8fix[q] = (int64_t)rint((double)T.s8[q] * two_q);
    for (int b = 0; b < T.tables(q); ++b)
      for (int i = 0; i < kQuantN; ++i) {
        double code = rint(T.wt64[q][b][i] / (double)T.s8[q]);
        code = std::min(127.0, std::max(-127.0, code));
        T.wq8[q][b][i] = (int8_t)code;
      }
    T.jx64[q].resize(kQuantN);
    T.jx32[q].resize(kQuantN);
    T.jxfix[q].resize(kQuantN);
    int64_t jmax = 0;
    for (int i = 0; i < kQuantN; ++i) {
      const double je = pp[q].Jx_mean + pp[q].Jx_sd * z[i];
      T.jx64[q][i] = je;
      T.jx32[q][i] = (float)je;
      T.jxfix[q][i] = (int64_t)rint((double)T.jx32[q][i] * two_q);
      jmax = std::max<int64_t>(jmax, std::llabs(T.jxfix[q][i]));
    }
    const int64_t bnd = (int64_t)(T.n_pois[q] + 1) * jmax;
    T.ext_bound = std::max(T.ext_bound, bnd);
  }
  return range_check(p, T);
}

// Fixed-point value of a stored efficacy, as the device computes it.
static int64_t stored_fix(const dpsnn_params& p, const HostTables& T, int q, int b, int i) {
  const double two_q = ldexp(1.0, p.q_frac_bits);
  if (p.weight_dtype == DPSNN_W_F32) return (int64_t)rint((double)T.wt32[q][b][i] * two_q);
  if (p.weight_dtype == DPSNN_W_F16) return (int64_t)rint(from_half(T.wt16[q][b][i]) * two_q);
  return (int64_t)T.wq8[q][b][i] * T.s8fix[q];
}

int64_t host_table(const HostTables& T, const char* name, void* out, int64_t cap) {
  auto put = [&](const void* src, int64_t bytes) -> int64_t {
    if (out && cap >= bytes) memcpy(out, src, (size_t)bytes);
    return bytes;
  };
  const int P = T.P;
  if (!strcmp(name, "prop_f64")) return put(T.prop64, 32 * (int64_t)P);
  if (!strcmp(name, "prop_f32")) return put(T.prop32, 16 * (int64_t)P);
  if (!strcmp(name, "n_arp")) return put(T.n_arp, 4 * (int64_t)P);
  if (!strcmp(name, "off_thr")) return put(T.off_thr.data(), 4 * (int64_t)T.off_thr.size());
  if (!strcmp(name, "off_xy")) return put(T.off_xy.data(), 4 * (int64_t)T.off_xy.size());
  if (!strcmp(name, "s8")) return put(T.s8, 4 * (int64_t)P);
  if (!strcmp(name, "s8fix")) return put(T.s8fix, 8 * (int64_t)P);
  if (!strcmp(name, "blocks")) {  // [pop][block][n, lo, hi, rule]
    int32_t v[kMaxPops * kMaxPops * 4] = {};
    for (int q = 0; q < P; ++q)
      for (int b = 0; b < T.n_blk[q]; ++b) {
        int32_t* e = v + (q * kMaxPops + b) * 4;
        e[0] = T.blk_n[q][b];
        e[1] = T.blk_lo[q][b];
        e[2] = T.blk_hi[q][b];
        e[3] = T.blk_rule[q][b];
      }
    return put(v, 16 * (int64_t)P * kMaxPops);
  }
  // "<stem>_<q>" per population; efficacy tables also "<stem>_<q>_<b>"
  // (the bare form is block 0)
  int q = -1, b = 0;
  char stem[16] = {0};
  {
    const char* us = strchr(name, '_');
    if (!us || us - name >= (long)sizeof(stem)) return DPSNN_E_INVAL;
    memcpy(stem, name, (size_t)(us - name));
    const char* d = us + 1;
    if (strlen(d) == 1 && d[0] >= '0' && d[0] <= '3') {
      q = d[0] - '0';
    } else if (strlen(d) == 3 && d[0] >= '0' && d[0] <= '3' && d[1] == '_' && d[2] >= '0' &&
               d[2] <= '3') {
      q = d[0] - '0';
      b = d[2] - '0';
    } else if (!strcmp(stem, "pois")) {  // pois_thr_<q>
      if (!strncmp(d, "thr_", 4) && strlen(d) == 5 && d[4] >= '0' && d[4] <= '3') {
        q = d[4] - '0';
        if (q >= P) return DPSNN_E_INVAL;
        return put(T.pois[q], 4 * (int64_t)T.n_pois[q]);
      }
      return DPSNN_E_INVAL;
    } else {
      return DPSNN_E_INVAL;
    }
  }
  if (q >= P) return DPSNN_E_INVAL;
  const bool per_pop = !strcmp(stem, "jx64") || !strcmp(stem, "jx32") || !strcmp(stem, "jxfix");
  if (per_pop) {
    if (strlen(name) != strlen(stem) + 2) return DPSNN_E_INVAL;
    if (!strcmp(stem, "jx64")) return put(T.jx64[q].data(), 8 * (int64_t)kQuantN);
    if (!strcmp(stem, "jx32")) return put(T.jx32[q].data(), 4 * (int64_t)kQuantN);
    return put(T.jxfix[q].data(), 8 * (int64_t)kQuantN);
  }
  if (b >= T.tables(q)) return DPSNN_E_INVAL;
  if (!strcmp(stem, "wt64")) return put(T.wt64[q][b].data(), 8 * (int64_t)kQuantN);
  if (!strcmp(stem, "wt32")) return put(T.wt32[q][b].data(), 4 * (int64_t)kQuantN);
  if (!strcmp(stem, "wt16")) return put(T.wt16[q][b].data(), 2 * (int64_t)kQuantN);
  if (!strcmp(stem, "wq8")) return put(T.wq8[q][b].data(), (int64_t)kQuantN);
  return DPSNN_E_INVAL;
}

// Fixed-point efficacy table of (source pop, block) for the stored format
// (host copy used by the build-time range check).
std::vector<int64_t> fix_table(const dpsnn_params& p, const HostTables& T, int q, int b) {
  std::vector<int64_t> v(kQuantN);
  for (int i = 0; i < kQuantN; ++i) v[i] = stored_fix(p, T, q, b, i);
  return v;
}

const std::vector<double>& standard_normal_grid() { return normal_grid(); }

}  // namespace dpsnn
