/*
 * dpsnn_oracle.c -- plain CPU oracle for the DPSNN cortical-grid hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see dpsnn_oracle.h).  Written for clarity, not
 * speed: one neuron at a time, one synapse at a time, no blocking, no
 * fusion.  Every function names the passage of the paper it follows.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (see oracle/build.py).
 * Contraction of a*b+c into a fused multiply-add would change binary32
 * results, so the build forbids it.
 */
#include "dpsnn_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ZN 65536              /* entries of every efficacy quantile table */
#define MAX_POIS 16           /* Poisson count thresholds kept per pop    */
#define MAXP 4                /* populations per module                   */
#define MAX_ATTEMPTS 64       /* draws of a module inside open boundaries */

enum { RULE_OWN = 0, RULE_OTHERS = 1, RULE_ALL = 2 };

struct orc_net {
  orc_params p;
  uint64_t seed;
  uint32_t key[2];
  int32_t mode, store_rows, status;

  int64_t N;                  /* neurons                                  */
  int32_t M;                  /* modules                                  */
  int32_t P;                  /* populations per module                   */
  int32_t pop_lo[MAXP], pop_hi[MAXP];  /* module-local index ranges       */
  int32_t D;                  /* ring slots = d_max + 1                   */
  int32_t n_del;              /* distinct delays = d_max - d_min + 1      */
  int32_t n_arp[MAXP];        /* refractory steps                         */

  /* per-population neuron parameters (binary64 copies of the inputs) */
  double tau_m[MAXP], E[MAXP], V_th[MAXP], V_r[MAXP], tau_arp[MAXP];
  double alpha_c[MAXP], tau_c[MAXP], gc[MAXP], I_const[MAXP];
  double nu_ext[MAXP], Jx_mean[MAXP], Jx_sd[MAXP];

  double Pm[MAXP], Pc[MAXP], PVc[MAXP], Iterm[MAXP];
  float Pm32[MAXP], Pc32[MAXP], PVc32[MAXP], Iterm32[MAXP];
  float E32[MAXP], Vth32[MAXP], Vr32[MAXP], al32[MAXP];

  /* projections of a source population: blocks of synapses, in order */
  int32_t n_blk[MAXP];
  int32_t blk_n[MAXP][MAXP];  /* synapses                                 */
  int32_t blk_lo[MAXP][MAXP], blk_hi[MAXP][MAXP];  /* target range        */
  int32_t blk_rule[MAXP][MAXP];
  double blk_J[MAXP][MAXP], blk_sd[MAXP][MAXP];

  int32_t off_rule;           /* offsets of RULE_OTHERS or RULE_ALL        */
  int32_t open;               /* open boundaries: draws outside rejected   */
  int32_t n_off;              /* offsets in the table                      */
  int32_t* off_xy;            /* (ox, oy) per offset index                */
  uint32_t* off_thr;          /* n_off - 1 cumulative thresholds          */

  int32_t n_pois[MAXP];
  uint32_t pois_thr[MAXP][MAX_POIS];

  double* wt64[MAXP][MAXP];   /* efficacy tables by (source pop, block)    */
  float* wt32[MAXP][MAXP];
  uint16_t* wt16[MAXP][MAXP];
  int8_t* wq8[MAXP][MAXP];
  int64_t* wfix[MAXP][MAXP];  /* fixed-point efficacy for weight_dtype    */
  float s8[MAXP];             /* int8 scale (binary32), by source pop     */
  int64_t s8fix[MAXP];        /* the scale in fixed point                 */
  double* jx64[MAXP];
  float* jx32[MAXP];
  int64_t* jxfix[MAXP];

  int32_t* r_tgt;             /* stored rows (store_rows = 1)             */
  uint8_t* r_del;
  uint16_t* r_widx;
  uint8_t* r_blk;
  uint16_t* r_doff;

  int64_t t;
  float* V32;
  float* c32;
  double* V64;
  double* c64;
  int32_t* ref;
  int64_t* ring_fix;
  double* ring64;

  int32_t* sp_t;
  int32_t* sp_id;
  int64_t n_sp, cap_sp;
  uint32_t* rates;
  int64_t rate_bins_cap, rate_bins_used;

  int32_t* tmp_tgt;           /* unsorted draws inside orc_gen_row        */
  uint8_t* tmp_del;
  uint16_t* tmp_widx;
  uint8_t* tmp_blk;
  int32_t* row_tgt;           /* a regenerated row (store_rows = 0)       */
  uint8_t* row_del;
  uint16_t* row_widx;
  uint8_t* row_blk;
  uint16_t* row_doff;
  int64_t* spk_step;          /* ids that spiked in the current step      */

  /* plasticity (p.plastic): per synapse [s * K_out + j], oracle row order */
  int32_t L;                  /* table length = stdp_update_steps          */
  int32_t* syn_t;             /* last activation step, -1 = never          */
  float* syn_y32;
  float* syn_w32;
  double* syn_y64;
  double* syn_w64;
  int32_t* t_post;            /* last spike step of each neuron, -1 = none */
  float* Ep32;                /* A+ e^(-k dt / tau+), A- e^(-k dt / tau-),  */
  float* Em32;                /* e^(-k dt / tau_y), k < L                   */
  float* Dy32;
  double* Ep64;
  double* Em64;
  double* Dy64;
  float eta32, wmax32;
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 3): each round
 * multiplies counter words 0 and 2 by fixed odd constants, swaps the halves
 * of the products across the words and mixes in the key; the key is bumped
 * by the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)prod1;
    uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)prod0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(const orc_net* n, uint32_t w0, uint32_t w1, uint32_t w3,
                 uint32_t out[4]) {
  uint32_t ctr[4] = {w0, w1, 0u, w3};
  orc_philox4x32_10(ctr, n->key, out);
}

/* The same with counter word 2 = w2 (repeated draws of one synapse). */
static void draw2(const orc_net* n, uint32_t w0, uint32_t w1, uint32_t w2,
                  uint32_t w3, uint32_t out[4]) {
  uint32_t ctr[4] = {w0, w1, w2, w3};
  orc_philox4x32_10(ctr, n->key, out);
}

/* floor(u * range / 2^32): maps a uniform 32-bit word onto [0, range). */
static uint32_t scale_u32(uint32_t u, uint32_t range) {
  return (uint32_t)(((uint64_t)u * (uint64_t)range) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Gaussian efficacies (Sec. 2.2: efficacies drawn from a Gaussian of mean J
 * and standard deviation Delta J).  A draw is a 16-bit index into the
 * midpoint quantile table mu + sigma * Phi^-1((i + 1/2) / 65536). */
static double std_normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* For p > 1/2 the symmetry Phi^-1(p) = -Phi^-1(1 - p) keeps the search in
 * the lower tail, where erfc carries full relative precision. */
double orc_normal_quantile(double p) {
  if (p > 0.5) return -orc_normal_quantile(1.0 - p);
  double lo = -40.0, hi = 40.0;
  for (int it = 0; it < 4096; it++) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (std_normal_cdf(mid) < p)
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

static double* zgrid(void) {
  static double* z = NULL;
  if (!z) {
    double* tmp = (double*)malloc(sizeof(double) * ZN);
    if (!tmp) return NULL;
    for (int i = 0; i < ZN; i++)
      tmp[i] = orc_normal_quantile(((double)i + 0.5) / (double)ZN);
    z = tmp;
  }
  return z;
}

/* IEEE 754 binary16 from binary64, round to nearest, ties to even. */
uint16_t orc_f64_to_f16(double x) {
  uint16_t sign = signbit(x) ? 0x8000u : 0u;
  double a = fabs(x);
  if (isnan(x)) return (uint16_t)(sign | 0x7E00u);
  if (a >= 65520.0) return (uint16_t)(sign | 0x7C00u);
  if (a < ldexp(1.0, -14)) {
    double r = rint(a * ldexp(1.0, 24));          /* subnormal quanta */
    return (uint16_t)(sign | (uint16_t)r);
  }
  int e2;
  frexp(a, &e2);
  int ex = e2 - 1;                                /* a in [2^ex, 2^(ex+1)) */
  double r = rint(ldexp(a, 10 - ex));             /* in [1024, 2048] */
  if (r == 2048.0) {
    r = 1024.0;
    ex += 1;
  }
  if (ex + 15 >= 31) return (uint16_t)(sign | 0x7C00u);
  return (uint16_t)(sign | (uint16_t)((ex + 15) << 10) |
                    (uint16_t)(r - 1024.0));
}

double orc_f16_to_f64(uint16_t h) {
  int s = (h >> 15) & 1, e = (h >> 10) & 31, m = h & 1023;
  double v;
  if (e == 0)
    v = ldexp((double)m, -24);
  else if (e == 31)
    v = m ? NAN : INFINITY;
  else
    v = ldexp((double)(m + 1024), e - 25);
  return s ? -v : v;
}

/* ------------------------------------------------------------------------ */
static int pop_of(const orc_net* n, int64_t i) {
  int l = (int)(i % n->p.K), q = 0;
  while (q + 1 < n->P && l >= n->pop_hi[q]) q++;
  return q;
}

static void release(orc_net* n) {
  if (!n) return;
  for (int q = 0; q < MAXP; q++) {
    for (int b = 0; b < MAXP; b++) {
      free(n->wt64[q][b]); free(n->wt32[q][b]); free(n->wt16[q][b]);
      free(n->wq8[q][b]); free(n->wfix[q][b]);
    }
    free(n->jx64[q]); free(n->jx32[q]); free(n->jxfix[q]);
  }
  free(n->off_xy); free(n->off_thr);
  free(n->r_tgt); free(n->r_del); free(n->r_widx); free(n->r_blk); free(n->r_doff);
  free(n->V32); free(n->c32); free(n->V64); free(n->c64); free(n->ref);
  free(n->ring_fix); free(n->ring64);
  free(n->sp_t); free(n->sp_id); free(n->rates);
  free(n->tmp_tgt); free(n->tmp_del); free(n->tmp_widx); free(n->tmp_blk);
  free(n->row_tgt); free(n->row_del); free(n->row_widx); free(n->row_blk);
  free(n->row_doff);
  free(n->spk_step);
  free(n->syn_t); free(n->syn_y32); free(n->syn_w32); free(n->syn_y64); free(n->syn_w64);
  free(n->t_post);
  free(n->Ep32); free(n->Em32); free(n->Dy32); free(n->Ep64); free(n->Em64); free(n->Dy64);
  free(n);
}

void orc_free(orc_net* n) { release(n); }

static int valid(const orc_params* p) {
  if (p->grid_w < 1 || p->grid_h < 1 || p->K < 2 || p->K_out < 0) return 0;
  if (!(p->lambda > 0.0) || !(p->dt_ms > 0.0)) return 0;
  if (p->d_min < 1 || p->d_max < p->d_min || p->d_max > 255) return 0;
  if (p->weight_dtype < ORC_WF32 || p->weight_dtype > ORC_WI8) return 0;
  if (p->acc_bits != 32 && p->acc_bits != 64) return 0;
  if (p->q_frac_bits < 0 || p->q_frac_bits > (p->acc_bits == 32 ? 30 : 40))
    return 0;
  if (p->rate_bin_steps < 1) return 0;
  if ((int64_t)p->grid_w * p->grid_h * p->K > 2147483647LL) return 0;
  if (p->K_out > 65535) return 0;
  if (p->plastic != 0 && p->plastic != 1) return 0;
  if (p->plastic) {
    if (p->weight_dtype != ORC_WF32 || p->stdp_update_steps < 1) return 0;
    if (!(p->stdp_A_plus >= 0.0) || !(p->stdp_A_minus >= 0.0)) return 0;
    if (!(p->stdp_tau_plus > 0.0) || !(p->stdp_tau_minus > 0.0) || !(p->stdp_tau_y > 0.0))
      return 0;
    if (!isfinite(p->stdp_eta) || !(p->stdp_w_max > 0.0) || !isfinite(p->stdp_w_max)) return 0;
  }
  if (p->n_pops == 0) {
    if (!(p->frac_exc >= 0.0 && p->frac_exc <= 1.0)) return 0;
    for (int q = 0; q < 2; q++) {
      if (!(p->frac_local[q] >= 0.0 && p->frac_local[q] <= 1.0)) return 0;
      if (!(p->tau_m[q] > 0.0) || !(p->tau_c[q] > 0.0)) return 0;
      if (!(p->tau_arp[q] >= 0.0) || !(p->nu_ext_hz[q] >= 0.0)) return 0;
      if (!(p->J_sd[q] >= 0.0) || !(p->Jext_sd[q] >= 0.0)) return 0;
    }
    if (p->torus != 0 && p->torus != 1) return 0;
    return 1;
  }
  if (p->n_pops < 2 || p->n_pops > MAXP) return 0;
  int64_t sum = 0;
  for (int q = 0; q < p->n_pops; q++) {
    if (p->pop_size[q] < 1) return 0;
    sum += p->pop_size[q];
    if (!(p->p_tau_m[q] > 0.0) || !(p->p_tau_c[q] > 0.0)) return 0;
    if (!(p->p_tau_arp[q] >= 0.0) || !(p->p_nu_ext_hz[q] >= 0.0)) return 0;
    if (!(p->p_Jext_sd[q] >= 0.0)) return 0;
  }
  if (sum != p->K) return 0;
  for (int s = 0; s < p->n_pops; s++) {
    int64_t deg = 0;
    for (int t = 0; t < p->n_pops; t++) {
      if (p->n_syn[t][s] < 0 || !(p->J_sd_ts[t][s] >= 0.0)) return 0;
      deg += p->n_syn[t][s];
      /* a block into the own population needs a second neuron */
      if (t == s && p->n_syn[t][s] > 0 && p->pop_size[t] < 2) return 0;
    }
    if (deg != p->K_out) return 0;
  }
  return 1;
}

/* Projection blocks of every source population, the neuron ranges of the
 * populations and their parameters, from either parameter model. */
static void set_model(orc_net* n) {
  const orc_params* p = &n->p;
  if (p->n_pops == 0) {
    /* two populations; a source's first round(frac_local K_out) synapses
     * stay in its module, the rest go to other modules (Eq. 1); targets are
     * any neuron of the module */
    const int K_exc = (int)llround(p->frac_exc * p->K);
    n->P = 2;
    n->pop_lo[0] = 0; n->pop_hi[0] = K_exc;
    n->pop_lo[1] = K_exc; n->pop_hi[1] = p->K;
    for (int q = 0; q < 2; q++) {
      n->tau_m[q] = p->tau_m[q]; n->E[q] = p->E[q]; n->V_th[q] = p->V_th[q];
      n->V_r[q] = p->V_r[q]; n->tau_arp[q] = p->tau_arp[q];
      n->alpha_c[q] = p->alpha_c[q]; n->tau_c[q] = p->tau_c[q];
      n->gc[q] = p->gc[q]; n->I_const[q] = p->I_const[q];
      n->nu_ext[q] = p->nu_ext_hz[q]; n->Jx_mean[q] = p->Jext_mean[q];
      n->Jx_sd[q] = p->Jext_sd[q];
      const int nl = (int)llround(p->frac_local[q] * p->K_out);
      n->n_blk[q] = 0;
      int b = 0;
      if (nl > 0) {
        n->blk_n[q][b] = nl; n->blk_lo[q][b] = 0; n->blk_hi[q][b] = p->K;
        n->blk_rule[q][b] = RULE_OWN; b++;
      }
      if (p->K_out - nl > 0) {
        n->blk_n[q][b] = p->K_out - nl; n->blk_lo[q][b] = 0; n->blk_hi[q][b] = p->K;
        n->blk_rule[q][b] = RULE_OTHERS; b++;
      }
      for (int k = 0; k < 2; k++) {  /* both blocks use the source's table */
        n->blk_J[q][k] = p->J_mean[q];
        n->blk_sd[q][k] = p->J_sd[q];
      }
      n->n_blk[q] = b;
    }
    n->off_rule = RULE_OTHERS;
    n->open = p->torus ? 0 : 1;  /* torus = 0: the grid has edges */
    return;
  }
  n->P = p->n_pops;
  int lo = 0;
  for (int q = 0; q < n->P; q++) {
    n->pop_lo[q] = lo;
    lo += p->pop_size[q];
    n->pop_hi[q] = lo;
    n->tau_m[q] = p->p_tau_m[q]; n->E[q] = p->p_E[q]; n->V_th[q] = p->p_V_th[q];
    n->V_r[q] = p->p_V_r[q]; n->tau_arp[q] = p->p_tau_arp[q];
    n->alpha_c[q] = p->p_alpha_c[q]; n->tau_c[q] = p->p_tau_c[q];
    n->gc[q] = p->p_gc[q]; n->I_const[q] = p->p_I_const[q];
    n->nu_ext[q] = p->p_nu_ext_hz[q]; n->Jx_mean[q] = p->p_Jext_mean[q];
    n->Jx_sd[q] = p->p_Jext_sd[q];
  }
  for (int s = 0; s < n->P; s++) {
    int b = 0;
    for (int t = 0; t < n->P; t++) {
      if (p->n_syn[t][s] == 0) continue;
      n->blk_n[s][b] = p->n_syn[t][s];
      n->blk_lo[s][b] = n->pop_lo[t];
      n->blk_hi[s][b] = n->pop_hi[t];
      n->blk_rule[s][b] = p->pop_exc[s] ? RULE_ALL : RULE_OWN;
      n->blk_J[s][b] = p->J_mean_ts[t][s];
      n->blk_sd[s][b] = p->J_sd_ts[t][s];
      b++;
    }
    n->n_blk[s] = b;
  }
  n->off_rule = RULE_ALL;
  n->open = p->open_boundary ? 1 : 0;
}

/* Host tables: propagators, Poisson thresholds, module-offset distribution,
 * efficacy quantile tables.  All computed in binary64, rounded once. */
/* Efficacy tables of a source population: one per block, at least one. */
static int n_tab(const orc_net* n, int q) { return n->n_blk[q] > 0 ? n->n_blk[q] : 1; }

static int build_tables(orc_net* n) {
  const orc_params* p = &n->p;
  const double twoQ = ldexp(1.0, p->q_frac_bits);

  for (int q = 0; q < n->P; q++) {
    /* Eq. 2 between inputs is linear: V relaxes to E with tau_m while the
     * fatigue c decays with tau_c and pulls V down at rate g_c c / C_m.
     * Over one step dt the exact solution is
     *   c' = c Pc,
     *   V' = E + (V - E) Pm - c (g_c/C_m) (Pc - Pm) / (1/tau_m - 1/tau_c)
     *        + I tau_m (1 - Pm)            (constant drive I, tests only).
     * Inhibitory neurons carry no c (Sec. 2.2): their gc is 0. */
    double a = 1.0 / n->tau_m[q], b = 1.0 / n->tau_c[q];
    n->Pm[q] = exp(-p->dt_ms / n->tau_m[q]);
    n->Pc[q] = exp(-p->dt_ms / n->tau_c[q]);
    if (a != b)
      n->PVc[q] = n->gc[q] * (n->Pc[q] - n->Pm[q]) / (a - b);
    else
      n->PVc[q] = n->gc[q] * p->dt_ms * n->Pm[q];
    n->Iterm[q] = n->I_const[q] * n->tau_m[q] * (1.0 - n->Pm[q]);
    n->Pm32[q] = (float)n->Pm[q];
    n->Pc32[q] = (float)n->Pc[q];
    n->PVc32[q] = (float)n->PVc[q];
    n->Iterm32[q] = (float)n->Iterm[q];
    n->E32[q] = (float)n->E[q];
    n->Vth32[q] = (float)n->V_th[q];
    n->Vr32[q] = (float)n->V_r[q];
    n->al32[q] = (float)n->alpha_c[q];
    n->n_arp[q] = (int32_t)llround(n->tau_arp[q] / p->dt_ms);

    /* External drive (Sec. 2.2 and Table S1): a Poisson process of total
     * rate nu_ext; per step the count k is Poisson with mean nu_ext dt.
     * k = number of thresholds floor(F(j) 2^32) not above the draw. */
    double mean = n->nu_ext[q] * p->dt_ms * 1e-3;
    n->n_pois[q] = 0;
    if (mean > 0.0) {
      double term = exp(-mean), F = term;
      for (int j = 0; j < MAX_POIS; j++) {
        if (j > 0) {
          term = term * mean / (double)j;
          F = F + term;
        }
        double v = floor(F * 4294967296.0);
        if (v >= 4294967295.0) break;
        n->pois_thr[q][n->n_pois[q]++] = (uint32_t)v;
      }
    }
  }

  /* Eq. 1: a target module at distance d is chosen with probability
   * proportional to exp(-d / lambda).
   *  - RULE_OTHERS (two-population model, torus): among all other modules;
   *    offsets (ox, oy) in [0,W) x [0,H) row-major without (0,0), d the
   *    Euclidean length of the shortest periodic image.
   *  - RULE_ALL on the torus: the same offsets with (0,0) (d = 0) first.
   *  - open boundaries: plane offsets (dx, dy) in [-(W-1), W-1] x
   *    [-(H-1), H-1] row-major, d = |(dx, dy)|, without (0,0) for
   *    RULE_OTHERS; a draw that leaves the grid is repeated, so that each
   *    source draws from exp(-d/l) restricted to the modules that exist. */
  const int W = p->grid_w, H = p->grid_h;
  int cnt_off;
  if (n->off_rule == RULE_OTHERS)
    cnt_off = n->M - 1;
  else if (!n->open)
    cnt_off = n->M;
  else
    cnt_off = (2 * W - 1) * (2 * H - 1);
  if (n->off_rule == RULE_OTHERS && n->open) cnt_off = (2 * W - 1) * (2 * H - 1) - 1;
  n->n_off = cnt_off;
  if (n->n_off > 0) {
    double* wgt = (double*)malloc(sizeof(double) * n->n_off);
    n->off_xy = (int32_t*)malloc(sizeof(int32_t) * 2 * n->n_off);
    n->off_thr = (uint32_t*)malloc(sizeof(uint32_t) * (n->n_off > 1 ? n->n_off - 1 : 1));
    if (!wgt || !n->off_xy || !n->off_thr) { free(wgt); return ORC_E_NOMEM; }
    int k = 0;
    double Z = 0.0;
    if (!n->open) {
      for (int oy = 0; oy < H; oy++)
        for (int ox = 0; ox < W; ox++) {
          if (ox == 0 && oy == 0 && n->off_rule == RULE_OTHERS) continue;
          int dx = ox < W - ox ? ox : W - ox;
          int dy = oy < H - oy ? oy : H - oy;
          double d = sqrt((double)(dx * dx + dy * dy));
          wgt[k] = exp(-d / p->lambda);
          n->off_xy[2 * k] = ox;
          n->off_xy[2 * k + 1] = oy;
          Z += wgt[k];
          k++;
        }
    } else {
      for (int dy = -(H - 1); dy <= H - 1; dy++)
        for (int dx = -(W - 1); dx <= W - 1; dx++) {
          if (dx == 0 && dy == 0 && n->off_rule == RULE_OTHERS) continue;
          double d = sqrt((double)(dx * dx + dy * dy));
          wgt[k] = exp(-d / p->lambda);
          n->off_xy[2 * k] = dx;
          n->off_xy[2 * k + 1] = dy;
          Z += wgt[k];
          k++;
        }
    }
    double cum = 0.0;
    for (k = 0; k + 1 < n->n_off; k++) {
      cum += wgt[k];
      double v = floor(cum / Z * 4294967296.0);
      n->off_thr[k] = v >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)v;
    }
    free(wgt);
  }

  /* Efficacy tables: recurrent by (source pop, block), external by target
   * pop.  int8: symmetric codes q = rint(w / s) with one scale per source
   * pop, s = (largest |w| of its tables) / 127 in binary32. */
  double* z = zgrid();
  if (!z) return ORC_E_NOMEM;
  for (int q = 0; q < n->P; q++) {
    double amax = 0.0;
    for (int b = 0; b < n_tab(n, q); b++) {
      n->wt64[q][b] = (double*)malloc(sizeof(double) * ZN);
      n->wt32[q][b] = (float*)malloc(sizeof(float) * ZN);
      n->wt16[q][b] = (uint16_t*)malloc(sizeof(uint16_t) * ZN);
      n->wq8[q][b] = (int8_t*)malloc(ZN);
      n->wfix[q][b] = (int64_t*)malloc(sizeof(int64_t) * ZN);
      if (!n->wt64[q][b] || !n->wt32[q][b] || !n->wt16[q][b] || !n->wq8[q][b] ||
          !n->wfix[q][b])
        return ORC_E_NOMEM;
      for (int i = 0; i < ZN; i++) {
        n->wt64[q][b][i] = n->blk_J[q][b] + n->blk_sd[q][b] * z[i];
        n->wt32[q][b][i] = (float)n->wt64[q][b][i];
        n->wt16[q][b][i] = orc_f64_to_f16(n->wt64[q][b][i]);
        if (fabs(n->wt64[q][b][i]) > amax) amax = fabs(n->wt64[q][b][i]);
      }
    }
    n->s8[q] = (float)(amax > 0.0 ? amax / 127.0 : 1.0);
    n->s8fix[q] = (int64_t)rint((double)n->s8[q] * twoQ);
    for (int b = 0; b < n_tab(n, q); b++)
      for (int i = 0; i < ZN; i++) {
        double c = rint(n->wt64[q][b][i] / (double)n->s8[q]);
        if (c > 127.0) c = 127.0;
        if (c < -127.0) c = -127.0;
        n->wq8[q][b][i] = (int8_t)c;
        if (p->weight_dtype == ORC_WF32)
          n->wfix[q][b][i] = (int64_t)rint((double)n->wt32[q][b][i] * twoQ);
        else if (p->weight_dtype == ORC_WF16)
          n->wfix[q][b][i] = (int64_t)rint(orc_f16_to_f64(n->wt16[q][b][i]) * twoQ);
        else
          n->wfix[q][b][i] = (int64_t)n->wq8[q][b][i] * n->s8fix[q];
      }
    n->jx64[q] = (double*)malloc(sizeof(double) * ZN);
    n->jx32[q] = (float*)malloc(sizeof(float) * ZN);
    n->jxfix[q] = (int64_t*)malloc(sizeof(int64_t) * ZN);
    if (!n->jx64[q] || !n->jx32[q] || !n->jxfix[q]) return ORC_E_NOMEM;
    for (int i = 0; i < ZN; i++) {
      n->jx64[q][i] = n->Jx_mean[q] + n->Jx_sd[q] * z[i];
      n->jx32[q][i] = (float)n->jx64[q][i];
      n->jxfix[q][i] = (int64_t)rint((double)n->jx32[q][i] * twoQ);
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One row of the connectivity of source s (Sec. 2.2, Eq. 1).  Synapse j
 * belongs to block b of the source's population (blocks in order, counts
 * n_blk); it targets a uniform neuron of the block's target range in a
 * module chosen by the block's rule:
 *   RULE_OWN    the source's own module; neuron from word 0;
 *   RULE_OTHERS another module by Eq. 1 (offsets without (0,0); with open
 *               boundaries a draw outside the grid is repeated as below);
 *   RULE_ALL    any module by Eq. 1 from d = 0; with open boundaries a draw
 *               outside the grid is repeated with counter word 2 = attempt
 *               (at most MAX_ATTEMPTS, then the own module);
 * module from word 0 and neuron from word 1 of the draw (s, j, attempt,
 * SYN).  In the own module the source itself is skipped (no autapse):
 * r uniform on [0, size-1) and r + (r >= own offset).  Delay uniform on
 * [d_min, d_max] from word 2; efficacy index = top 16 bits of word 3 of the
 * accepted draw.  Then a stable sort by delay. */
static void draw_synapse(const orc_net* n, int64_t s, int j, int32_t* target,
                         uint8_t* dly, uint16_t* wi, uint8_t* bk) {
  const orc_params* p = &n->p;
  const int K = p->K, W = p->grid_w, H = p->grid_h;
  const int ps = pop_of(n, s);
  const int32_t ms = (int32_t)(s / K), ls = (int32_t)(s % K);
  const int xs = ms % W, ys = ms / W;
  int b = 0, first = 0;
  while (b + 1 < n->n_blk[ps] && j >= first + n->blk_n[ps][b]) {
    first += n->blk_n[ps][b];
    b++;
  }
  const int lo = n->blk_lo[ps][b], size = n->blk_hi[ps][b] - lo;
  const int rule = n->blk_rule[ps][b];
  uint32_t u[4];
  int32_t mt = ms;
  uint32_t nu;                 /* the word that picks the neuron          */
  if (rule == RULE_OWN) {
    draw(n, (uint32_t)s, (uint32_t)j, ORC_TAG_SYN, u);
    nu = u[0];
  } else {
    int att = 0;
    for (;;) {
      draw2(n, (uint32_t)s, (uint32_t)j, (uint32_t)att, ORC_TAG_SYN, u);
      /* offset index = number of cumulative thresholds <= u[0] */
      int a = 0, z = n->n_off - 1;
      while (a < z) {
        int mid = (a + z) / 2;
        if (n->off_thr[mid] <= u[0])
          a = mid + 1;
        else
          z = mid;
      }
      int xt, yt;
      if (!n->open) {
        xt = (xs + n->off_xy[2 * a]) % W;
        yt = (ys + n->off_xy[2 * a + 1]) % H;
      } else {
        xt = xs + n->off_xy[2 * a];
        yt = ys + n->off_xy[2 * a + 1];
      }
      if (xt >= 0 && xt < W && yt >= 0 && yt < H) {
        mt = yt * W + xt;
        break;
      }
      if (++att == MAX_ATTEMPTS) {
        mt = ms;
        break;
      }
    }
    nu = u[1];
  }
  uint32_t r;
  if (mt == ms && ls >= lo && ls < lo + size) {
    r = scale_u32(nu, (uint32_t)(size - 1));
    r += r >= (uint32_t)(ls - lo) ? 1u : 0u;
  } else {
    r = scale_u32(nu, (uint32_t)size);
  }
  *target = mt * K + lo + (int32_t)r;
  *dly = (uint8_t)(p->d_min + (int)scale_u32(u[2], (uint32_t)n->n_del));
  *wi = (uint16_t)(u[3] >> 16);
  *bk = (uint8_t)b;
}

int32_t orc_gen_row_blocks(const orc_net* n, int64_t s, int32_t* tgt, uint8_t* delay,
                           uint16_t* widx, uint16_t* doff, uint8_t* blk) {
  const orc_params* p = &n->p;
  if (s < 0 || s >= n->N) return ORC_E_INVAL;
  const int Ko = p->K_out;
  int32_t* t0 = n->tmp_tgt;
  uint8_t* d0 = n->tmp_del;
  uint16_t* w0 = n->tmp_widx;
  uint8_t* b0 = n->tmp_blk;
  for (int j = 0; j < Ko; j++) draw_synapse(n, s, j, &t0[j], &d0[j], &w0[j], &b0[j]);
  /* stable counting sort by delay */
  int32_t cnt[256];
  memset(cnt, 0, sizeof(cnt));
  for (int j = 0; j < Ko; j++) cnt[d0[j] - p->d_min]++;
  int32_t pos[257];
  pos[0] = 0;
  for (int k = 0; k < n->n_del; k++) pos[k + 1] = pos[k] + cnt[k];
  for (int k = 0; k <= n->n_del; k++) doff[k] = (uint16_t)pos[k];
  for (int j = 0; j < Ko; j++) {
    int k = d0[j] - p->d_min;
    int at = pos[k]++;
    tgt[at] = t0[j];
    delay[at] = d0[j];
    widx[at] = w0[j];
    if (blk) blk[at] = b0[j];
  }
  return ORC_OK;
}

int32_t orc_gen_row(const orc_net* n, int64_t s, int32_t* tgt, uint8_t* delay,
                    uint16_t* widx, uint16_t* doff) {
  return orc_gen_row_blocks(n, s, tgt, delay, widx, doff, NULL);
}

int32_t orc_n_pops(const orc_net* n) { return n->P; }

/* ------------------------------------------------------------------------ */
/* External Poisson input (Sec. 2.1: external synapses are not stored;
 * counts and efficacies are generated on the fly).  The
 * count of neuron i at step t comes from word (i mod 4) of the draw
 * (i / 4, t, EXT).  Efficacy e of the neuron uses 16 bits of the draw
 * (i / 4, t, EXTJ | (e / 2) << 8): word (i mod 4), high half for even e,
 * low half for odd e. */
int32_t orc_ext_input(const orc_net* n, int64_t i, int64_t t, int64_t* fix_sum,
                      double* f64_sum) {
  if (i < 0 || i >= n->N || t < 0) return ORC_E_INVAL;
  const int q = pop_of(n, i);
  uint32_t u[4];
  draw(n, (uint32_t)(i >> 2), (uint32_t)t, ORC_TAG_EXT, u);
  uint32_t x = u[i & 3];
  int32_t k = 0;
  for (int j = 0; j < n->n_pois[q]; j++)
    if (x >= n->pois_thr[q][j]) k++;
  int64_t fs = 0;
  double ds = 0.0;
  uint32_t v[4];
  for (int e = 0; e < k; e++) {
    if ((e & 1) == 0)
      draw(n, (uint32_t)(i >> 2), (uint32_t)t,
           ORC_TAG_EXTJ | ((uint32_t)(e >> 1) << 8), v);
    uint32_t word = v[i & 3];
    uint32_t idx = (e & 1) ? (word & 0xFFFFu) : (word >> 16);
    fs += n->jxfix[q][idx];
    ds += n->jx64[q][idx];
  }
  if (fix_sum) *fix_sum = fs;
  if (f64_sum) *f64_sum = ds;
  return k;
}

/* ------------------------------------------------------------------------ */
orc_net* orc_create(const orc_params* p, uint64_t seed, int32_t mode,
                    int32_t store_rows, int32_t* err) {
  int32_t dummy;
  if (!err) err = &dummy;
  *err = ORC_E_INVAL;
  if (!p || !valid(p) || (mode != ORC_MIRROR32 && mode != ORC_EXACT64))
    return NULL;
  orc_net* n = (orc_net*)calloc(1, sizeof(orc_net));
  if (!n) { *err = ORC_E_NOMEM; return NULL; }
  n->p = *p;
  n->seed = seed;
  n->key[0] = (uint32_t)seed;
  n->key[1] = (uint32_t)(seed >> 32);
  n->mode = mode;
  n->store_rows = store_rows;
  n->M = p->grid_w * p->grid_h;
  n->N = (int64_t)n->M * p->K;
  n->D = p->d_max + 1;
  n->n_del = p->d_max - p->d_min + 1;
  set_model(n);
  /* a single module has nowhere else to send synapses to other modules */
  for (int q = 0; q < n->P; q++)
    for (int b = 0; b < n->n_blk[q]; b++)
      if (n->M == 1 && n->blk_rule[q][b] == RULE_OTHERS) {
        release(n);
        return NULL;
      }
  int rc = build_tables(n);
  if (rc != ORC_OK) { *err = rc; release(n); return NULL; }

  const int64_t N = n->N, Ko = p->K_out;
  n->tmp_tgt = (int32_t*)malloc(sizeof(int32_t) * (Ko ? Ko : 1));
  n->tmp_del = (uint8_t*)malloc(Ko ? Ko : 1);
  n->tmp_widx = (uint16_t*)malloc(sizeof(uint16_t) * (Ko ? Ko : 1));
  n->tmp_blk = (uint8_t*)malloc(Ko ? Ko : 1);
  n->row_blk = (uint8_t*)malloc(Ko ? Ko : 1);
  n->row_tgt = (int32_t*)malloc(sizeof(int32_t) * (Ko ? Ko : 1));
  n->row_del = (uint8_t*)malloc(Ko ? Ko : 1);
  n->row_widx = (uint16_t*)malloc(sizeof(uint16_t) * (Ko ? Ko : 1));
  n->row_doff = (uint16_t*)malloc(sizeof(uint16_t) * (n->n_del + 1));
  n->spk_step = (int64_t*)malloc(sizeof(int64_t) * N);
  n->ref = (int32_t*)calloc(N, sizeof(int32_t));
  if (!n->tmp_tgt || !n->tmp_del || !n->tmp_widx || !n->tmp_blk || !n->row_blk || !n->row_tgt ||
      !n->row_del || !n->row_widx || !n->row_doff || !n->spk_step || !n->ref) {
    *err = ORC_E_NOMEM; release(n); return NULL;
  }
  if (mode == ORC_MIRROR32) {
    n->V32 = (float*)malloc(sizeof(float) * N);
    n->c32 = (float*)calloc(N, sizeof(float));
    n->ring_fix = (int64_t*)calloc((size_t)n->D * N, sizeof(int64_t));
    if (!n->V32 || !n->c32 || !n->ring_fix) {
      *err = ORC_E_NOMEM; release(n); return NULL;
    }
  } else {
    n->V64 = (double*)malloc(sizeof(double) * N);
    n->c64 = (double*)calloc(N, sizeof(double));
    n->ring64 = (double*)calloc((size_t)n->D * N, sizeof(double));
    if (!n->V64 || !n->c64 || !n->ring64) {
      *err = ORC_E_NOMEM; release(n); return NULL;
    }
  }
  /* Initial condition (not given in the paper): V uniform on [E, V_th)
   * from the draw (i, 0, INIT), computed in binary32 for both precisions
   * so that they start from the same state; c = 0; not refractory. */
  for (int64_t i = 0; i < N; i++) {
    int q = pop_of(n, i);
    uint32_t u[4];
    draw(n, (uint32_t)i, 0u, ORC_TAG_INIT, u);
    float f = (float)(u[0] >> 8) * 0x1p-24f;
    float v0 = n->E32[q] + (n->Vth32[q] - n->E32[q]) * f;
    if (mode == ORC_MIRROR32)
      n->V32[i] = v0;
    else
      n->V64[i] = (double)v0;
  }
  if (store_rows && Ko > 0) {
    n->r_tgt = (int32_t*)malloc(sizeof(int32_t) * N * Ko);
    n->r_del = (uint8_t*)malloc((size_t)N * Ko);
    n->r_widx = (uint16_t*)malloc(sizeof(uint16_t) * N * Ko);
    n->r_blk = (uint8_t*)malloc((size_t)N * Ko);
    n->r_doff = (uint16_t*)malloc(sizeof(uint16_t) * N * (n->n_del + 1));
    if (!n->r_tgt || !n->r_del || !n->r_widx || !n->r_blk || !n->r_doff) {
      *err = ORC_E_NOMEM; release(n); return NULL;
    }
    for (int64_t s = 0; s < N; s++)
      orc_gen_row_blocks(n, s, n->r_tgt + s * Ko, n->r_del + s * Ko,
                         n->r_widx + s * Ko, n->r_doff + s * (n->n_del + 1),
                         n->r_blk + s * Ko);
  }
  if (p->plastic) {
    const int32_t L = p->stdp_update_steps;
    const size_t ns = (size_t)N * (size_t)(Ko ? Ko : 1);
    n->L = L;
    n->syn_t = (int32_t*)malloc(sizeof(int32_t) * ns);
    n->t_post = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    n->Ep32 = (float*)malloc(sizeof(float) * L);
    n->Em32 = (float*)malloc(sizeof(float) * L);
    n->Dy32 = (float*)malloc(sizeof(float) * L);
    n->Ep64 = (double*)malloc(sizeof(double) * L);
    n->Em64 = (double*)malloc(sizeof(double) * L);
    n->Dy64 = (double*)malloc(sizeof(double) * L);
    if (mode == ORC_MIRROR32) {
      n->syn_y32 = (float*)calloc(ns, sizeof(float));
      n->syn_w32 = (float*)malloc(sizeof(float) * ns);
    } else {
      n->syn_y64 = (double*)calloc(ns, sizeof(double));
      n->syn_w64 = (double*)malloc(sizeof(double) * ns);
    }
    if (!n->syn_t || !n->t_post || !n->Ep32 || !n->Em32 || !n->Dy32 || !n->Ep64 ||
        !n->Em64 || !n->Dy64 || (mode == ORC_MIRROR32 ? (!n->syn_y32 || !n->syn_w32)
                                                     : (!n->syn_y64 || !n->syn_w64))) {
      *err = ORC_E_NOMEM; release(n); return NULL;
    }
    for (int32_t k = 0; k < L; k++) {
      const double x = (double)k * p->dt_ms;
      n->Ep64[k] = p->stdp_A_plus * exp(-x / p->stdp_tau_plus);
      n->Em64[k] = p->stdp_A_minus * exp(-x / p->stdp_tau_minus);
      n->Dy64[k] = exp(-x / p->stdp_tau_y);
      n->Ep32[k] = (float)n->Ep64[k];
      n->Em32[k] = (float)n->Em64[k];
      n->Dy32[k] = (float)n->Dy64[k];
    }
    n->eta32 = (float)p->stdp_eta;
    n->wmax32 = (float)p->stdp_w_max;
    for (int64_t i = 0; i < N; i++) n->t_post[i] = -1;
    /* initial efficacies: the table values of the stored format */
    for (int64_t s0 = 0; s0 < N; s0++) {
      const uint16_t* wi;
      const uint8_t* bk;
      if (store_rows) {
        wi = n->r_widx + s0 * Ko;
        bk = n->r_blk + s0 * Ko;
      } else {
        orc_gen_row_blocks(n, s0, n->row_tgt, n->row_del, n->row_widx, n->row_doff,
                           n->row_blk);
        wi = n->row_widx;
        bk = n->row_blk;
      }
      const int q = pop_of(n, s0);
      for (int64_t j = 0; j < Ko; j++) {
        const size_t at = (size_t)s0 * (size_t)Ko + (size_t)j;
        n->syn_t[at] = -1;
        if (mode == ORC_MIRROR32)
          n->syn_w32[at] = n->wt32[q][bk[j]][wi[j]];
        else
          n->syn_w64[at] = n->wt64[q][bk[j]][wi[j]];
      }
    }
  }
  *err = ORC_OK;
  return n;
}

int64_t orc_n_neurons(const orc_net* n) { return n->N; }
int32_t orc_n_slots(const orc_net* n) { return n->D; }
int64_t orc_time(const orc_net* n) { return n->t; }
int32_t orc_status(const orc_net* n) { return n->status; }

static int record_spike(orc_net* n, int64_t t, int64_t i) {
  if (n->n_sp == n->cap_sp) {
    int64_t cap = n->cap_sp ? 2 * n->cap_sp : 4096;
    int32_t* a = (int32_t*)realloc(n->sp_t, sizeof(int32_t) * cap);
    if (!a) return ORC_E_NOMEM;
    n->sp_t = a;
    int32_t* b = (int32_t*)realloc(n->sp_id, sizeof(int32_t) * cap);
    if (!b) return ORC_E_NOMEM;
    n->sp_id = b;
    n->cap_sp = cap;
  }
  n->sp_t[n->n_sp] = (int32_t)t;
  n->sp_id[n->n_sp] = (int32_t)i;
  n->n_sp++;
  /* 5 ms population rates (Sec. 2.3): counts per (bin, module, pop). */
  int64_t bin = t / n->p.rate_bin_steps;
  if (bin >= n->rate_bins_cap) {
    int64_t cap = n->rate_bins_cap ? n->rate_bins_cap : 64;
    while (cap <= bin) cap *= 2;
    uint32_t* r = (uint32_t*)realloc(n->rates, sizeof(uint32_t) * cap * n->M * n->P);
    if (!r) return ORC_E_NOMEM;
    memset(r + n->rate_bins_cap * n->M * n->P, 0,
           sizeof(uint32_t) * (cap - n->rate_bins_cap) * n->M * n->P);
    n->rates = r;
    n->rate_bins_cap = cap;
  }
  if (bin + 1 > n->rate_bins_used) n->rate_bins_used = bin + 1;
  n->rates[(bin * n->M + i / n->p.K) * n->P + pop_of(n, i)] += 1;
  return ORC_OK;
}

/* Eq. 2 over one step for neuron i with input sum already in mV. */
static int update_neuron32(orc_net* n, int64_t i, float dv) {
  const int q = pop_of(n, i);
  float V = n->V32[i], c = n->c32[i];
  int spiked = 0;
  if (n->ref[i] > 0) {
    /* refractory: V held at the reset value, inputs discarded, c decays */
    n->ref[i] -= 1;
    c = c * n->Pc32[q];
  } else {
    float v = V - n->E32[q];
    v = v * n->Pm32[q];
    v = n->E32[q] + v;
    float cv = c * n->PVc32[q];
    v = v - cv;
    v = v + n->Iterm32[q];
    v = v + dv;
    c = c * n->Pc32[q];
    /* a spike when V exceeds the threshold (Sec. 2.2): reset, refractory
     * period, fatigue incremented by alpha_c */
    if (v > n->Vth32[q]) {
      spiked = 1;
      v = n->Vr32[q];
      c = c + n->al32[q];
      n->ref[i] = n->n_arp[q];
    }
    V = v;
  }
  n->V32[i] = V;
  n->c32[i] = c;
  return spiked;
}

static int update_neuron64(orc_net* n, int64_t i, double dv) {
  const int q = pop_of(n, i);
  double V = n->V64[i], c = n->c64[i];
  int spiked = 0;
  if (n->ref[i] > 0) {
    n->ref[i] -= 1;
    c = c * n->Pc[q];
  } else {
    double v = V - n->E[q];
    v = v * n->Pm[q];
    v = n->E[q] + v;
    double cv = c * n->PVc[q];
    v = v - cv;
    v = v + n->Iterm[q];
    v = v + dv;
    c = c * n->Pc[q];
    if (v > n->V_th[q]) {
      spiked = 1;
      v = n->V_r[q];
      c = c + n->alpha_c[q];
      n->ref[i] = n->n_arp[q];
    }
    V = v;
  }
  n->V64[i] = V;
  n->c64[i] = c;
  return spiked;
}

/* Is population q excitatory (its synapses are the plastic ones)? */
static int pop_is_exc(const orc_net* n, int q) {
  return n->p.n_pops == 0 ? q == 0 : n->p.pop_exc[q] != 0;
}

/* Plasticity event of synapse `at` activated at step ta (Sec. 2.1: the
 * synapse notes its previous activation; contributions through a low-pass
 * filter), target's last spike tp; the reading is in the header. */
static void stdp_event(orc_net* n, size_t at, int64_t ta, int64_t tp) {
  const int64_t L = n->L;
  const int64_t tl = n->syn_t[at];
  if (n->mode == ORC_MIRROR32) {
    float y = n->syn_y32[at];
    y = (tl >= 0 && ta - tl < L) ? y * n->Dy32[ta - tl] : 0.0f;
    if (tl >= 0 && tp > tl && tp - tl < L && ta - tp < L)
      y = y + n->Ep32[tp - tl] * n->Dy32[ta - tp];
    if (tp >= 0 && ta - tp < L) y = y - n->Em32[ta - tp];
    n->syn_y32[at] = y;
  } else {
    double y = n->syn_y64[at];
    y = (tl >= 0 && ta - tl < L) ? y * n->Dy64[ta - tl] : 0.0;
    if (tl >= 0 && tp > tl && tp - tl < L && ta - tp < L)
      y = y + n->Ep64[tp - tl] * n->Dy64[ta - tp];
    if (tp >= 0 && ta - tp < L) y = y - n->Em64[ta - tp];
    n->syn_y64[at] = y;
  }
  n->syn_t[at] = (int32_t)ta;
}

/* Delivery with plastic efficacies: each synapse's own efficacy (in fixed
 * point rint(w 2^Q) in MIRROR32 mode); the synapses of excitatory sources
 * register the activation first. */
static void deliver_plastic(orc_net* n, int64_t s, int64_t t, int q, const int32_t* tgt,
                            const uint8_t* del) {
  const int Ko = n->p.K_out;
  const double twoQ = ldexp(1.0, n->p.q_frac_bits);
  const int plastic = pop_is_exc(n, q);
  for (int j = 0; j < Ko; j++) {
    const size_t si = (size_t)s * (size_t)Ko + (size_t)j;
    if (plastic) stdp_event(n, si, t, n->t_post[tgt[j]]);
    int64_t slot = (t + del[j]) % n->D;
    size_t at = (size_t)slot * (size_t)n->N + (size_t)tgt[j];
    if (n->mode == ORC_MIRROR32)
      n->ring_fix[at] += (int64_t)rint((double)n->syn_w32[si] * twoQ);
    else
      n->ring64[at] += n->syn_w64[si];
  }
}

/* Periodic efficacy update at step T (Sec. 2.1: every plastic synapse
 * applies its integrated signal): w <- clip(w + eta y(T), 0, w_max), y <- 0. */
static void stdp_update(orc_net* n, int64_t T) {
  const int64_t Ko = n->p.K_out, L = n->L;
  for (int64_t s = 0; s < n->N; s++) {
    if (!pop_is_exc(n, pop_of(n, s))) continue;
    for (int64_t j = 0; j < Ko; j++) {
      const size_t at = (size_t)s * (size_t)Ko + (size_t)j;
      const int64_t tl = n->syn_t[at];
      const int live = tl >= 0 && T - tl < L;
      if (n->mode == ORC_MIRROR32) {
        if (live) {
          float w = n->syn_w32[at] + n->eta32 * (n->syn_y32[at] * n->Dy32[T - tl]);
          w = w < 0.0f ? 0.0f : (w > n->wmax32 ? n->wmax32 : w);
          n->syn_w32[at] = w;
        }
        n->syn_y32[at] = 0.0f;
      } else {
        if (live) {
          double w = n->syn_w64[at] + n->p.stdp_eta * (n->syn_y64[at] * n->Dy64[T - tl]);
          w = w < 0.0 ? 0.0 : (w > n->p.stdp_w_max ? n->p.stdp_w_max : w);
          n->syn_w64[at] = w;
        }
        n->syn_y64[at] = 0.0;
      }
    }
  }
}

int32_t orc_plasticity(const orc_net* n, int64_t s, int32_t* t_act, double* y, double* w) {
  if (!n->p.plastic || s < 0 || s >= n->N) return ORC_E_INVAL;
  const int64_t Ko = n->p.K_out;
  for (int64_t j = 0; j < Ko; j++) {
    const size_t at = (size_t)s * (size_t)Ko + (size_t)j;
    if (t_act) t_act[j] = n->syn_t[at];
    if (y) y[j] = n->mode == ORC_MIRROR32 ? (double)n->syn_y32[at] : n->syn_y64[at];
    if (w) w[j] = n->mode == ORC_MIRROR32 ? (double)n->syn_w32[at] : n->syn_w64[at];
  }
  return ORC_OK;
}

/* Delivery of one spike (Sec. 2.1.1, steps 3-4): every synapse of the
 * source adds its efficacy to the input queue of its target, in the slot of
 * the step at which the delay expires. */
static void deliver(orc_net* n, int64_t s, int64_t t) {
  const orc_params* p = &n->p;
  const int Ko = p->K_out;
  if (Ko == 0) return;
  const int32_t* tgt;
  const uint8_t* del;
  const uint16_t* widx;
  const uint8_t* blk;
  if (n->store_rows) {
    tgt = n->r_tgt + s * Ko;
    del = n->r_del + s * Ko;
    widx = n->r_widx + s * Ko;
    blk = n->r_blk + s * Ko;
  } else {
    orc_gen_row_blocks(n, s, n->row_tgt, n->row_del, n->row_widx, n->row_doff,
                       n->row_blk);
    tgt = n->row_tgt;
    del = n->row_del;
    widx = n->row_widx;
    blk = n->row_blk;
  }
  const int q = pop_of(n, s);
  if (n->p.plastic) {
    deliver_plastic(n, s, t, q, tgt, del);
    return;
  }
  for (int j = 0; j < Ko; j++) {
    int64_t slot = (t + del[j]) % n->D;
    size_t at = (size_t)slot * (size_t)n->N + (size_t)tgt[j];
    if (n->mode == ORC_MIRROR32)
      n->ring_fix[at] += n->wfix[q][blk[j]][widx[j]];
    else
      n->ring64[at] += n->wt64[q][blk[j]][widx[j]];
  }
}

static int step_once(orc_net* n) {
  const int64_t t = n->t, N = n->N;
  const int64_t slot = t % n->D;
  const int Q = n->p.q_frac_bits;
  const float inv2q = ldexpf(1.0f, -Q);
  int64_t n_spk = 0;
  for (int64_t i = 0; i < N; i++) {
    int64_t fix;
    double f64;
    orc_ext_input(n, i, t, &fix, &f64);
    size_t at = (size_t)slot * (size_t)N + (size_t)i;
    int spiked;
    if (n->mode == ORC_MIRROR32) {
      int64_t I = n->ring_fix[at] + fix;
      n->ring_fix[at] = 0;
      if (n->p.acc_bits == 32 && (I > 2147483647LL || I < -2147483648LL))
        n->status = ORC_E_RANGE;
      float dv = (float)I * inv2q;
      spiked = update_neuron32(n, i, dv);
    } else {
      double I = n->ring64[at] + f64;
      n->ring64[at] = 0.0;
      spiked = update_neuron64(n, i, I);
    }
    if (spiked) {
      n->spk_step[n_spk++] = i;
      if (n->p.plastic) n->t_post[i] = (int32_t)t;
    }
  }
  for (int64_t k = 0; k < n_spk; k++) {
    int rc = record_spike(n, t, n->spk_step[k]);
    if (rc != ORC_OK) return rc;
    deliver(n, n->spk_step[k], t);
  }
  n->t = t + 1;
  return ORC_OK;
}

int32_t orc_step(orc_net* n, int64_t n_steps) {
  if (!n || n_steps < 0) return ORC_E_INVAL;
  for (int64_t k = 0; k < n_steps; k++) {
    int rc = step_once(n);
    if (rc != ORC_OK) return rc;
    if (n->p.plastic && n->t % n->p.stdp_update_steps == 0) stdp_update(n, n->t);
  }
  return n->status;
}

int32_t orc_get_state(const orc_net* n, double* V, double* c, int32_t* ref) {
  for (int64_t i = 0; i < n->N; i++) {
    if (V) V[i] = n->mode == ORC_MIRROR32 ? (double)n->V32[i] : n->V64[i];
    if (c) c[i] = n->mode == ORC_MIRROR32 ? (double)n->c32[i] : n->c64[i];
    if (ref) ref[i] = n->ref[i];
  }
  return ORC_OK;
}

int32_t orc_set_state(orc_net* n, const double* V, const double* c,
                      const int32_t* ref) {
  for (int64_t i = 0; i < n->N; i++) {
    if (n->mode == ORC_MIRROR32) {
      if (V) n->V32[i] = (float)V[i];
      if (c) n->c32[i] = (float)c[i];
    } else {
      if (V) n->V64[i] = V[i];
      if (c) n->c64[i] = c[i];
    }
    if (ref) n->ref[i] = ref[i];
  }
  return ORC_OK;
}

int32_t orc_get_ring(const orc_net* n, int64_t* ring_fix, double* ring_f64) {
  size_t cnt = (size_t)n->D * (size_t)n->N;
  if (n->mode == ORC_MIRROR32) {
    if (!ring_fix) return ORC_E_INVAL;
    memcpy(ring_fix, n->ring_fix, cnt * sizeof(int64_t));
  } else {
    if (!ring_f64) return ORC_E_INVAL;
    memcpy(ring_f64, n->ring64, cnt * sizeof(double));
  }
  return ORC_OK;
}

int32_t orc_set_ring(orc_net* n, const int64_t* ring_fix, const double* ring_f64) {
  size_t cnt = (size_t)n->D * (size_t)n->N;
  if (n->mode == ORC_MIRROR32) {
    if (!ring_fix) return ORC_E_INVAL;
    memcpy(n->ring_fix, ring_fix, cnt * sizeof(int64_t));
  } else {
    if (!ring_f64) return ORC_E_INVAL;
    memcpy(n->ring64, ring_f64, cnt * sizeof(double));
  }
  return ORC_OK;
}

int32_t orc_set_time(orc_net* n, int64_t t) {
  if (t < 0) return ORC_E_INVAL;
  n->t = t;
  return ORC_OK;
}

int64_t orc_spikes(const orc_net* n, int32_t* step, int32_t* id, int64_t cap) {
  int64_t m = n->n_sp < cap ? n->n_sp : cap;
  if (step) memcpy(step, n->sp_t, sizeof(int32_t) * (size_t)(m > 0 ? m : 0));
  if (id) memcpy(id, n->sp_id, sizeof(int32_t) * (size_t)(m > 0 ? m : 0));
  return n->n_sp;
}

int64_t orc_rates(const orc_net* n, uint32_t* counts, int64_t cap_bins) {
  int64_t bins = n->t / n->p.rate_bin_steps + (n->t % n->p.rate_bin_steps ? 1 : 0);
  int64_t m = bins < cap_bins ? bins : cap_bins;
  if (counts && m > 0) {
    memset(counts, 0, sizeof(uint32_t) * (size_t)(m * n->M * n->P));
    int64_t have = n->rate_bins_used < m ? n->rate_bins_used : m;
    if (have > 0)
      memcpy(counts, n->rates, sizeof(uint32_t) * (size_t)(have * n->M * n->P));
  }
  return bins;
}

/* ------------------------------------------------------------------------ */
static int64_t put(void* out, int64_t cap, const void* src, int64_t bytes) {
  if (out && cap >= bytes) memcpy(out, src, (size_t)bytes);
  return bytes;
}

int64_t orc_table(const orc_net* n, const char* name, void* out, int64_t cap) {
  if (!n || !name) return ORC_E_INVAL;
  const int P = n->P;
  if (!strcmp(name, "prop_f64")) {     /* [pop][Pm, Pc, PVc, Iterm] */
    double v[4 * MAXP];
    for (int q = 0; q < P; q++) {
      v[4 * q] = n->Pm[q]; v[4 * q + 1] = n->Pc[q];
      v[4 * q + 2] = n->PVc[q]; v[4 * q + 3] = n->Iterm[q];
    }
    return put(out, cap, v, 32 * (int64_t)P);
  }
  if (!strcmp(name, "prop_f32")) {
    float v[4 * MAXP];
    for (int q = 0; q < P; q++) {
      v[4 * q] = n->Pm32[q]; v[4 * q + 1] = n->Pc32[q];
      v[4 * q + 2] = n->PVc32[q]; v[4 * q + 3] = n->Iterm32[q];
    }
    return put(out, cap, v, 16 * (int64_t)P);
  }
  if (!strcmp(name, "n_arp")) return put(out, cap, n->n_arp, 4 * (int64_t)P);
  if (!strcmp(name, "off_thr"))
    return put(out, cap, n->off_thr, 4 * (int64_t)(n->n_off > 1 ? n->n_off - 1 : 0));
  if (!strcmp(name, "off_xy"))
    return put(out, cap, n->off_xy, 8 * (int64_t)n->n_off);
  if (!strcmp(name, "s8")) return put(out, cap, n->s8, 4 * (int64_t)P);
  if (!strcmp(name, "s8fix")) return put(out, cap, n->s8fix, 8 * (int64_t)P);
  if (!strcmp(name, "blocks")) {     /* [pop][block][n, lo, hi, rule] */
    int32_t v[MAXP * MAXP * 4];
    memset(v, 0, sizeof(v));
    for (int q = 0; q < P; q++)
      for (int b = 0; b < n->n_blk[q]; b++) {
        int32_t* e = v + (q * MAXP + b) * 4;
        e[0] = n->blk_n[q][b]; e[1] = n->blk_lo[q][b];
        e[2] = n->blk_hi[q][b]; e[3] = n->blk_rule[q][b];
      }
    return put(out, cap, v, 16 * (int64_t)P * MAXP);
  }
  /* per-population tables "<name>_<q>"; efficacy tables "<name>_<q>" (block
   * 0) and "<name>_<q>_<b>" */
  for (int q = 0; q < P; q++) {
    char nm[40];
    snprintf(nm, sizeof nm, "pois_thr_%d", q);
    if (!strcmp(name, nm)) return put(out, cap, n->pois_thr[q], 4 * (int64_t)n->n_pois[q]);
    snprintf(nm, sizeof nm, "jx64_%d", q);
    if (!strcmp(name, nm)) return put(out, cap, n->jx64[q], 8 * (int64_t)ZN);
    snprintf(nm, sizeof nm, "jx32_%d", q);
    if (!strcmp(name, nm)) return put(out, cap, n->jx32[q], 4 * (int64_t)ZN);
    snprintf(nm, sizeof nm, "jxfix_%d", q);
    if (!strcmp(name, nm)) return put(out, cap, n->jxfix[q], 8 * (int64_t)ZN);
    for (int b = -1; b < n_tab(n, q); b++) {
      const int bb = b < 0 ? 0 : b;
      char sfx[16];
      if (b < 0)
        snprintf(sfx, sizeof sfx, "_%d", q);
      else
        snprintf(sfx, sizeof sfx, "_%d_%d", q, b);
      snprintf(nm, sizeof nm, "wt64%s", sfx);
      if (!strcmp(name, nm)) return put(out, cap, n->wt64[q][bb], 8 * (int64_t)ZN);
      snprintf(nm, sizeof nm, "wt32%s", sfx);
      if (!strcmp(name, nm)) return put(out, cap, n->wt32[q][bb], 4 * (int64_t)ZN);
      snprintf(nm, sizeof nm, "wt16%s", sfx);
      if (!strcmp(name, nm)) return put(out, cap, n->wt16[q][bb], 2 * (int64_t)ZN);
      snprintf(nm, sizeof nm, "wq8%s", sfx);
      if (!strcmp(name, nm)) return put(out, cap, n->wq8[q][bb], (int64_t)ZN);
      snprintf(nm, sizeof nm, "wfix%s", sfx);
      if (!strcmp(name, nm)) return put(out, cap, n->wfix[q][bb], 8 * (int64_t)ZN);
    }
  }
  return ORC_E_INVAL;
}
