/* Slow-wave analysis of the module rates, CPU oracle (test infrastructure
 * only: the product path never calls it).
 *
 * Follows Sec. 2.3 of the paper: the multi-unit activity MUA(t) of a module
 * is its firing rate in bins of 5 ms; the analysed signal is
 * log(MUA / MUA_down) plus zero-mean white noise of variance 0.5, with
 * MUA_down the mean MUA in the Down state; a threshold gives the Down-to-Up
 * transition time T(x, y) of every grid point, and Eq. 4 the wavefront
 * speed V = 1 / |grad T|, averaged over the positions of a wave.
 *
 * The paper fixes neither the Down-state classification, nor the threshold,
 * nor how transitions are grouped into waves.  Readings taken here:
 *   - c(k) = spikes of the module in bin k (all populations); the Down bins
 *     are those with c at or below the lower median of the window, the Up
 *     bins the others; c_down and c_up are their mean counts rounded to the
 *     nearest integer (halves up), so that every logarithm is the log of an
 *     integer (one spike is added to every count: log(c + 1));
 *   - L(k) = log(c(k) + 1) - log(c_down + 1) + eta(k), eta = sqrt(noise_var)
 *     * z[u >> 16], u = word 0 of Philox(m, bin, bin >> 32, WAVE) keyed by
 *     the seed, z the 65536 standard normal quantiles at (i + 0.5) / 65536;
 *   - threshold theta = (log(c_up + 1) - log(c_down + 1)) / 2, halfway
 *     between the two levels;
 *   - a Down-to-Up transition at bin k: L <= theta on the min_down bins
 *     before k and L > theta on the min_up bins from k; its time is the
 *     linear interpolation of L between the centres of bins k-1 and k;
 *   - transitions of all modules ordered by (k, q, m) with q the 32-bit
 *     fixed-point fraction of the interpolation, then grouped greedily:
 *     a wave ends where a module would enter it a second time;
 *   - dT/dx and dT/dy: central differences where both neighbours took part
 *     in the wave, one-sided where one did (no wrap-around); a module
 *     contributes V = 1000 / sqrt(Tx^2 + Ty^2) (inter-module distances per
 *     second, T in ms) where both are defined and not both zero; the wave
 *     speed is the mean of V over the contributing modules, for waves of at
 *     least min_modules modules.
 * All arithmetic in binary64.
 */
#include "dpsnn_waves.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "dpsnn_oracle.h"

#define WAVE_TAG 5u
#define ZN 65536

typedef struct {
  uint32_t k;    /* window bin of the first Up bin */
  uint32_t q;    /* fraction of the interpolation, 32-bit fixed point */
  int32_t m;     /* module */
  double T;      /* transition time, ms */
} tr_t;

static int cmp_u32(const void* a, const void* b) {
  const uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : x > y;
}

static int cmp_tr(const void* a, const void* b) {
  const tr_t* x = (const tr_t*)a;
  const tr_t* y = (const tr_t*)b;
  if (x->k != y->k) return x->k < y->k ? -1 : 1;
  if (x->q != y->q) return x->q < y->q ? -1 : 1;
  return x->m < y->m ? -1 : x->m > y->m;
}

int64_t orc_wave_transitions_max(int64_t n_bins, int32_t min_down, int32_t min_up) {
  return n_bins / (min_down + min_up) + 1;
}

int64_t orc_waves(const orc_wave_params* wp, const uint32_t* counts, int64_t nb,
                  int32_t* tr_module, double* tr_T, int32_t* tr_wave, int64_t cap_tr,
                  double* wave_speed, double* wave_t0, int32_t* wave_n, int64_t cap_w,
                  int64_t* n_waves) {
  const int W = wp->W, H = wp->H, P = wp->n_pops;
  const int64_t M = (int64_t)W * H;
  if (W < 1 || H < 1 || P < 1 || nb < 1 || wp->min_down < 1 || wp->min_up < 1 ||
      wp->noise_var < 0.0 || wp->bin_steps < 1 || !(wp->dt_ms > 0.0))
    return -1;
  const double dbin = wp->bin_steps * wp->dt_ms;
  const double sd = sqrt(wp->noise_var);
  const uint32_t key[2] = {(uint32_t)wp->seed, (uint32_t)(wp->seed >> 32)};

  /* standard normal quantiles */
  double* z = (double*)malloc(sizeof(double) * ZN);
  uint32_t* c = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)nb);
  uint32_t* srt = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)nb);
  double* L = (double*)malloc(sizeof(double) * (size_t)nb);
  int64_t cap_all = M * orc_wave_transitions_max(nb, wp->min_down, wp->min_up);
  tr_t* tr = (tr_t*)malloc(sizeof(tr_t) * (size_t)cap_all);
  if (!z || !c || !srt || !L || !tr) {
    free(z); free(c); free(srt); free(L); free(tr);
    return -2;
  }
  for (int i = 0; i < ZN; i++) z[i] = orc_normal_quantile(((double)i + 0.5) / (double)ZN);

  int64_t n_tr = 0;
  for (int64_t m = 0; m < M; m++) {
    /* module signal: spikes per bin, all populations */
    for (int64_t k = 0; k < nb; k++) {
      uint32_t s = 0;
      for (int p = 0; p < P; p++) s += counts[(k * M + m) * P + p];
      c[k] = s;
    }
    memcpy(srt, c, sizeof(uint32_t) * (size_t)nb);
    qsort(srt, (size_t)nb, sizeof(uint32_t), cmp_u32);
    const uint32_t med = srt[(nb - 1) / 2];
    uint64_t s_lo = 0, n_lo = 0, s_hi = 0, n_hi = 0;
    for (int64_t k = 0; k < nb; k++) {
      if (c[k] <= med) {
        s_lo += c[k];
        n_lo++;
      } else {
        s_hi += c[k];
        n_hi++;
      }
    }
    if (n_hi == 0) continue;  /* no Up bins: no transitions */
    const uint64_t cd = (2 * s_lo + n_lo) / (2 * n_lo);
    const uint64_t cu = (2 * s_hi + n_hi) / (2 * n_hi);
    const double ld = log((double)(cd + 1));
    const double theta = 0.5 * (log((double)(cu + 1)) - ld);
    for (int64_t k = 0; k < nb; k++) {
      const uint64_t bin = (uint64_t)(wp->bin0 + k);
      const uint32_t ctr[4] = {(uint32_t)m, (uint32_t)bin, (uint32_t)(bin >> 32), WAVE_TAG};
      uint32_t u[4];
      orc_philox4x32_10(ctr, key, u);
      const double eta = sd * z[u[0] >> 16];
      L[k] = (log((double)c[k] + 1.0) - ld) + eta;
    }
    for (int64_t k = wp->min_down; k + wp->min_up <= nb; k++) {
      int ok = 1;
      for (int64_t j = k - wp->min_down; j < k && ok; j++) ok = L[j] <= theta;
      for (int64_t j = k; j < k + wp->min_up && ok; j++) ok = L[j] > theta;
      if (!ok) continue;
      const double frac = (theta - L[k - 1]) / (L[k] - L[k - 1]);
      tr[n_tr].k = (uint32_t)k;
      const double fq = frac * 4294967296.0;
      tr[n_tr].q = fq < 4294967295.0 ? (uint32_t)fq : 4294967295u;
      tr[n_tr].m = (int32_t)m;
      tr[n_tr].T = ((double)(wp->bin0 + k) - 0.5 + frac) * dbin;
      n_tr++;
    }
  }
  qsort(tr, (size_t)n_tr, sizeof(tr_t), cmp_tr);

  /* greedy grouping: a module entering the current wave again starts the
   * next wave */
  int32_t* last = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
  int32_t* wid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_tr > 0 ? n_tr : 1));
  double* grid = (double*)malloc(sizeof(double) * (size_t)M);
  if (!last || !wid || !grid) {
    free(z); free(c); free(srt); free(L); free(tr); free(last); free(wid); free(grid);
    return -2;
  }
  for (int64_t m = 0; m < M; m++) last[m] = -1;
  int32_t w = 0;
  for (int64_t i = 0; i < n_tr; i++) {
    if (last[tr[i].m] == w) w++;
    last[tr[i].m] = w;
    wid[i] = w;
  }
  const int64_t nw = n_tr > 0 ? (int64_t)w + 1 : 0;
  *n_waves = nw;

  /* Eq. 4 per wave */
  int64_t i0 = 0;
  for (int64_t v = 0; v < nw; v++) {
    int64_t i1 = i0;
    while (i1 < n_tr && wid[i1] == v) i1++;
    for (int64_t m = 0; m < M; m++) grid[m] = NAN;
    double t0 = INFINITY;
    for (int64_t i = i0; i < i1; i++) {
      grid[tr[i].m] = tr[i].T;
      if (tr[i].T < t0) t0 = tr[i].T;
    }
    double sum = 0.0;
    int64_t cnt = 0;
    if (i1 - i0 >= wp->min_modules) {
      for (int64_t m = 0; m < M; m++) {
        const double Tm = grid[m];
        if (isnan(Tm)) continue;
        const int x = (int)(m % W), y = (int)(m / W);
        const double tl = x > 0 ? grid[m - 1] : NAN, tr_ = x + 1 < W ? grid[m + 1] : NAN;
        const double td = y > 0 ? grid[m - W] : NAN, tu = y + 1 < H ? grid[m + W] : NAN;
        double gx, gy;
        if (!isnan(tl) && !isnan(tr_)) gx = 0.5 * (tr_ - tl);
        else if (!isnan(tr_)) gx = tr_ - Tm;
        else if (!isnan(tl)) gx = Tm - tl;
        else continue;
        if (!isnan(td) && !isnan(tu)) gy = 0.5 * (tu - td);
        else if (!isnan(tu)) gy = tu - Tm;
        else if (!isnan(td)) gy = Tm - td;
        else continue;
        const double g2 = gx * gx + gy * gy;
        if (g2 == 0.0) continue;
        sum += 1000.0 / sqrt(g2);
        cnt++;
      }
    }
    if (v < cap_w) {
      if (wave_speed) wave_speed[v] = cnt > 0 ? sum / (double)cnt : NAN;
      if (wave_t0) wave_t0[v] = t0;
      if (wave_n) wave_n[v] = (int32_t)(i1 - i0);
    }
    i0 = i1;
  }
  for (int64_t i = 0; i < n_tr && i < cap_tr; i++) {
    if (tr_module) tr_module[i] = tr[i].m;
    if (tr_T) tr_T[i] = tr[i].T;
    if (tr_wave) tr_wave[i] = wid[i];
  }
  free(z); free(c); free(srt); free(L); free(tr); free(last); free(wid); free(grid);
  return n_tr;
}
