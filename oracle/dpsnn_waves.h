/* Slow-wave analysis of module rates (Sec. 2.3, Eq. 4): CPU oracle, test
 * infrastructure only.  The readings of the paper it takes are listed in
 * dpsnn_waves.c. */
#ifndef DPSNN_WAVES_ORACLE_H
#define DPSNN_WAVES_ORACLE_H

#include <stdint.h>

typedef struct orc_wave_params {
  int32_t W, H;          /* grid of modules; module m at x = m % W, y = m / W */
  int32_t n_pops;        /* populations per module in the counts */
  int32_t bin_steps;     /* steps per bin */
  double dt_ms;          /* step, ms */
  int64_t bin0;          /* absolute index of the first bin of the window */
  double noise_var;      /* variance of the added white noise (0.5) */
  uint64_t seed;         /* Philox key of the noise */
  int32_t min_down;      /* bins at or below threshold before a transition */
  int32_t min_up;        /* bins above threshold from a transition on */
  int32_t min_modules;   /* smallest wave whose speed is measured */
  int32_t reserved;
} orc_wave_params;

/* Upper bound of the transitions of one module in n_bins bins. */
int64_t orc_wave_transitions_max(int64_t n_bins, int32_t min_down, int32_t min_up);

/* counts: [nb][W*H][n_pops] spike counts.  Writes up to cap_tr transitions
 * in the order (bin, fraction, module) with their module, time (ms) and
 * wave, and up to cap_w waves (speed in inter-module distances per second,
 * NaN where not measured; first transition time; modules).  Returns the
 * number of transitions, *n_waves the number of waves; negative on invalid
 * parameters (-1) or memory (-2). */
int64_t orc_waves(const orc_wave_params* wp, const uint32_t* counts, int64_t nb,
                  int32_t* tr_module, double* tr_T, int32_t* tr_wave, int64_t cap_tr,
                  double* wave_speed, double* wave_t0, int32_t* wave_n, int64_t cap_w,
                  int64_t* n_waves);

#endif
