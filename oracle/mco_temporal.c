/*
 * mco_temporal.c -- oracle of the time-axis grid predictor: a further grid
 * compressor C(x1) (Sec. IV-D admits any; Sec. I notes that analyses use
 * many timesteps of one mesh), predicting each node of the prequantised grid
 * p of timestep t from a reference grid r that both sides hold, normally
 * the reconstructed grid x1' of timestep t - 1.
 *
 * TEST INFRASTRUCTURE, like the rest of this directory.
 *
 *   s_j    = ((double)r_j - c) * inv1         (c, inv1 of this timestep)
 *   P_j    = rint(s_j) when |s_j| < 2^27, else 0 (also for NaN)
 *   d_j    = p_j - P_j, coded as d + R, or 0 with (j, d) listed in ascending
 *            j when |d| > R - 1
 *   decode p_j = P_j + d_j
 */
#include <math.h>
#include <stdint.h>

#include "mco.h"

static int64_t temporal_pred(float r, const mco_bound* b)
{
    const double s = ((double)r - b->c) * b->inv1;
    return fabs(s) < 134217728.0 ? (int64_t)rint(s) : 0;
}

int mco_temporal_codes(const int32_t* p, const float* ref, int64_t ng, const mco_bound* b, uint16_t* codes,
                       int32_t* out_idx, int32_t* out_delta, int64_t cap, int64_t* n_out)
{
    int64_t k = 0;
    for (int64_t j = 0; j < ng; ++j) {
        const int64_t d = (int64_t)p[j] - temporal_pred(ref[j], b);
        if (d >= -(MCO_RADIUS - 1) && d <= MCO_RADIUS - 1) {
            codes[j] = (uint16_t)(d + MCO_RADIUS);
        } else {
            codes[j] = 0;
            if (k < cap) { out_idx[k] = (int32_t)j; out_delta[k] = (int32_t)d; }
            ++k;
        }
    }
    *n_out = k;
    return k > cap ? MCO_ERR_CAPACITY : MCO_OK;
}

int mco_temporal_decode(const uint16_t* codes, const int32_t* out_idx, const int32_t* out_delta, int64_t n_out,
                        const float* ref, int64_t ng, const mco_bound* b, int32_t* p)
{
    for (int64_t j = 0; j < ng; ++j) p[j] = (int32_t)(temporal_pred(ref[j], b) + ((int64_t)codes[j] - MCO_RADIUS));
    for (int64_t k = 0; k < n_out; ++k) {
        const int64_t j = out_idx[k];
        if (j < 0 || j >= ng || codes[j] != 0) return MCO_ERR_ARG;
        p[j] = (int32_t)(temporal_pred(ref[j], b) + out_delta[k]);
    }
    return MCO_OK;
}
