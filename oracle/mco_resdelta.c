/*
 * mco_resdelta.c -- oracle of the residual compressor with a 1-D Lorenzo
 * predictor along the vertex order: the residuals, serialised as a 1-D
 * array, go through a predictive quantiser as the paper's underlying
 * compressors do with them (Sec. IV-B: the residuals are serialised into a
 * 1-D array and compressed), instead of being quantised value by value.
 *
 * TEST INFRASTRUCTURE, like the rest of this directory.
 *
 *   q_i  = rint((x_i - g_i) / (2 tau2))     FP64, |.| < 2^27 (else MCO_ERR_RANGE)
 *   x'_i = (T)(g_i + q_i 2 tau2),  ok_i = |x_i - x'_i| <= tau2
 *   d_i  = q_i - q_{i-1},  q_{-1} = 0
 *   code_i = d_i + R  if ok_i and |d_i| <= R - 1, else 0 with x_i stored raw.
 * The decoder's q is the running sum of the codes, restarted at a raw value
 * from rint((raw - g_i) / (2 tau2)), which is the encoder's q_i there.
 */
#include <math.h>
#include <stdint.h>

#include "mco.h"

static double val_at(const void* x, int dtype, int64_t i)
{
    return dtype == MCO_F64 ? ((const double*)x)[i] : (double)((const float*)x)[i];
}

int mco_residual_delta(const void* x, int dtype, int64_t nv, const float* gv, const mco_bound* b, uint16_t* codes,
                       int32_t* out_idx, void* out_val, int64_t cap, int64_t* n_out)
{
    int64_t k = 0, prev = 0;
    for (int64_t i = 0; i < nv; ++i) {
        const double xi = val_at(x, dtype, i);
        const double s = (xi - (double)gv[i]) * b->inv2;
        if (!(fabs(s) < 134217728.0)) return MCO_ERR_RANGE;
        const int64_t q = (int64_t)rint(s);
        const double sum = (double)gv[i] + (double)q * b->step2;
        const double xr = dtype == MCO_F64 ? sum : (double)(float)sum;
        const int64_t d = q - prev;
        prev = q;
        if (fabs(xi - xr) <= b->tau2 && d >= -(MCO_RADIUS - 1) && d <= MCO_RADIUS - 1) {
            codes[i] = (uint16_t)(d + MCO_RADIUS);
        } else {
            codes[i] = 0;
            if (k < cap) {
                out_idx[k] = (int32_t)i;
                if (dtype == MCO_F64) ((double*)out_val)[k] = xi;
                else ((float*)out_val)[k] = (float)xi;
            }
            ++k;
        }
    }
    *n_out = k;
    return k > cap ? MCO_ERR_CAPACITY : MCO_OK;
}

void mco_vertex_decode_delta(const uint16_t* codes, const int32_t* out_idx, const void* out_val, int64_t n_out,
                             const float* gv, const mco_bound* b, int dtype, int64_t nv, void* xout)
{
    int64_t q = 0, k = 0;
    for (int64_t i = 0; i < nv; ++i) {
        double v;
        if (codes[i] != 0) {
            q += (int64_t)codes[i] - MCO_RADIUS;
            v = (double)gv[i] + (double)q * b->step2;
        } else {
            while (k < n_out && out_idx[k] < i) ++k;
            v = (k < n_out && out_idx[k] == i) ? val_at(out_val, dtype, k) : 0.0;
            q = (int64_t)rint((v - (double)gv[i]) * b->inv2);
        }
        if (dtype == MCO_F64) ((double*)xout)[i] = v;
        else ((float*)xout)[i] = (float)v;
    }
}
