/*
 * mco_serial.c -- oracle of the 1-D serialisation baseline: the vertex
 * array compressed as a plain 1-D signal by the same kind of error-bounded
 * predictor-quantiser (the "default" compression that the paper's
 * multi-component scheme is compared with in Sec. V-C, where the underlying
 * compressor sees the serialised vertex values).
 *
 * TEST INFRASTRUCTURE, like the rest of this directory.
 *
 * With the whole bound tau on the one component (step = 2 tau, c = the
 * mid-range of the field):
 *   p_i  = rint((x_i - c) / (2 tau))          FP64, |.| < 2^27
 *   d_i  = p_i - p_{i-1}                      (p_{-1} = 0), 1-D Lorenzo
 *   x'_i = (T)(c + p_i * 2 tau)
 *   code_i = d_i + R  if |d_i| <= R - 1 and |x_i - x'_i| <= tau,
 *            0        otherwise (the raw value is stored, index order).
 * The decoder rebuilds p_i as the running sum of the codes, restarting at
 * every raw value from p_i = rint((raw - c) / (2 tau)), which is the
 * encoder's p_i for that vertex.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "mco.h"

static double val_at(const void* x, int dtype, int64_t i)
{
    return dtype == MCO_F64 ? ((const double*)x)[i] : (double)((const float*)x)[i];
}

static double as_t(double v, int dtype)
{
    return dtype == MCO_F64 ? v : (double)(float)v;
}

int mco_serial_compress(const void* x, int dtype, int64_t n, double eb, int relative, uint16_t* codes,
                        int32_t* out_idx, void* out_val, int64_t cap, int64_t* n_out, mco_bound* b)
{
    int st = mco_bound_compute(x, dtype, n, eb, relative, 0.5, b);
    if (st != MCO_OK) return st;
    const double step = 2.0 * b->tau, inv = 1.0 / (2.0 * b->tau);
    int64_t prev = 0, k = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double xi = val_at(x, dtype, i);
        const double s = (xi - b->c) * inv;
        if (!(fabs(s) < 134217728.0)) return MCO_ERR_RANGE;
        const int64_t p = (int64_t)rint(s);
        const int64_t d = p - prev;
        prev = p;
        const double xr = as_t(b->c + (double)p * step, dtype);
        if (d >= -(MCO_RADIUS - 1) && d <= MCO_RADIUS - 1 && fabs(xi - xr) <= b->tau) {
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

void mco_serial_decompress(const uint16_t* codes, const int32_t* out_idx, const void* out_val, int64_t n_out,
                           int64_t n, const mco_bound* b, int dtype, void* out)
{
    const double step = 2.0 * b->tau, inv = 1.0 / (2.0 * b->tau);
    int64_t p = 0, k = 0;
    for (int64_t i = 0; i < n; ++i) {
        double xr;
        if (codes[i] != 0) {
            p += (int64_t)codes[i] - MCO_RADIUS;
            xr = as_t(b->c + (double)p * step, dtype);
        } else {
            while (k < n_out && out_idx[k] < i) ++k;
            const double raw = (k < n_out && out_idx[k] == i) ? val_at(out_val, dtype, k) : 0.0;
            p = (int64_t)rint((raw - b->c) * inv);
            xr = raw;
        }
        if (dtype == MCO_F64) ((double*)out)[i] = xr;
        else ((float*)out)[i] = (float)xr;
    }
}
