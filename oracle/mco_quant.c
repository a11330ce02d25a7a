/*
 * mco_quant.c -- oracle error-bound split, grid compressor (Lorenzo
 * prediction on prequantised integers + linear quantisation), residual
 * quantiser, per-block learned/plain choice and the two decoders.
 *
 * TEST INFRASTRUCTURE (see mco.h).
 */
#include "mco.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double field_at(const void* x, int dtype, int64_t i)
{
    return dtype == MCO_F64 ? ((const double*)x)[i] : (double)((const float*)x)[i];
}

/* tau = eb * (xmax - xmin) (relative) or eb (absolute); tau1 = split * tau
 * is the grid's share, tau2 = tau - tau1 the residuals' share, so that
 * tau1 + tau2 <= tau (Sec. III).  c = 0.5 * (xmin + xmax) centres the
 * prequantised integers.  Rejects NaN/Inf fields, eb <= 0, split outside
 * (0, 1) and a share that rounds to zero. */
int mco_bound_compute(const void* x, int dtype, int64_t n, double eb, int relative,
                      double split, mco_bound* out)
{
    return mco_bound_compute_mode(x, dtype, n, eb, relative, split, MCO_SPLIT_SUM, out);
}

/* mode MCO_SPLIT_SUM: tau1 = split tau, tau2 = tau - tau1 (Sec. III: the
 * two components' bounds add up to tau), split in (0, 1).
 * mode MCO_SPLIT_FULL: tau1 = split tau, tau2 = tau, split in (0, 16]: the
 * residual is taken against the reconstructed grid, so a vertex's error is
 * the residual's own quantisation error and tau2 alone bounds it; tau1 then
 * only sets the grid's step. */
int mco_bound_compute_mode(const void* x, int dtype, int64_t n, double eb, int relative,
                           double split, int mode, mco_bound* out)
{
    memset(out, 0, sizeof *out);
    if (n <= 0 || !(eb > 0.0) || !isfinite(eb) || !(split > 0.0)) return MCO_ERR_ARG;
    if (mode == MCO_SPLIT_SUM ? !(split < 1.0) : (mode != MCO_SPLIT_FULL || !(split <= 16.0))) return MCO_ERR_ARG;
    double mn = field_at(x, dtype, 0), mx = mn;
    for (int64_t i = 0; i < n; ++i) {
        double v = field_at(x, dtype, i);
        if (!isfinite(v)) return MCO_ERR_ARG;
        if (v < mn) mn = v;
        if (v > mx) mx = v;
    }
    double tau = relative ? eb * (mx - mn) : eb;
    double tau1 = split * tau;
    double tau2 = mode == MCO_SPLIT_FULL ? tau : tau - tau1;
    if (!(tau1 > 0.0) || !(tau2 > 0.0)) return MCO_ERR_ARG;
    out->tau = tau;
    out->tau1 = tau1;
    out->tau2 = tau2;
    out->xmin = mn;
    out->xmax = mx;
    out->c = 0.5 * (mn + mx);
    out->step1 = 2.0 * tau1;
    out->inv1 = 1.0 / (2.0 * tau1);
    out->step2 = 2.0 * tau2;
    out->inv2 = 1.0 / (2.0 * tau2);
    return MCO_OK;
}

static int64_t pget(const int32_t* p, const mco_grid* g, int64_t i0, int64_t i1, int64_t i2)
{
    if (i0 < 0 || i1 < 0 || i2 < 0) return 0;
    return p[i0 + g->n[0] * (i1 + g->n[1] * i2)];
}

/* Lorenzo prediction error of the integer field p with zeros outside the
 * grid, in int64:
 *   2-D: d = p(i,j) - (p(i-1,j) + p(i,j-1) - p(i-1,j-1))
 *   3-D: d = p - (p100 + p010 + p001 - p110 - p101 - p011 + p111),
 *        pXYZ the neighbour at offset (-X,-Y,-Z). */
void mco_lorenzo(const int32_t* p, const mco_grid* g, int64_t* delta)
{
    for (int64_t i2 = 0; i2 < g->n[2]; ++i2)
        for (int64_t i1 = 0; i1 < g->n[1]; ++i1)
            for (int64_t i0 = 0; i0 < g->n[0]; ++i0) {
                int64_t j = i0 + g->n[0] * (i1 + g->n[1] * i2);
                int64_t pred;
                if (g->dim == 2) {
                    pred = pget(p, g, i0 - 1, i1, 0) + pget(p, g, i0, i1 - 1, 0)
                         - pget(p, g, i0 - 1, i1 - 1, 0);
                } else {
                    pred = pget(p, g, i0 - 1, i1, i2) + pget(p, g, i0, i1 - 1, i2)
                         + pget(p, g, i0, i1, i2 - 1) - pget(p, g, i0 - 1, i1 - 1, i2)
                         - pget(p, g, i0 - 1, i1, i2 - 1) - pget(p, g, i0, i1 - 1, i2 - 1)
                         + pget(p, g, i0 - 1, i1 - 1, i2 - 1);
                }
                delta[j] = (int64_t)p[j] - pred;
            }
}

/* Lorenzo codes of the prequantised grid p: code d + R, or 0 with (index,
 * d) listed when |d| > R - 1. */
static int grid_codes_from_p(const int32_t* p, const mco_grid* g, uint16_t* codes, int32_t* out_idx,
                             int32_t* out_delta, int64_t cap, int64_t* n_out)
{
    int64_t ng = g->n[0] * g->n[1] * g->n[2];
    int64_t* delta = (int64_t*)malloc((size_t)ng * sizeof(int64_t));
    if (!delta) return MCO_ERR_ARG;
    mco_lorenzo(p, g, delta);
    int64_t k = 0;
    for (int64_t j = 0; j < ng; ++j) {
        int64_t d = delta[j];
        if (d >= -(MCO_RADIUS - 1) && d <= MCO_RADIUS - 1) {
            codes[j] = (uint16_t)(d + MCO_RADIUS);
        } else {
            codes[j] = 0;
            if (k < cap) { out_idx[k] = (int32_t)j; out_delta[k] = (int32_t)d; }
            ++k;
        }
    }
    free(delta);
    *n_out = k;
    return k > cap ? MCO_ERR_CAPACITY : MCO_OK;
}

/* Grid compressor C(x1) with bound tau1.  Prequantise
 * p = (int32) rint(((double)v - c) * inv1), requiring
 * |((double)v - c) * inv1| < 2^27; Lorenzo-predict on the integers; a
 * prediction error |d| <= R-1 becomes code d + R, anything larger code 0
 * plus an outlier (j, d) in ascending j.  Returns MCO_ERR_RANGE or
 * MCO_ERR_CAPACITY (n_out still counts every outlier). */
int mco_grid_quantize(const float* v, const mco_grid* g, const mco_bound* b, int32_t* p,
                      uint16_t* codes, int32_t* out_idx, int32_t* out_delta, int64_t cap,
                      int64_t* n_out)
{
    int64_t ng = g->n[0] * g->n[1] * g->n[2];
    for (int64_t j = 0; j < ng; ++j) {
        double s = ((double)v[j] - b->c) * b->inv1;
        if (!(fabs(s) < 134217728.0)) return MCO_ERR_RANGE;
        p[j] = (int32_t)rint(s);
    }
    return grid_codes_from_p(p, g, codes, out_idx, out_delta, cap, n_out);
}

/* The same for FP64 grid values (the cluster-mean f). */
int mco_grid_quantize_f64(const double* v, const mco_grid* g, const mco_bound* b, int32_t* p,
                          uint16_t* codes, int32_t* out_idx, int32_t* out_delta, int64_t cap,
                          int64_t* n_out)
{
    int64_t ng = g->n[0] * g->n[1] * g->n[2];
    for (int64_t j = 0; j < ng; ++j) {
        double s = (v[j] - b->c) * b->inv1;
        if (!(fabs(s) < 134217728.0)) return MCO_ERR_RANGE;
        p[j] = (int32_t)rint(s);
    }
    return grid_codes_from_p(p, g, codes, out_idx, out_delta, cap, n_out);
}

/* Reconstructed grid x1' = (float)(c + (double)p * step1); known at
 * compression time without decoding. */
void mco_grid_recon(const int32_t* p, int64_t ng, const mco_bound* b, float* xhat)
{
    for (int64_t j = 0; j < ng; ++j) xhat[j] = (float)(b->c + (double)p[j] * b->step1);
}

/* Grid decoder D(mu1): d = code - R, or the outlier's d where code is 0;
 * p = inclusive prefix sum of d along axis 0, then 1, then 2 (the inverse
 * of the Lorenzo predictor). */
int mco_grid_decode(const uint16_t* codes, const int32_t* out_idx, const int32_t* out_delta,
                    int64_t n_out, const mco_grid* g, int32_t* p)
{
    int64_t n0 = g->n[0], n1 = g->n[1], n2 = g->n[2], ng = n0 * n1 * n2;
    int64_t* s = (int64_t*)malloc((size_t)ng * sizeof(int64_t));
    if (!s) return MCO_ERR_ARG;
    for (int64_t j = 0; j < ng; ++j) s[j] = (int64_t)codes[j] - MCO_RADIUS;
    for (int64_t k = 0; k < n_out; ++k) {
        int64_t j = out_idx[k];
        if (j < 0 || j >= ng || codes[j] != 0) { free(s); return MCO_ERR_ARG; }
        s[j] = out_delta[k];
    }
    for (int64_t i2 = 0; i2 < n2; ++i2)
        for (int64_t i1 = 0; i1 < n1; ++i1)
            for (int64_t i0 = 1; i0 < n0; ++i0) {
                int64_t j = i0 + n0 * (i1 + n1 * i2);
                s[j] += s[j - 1];
            }
    for (int64_t i2 = 0; i2 < n2; ++i2)
        for (int64_t i1 = 1; i1 < n1; ++i1)
            for (int64_t i0 = 0; i0 < n0; ++i0) {
                int64_t j = i0 + n0 * (i1 + n1 * i2);
                s[j] += s[j - n0];
            }
    for (int64_t i2 = 1; i2 < n2; ++i2)
        for (int64_t i1 = 0; i1 < n1; ++i1)
            for (int64_t i0 = 0; i0 < n0; ++i0) {
                int64_t j = i0 + n0 * (i1 + n1 * i2);
                s[j] += s[j - n0 * n1];
            }
    for (int64_t j = 0; j < ng; ++j) p[j] = (int32_t)s[j];
    free(s);
    return MCO_OK;
}

/* One vertex of the residual compressor C(x2) with bound tau2, against the
 * reconstructed grid (closed loop): r = (double)x - (double)g,
 * q = rint(r * inv2), candidate x' = (T)((double)g + q * step2); accepted
 * iff |q| <= R-1 and |(double)x - (double)x'| <= tau2. */
static int residual_one(double x, float gv, int dtype, const mco_bound* b, double* q_out)
{
    double r = x - (double)gv;
    double q = rint(r * b->inv2);
    double xr = (double)gv + q * b->step2;
    if (dtype == MCO_F32) xr = (double)(float)xr;
    *q_out = q;
    return fabs(q) <= (double)(MCO_RADIUS - 1) && fabs(x - xr) <= b->tau2;
}

static void put_val(void* out_val, int dtype, int64_t k, const void* x, int64_t v)
{
    if (dtype == MCO_F64) ((double*)out_val)[k] = ((const double*)x)[v];
    else ((float*)out_val)[k] = ((const float*)x)[v];
}

/* Residual codes: accepted vertex -> q + R, otherwise code 0 and an
 * outlier (v, raw x) in ascending v. */
int mco_residual_quantize(const void* x, int dtype, int64_t nv, const float* gv,
                          const mco_bound* b, uint16_t* codes, int32_t* out_idx,
                          void* out_val, int64_t cap, int64_t* n_out)
{
    int64_t k = 0;
    for (int64_t v = 0; v < nv; ++v) {
        double q;
        if (residual_one(field_at(x, dtype, v), gv[v], dtype, b, &q)) {
            codes[v] = (uint16_t)((int32_t)q + MCO_RADIUS);
        } else {
            codes[v] = 0;
            if (k < cap) { out_idx[k] = (int32_t)v; put_val(out_val, dtype, k, x, v); }
            ++k;
        }
    }
    *n_out = k;
    return k > cap ? MCO_ERR_CAPACITY : MCO_OK;
}

static int bitlen_zigzag(int32_t k)
{
    uint32_t z = ((uint32_t)k << 1) ^ (uint32_t)(k >> 31);
    int n = 0;
    while (z) { ++n; z >>= 1; }
    return n;
}

/* Learned codes given the predictor's per-vertex integer shift rho_q.  For
 * a plainly accepted vertex, the learned code is q - rho_q (+R) if it stays
 * within R-1, otherwise the vertex becomes an outlier.  Per block of 4096
 * consecutive vertices the cost of each variant is
 *   sum over coded vertices of bitlen(zigzag(code - R))
 *   + sum over outliers of (32 + 8 * sizeof(T)),
 * and the block is learned iff its learned cost is strictly smaller (bit b
 * of block_flags[b/32]).  The outlier list collects the chosen variant's
 * outliers in ascending v. */
int mco_learned_codes(const void* x, int dtype, int64_t nv, const float* gv,
                      const mco_bound* b, const int32_t* rho_q, uint16_t* codes,
                      uint32_t* block_flags, int32_t* out_idx, void* out_val, int64_t cap,
                      int64_t* n_out)
{
    int64_t nblocks = (nv + MCO_BLOCK - 1) / MCO_BLOCK;
    int outlier_cost = 32 + 8 * (dtype == MCO_F64 ? 8 : 4);
    memset(block_flags, 0, (size_t)((nblocks + 31) / 32) * sizeof(uint32_t));
    int64_t k = 0;
    for (int64_t blk = 0; blk < nblocks; ++blk) {
        int64_t v0 = blk * MCO_BLOCK, v1 = v0 + MCO_BLOCK < nv ? v0 + MCO_BLOCK : nv;
        int64_t cost_p = 0, cost_l = 0;
        for (int64_t v = v0; v < v1; ++v) {
            double q;
            if (residual_one(field_at(x, dtype, v), gv[v], dtype, b, &q)) {
                int32_t qi = (int32_t)q;
                int32_t cl = qi - rho_q[v];
                cost_p += bitlen_zigzag(qi);
                if (cl >= -(MCO_RADIUS - 1) && cl <= MCO_RADIUS - 1) cost_l += bitlen_zigzag(cl);
                else cost_l += outlier_cost;
            } else {
                cost_p += outlier_cost;
                cost_l += outlier_cost;
            }
        }
        int learned = cost_l < cost_p;
        if (learned) block_flags[blk / 32] |= 1u << (blk % 32);
        for (int64_t v = v0; v < v1; ++v) {
            double q;
            int ok = residual_one(field_at(x, dtype, v), gv[v], dtype, b, &q);
            int32_t code = ok ? (int32_t)q : 0;
            if (ok && learned) {
                code -= rho_q[v];
                if (code < -(MCO_RADIUS - 1) || code > MCO_RADIUS - 1) ok = 0;
            }
            if (ok) {
                codes[v] = (uint16_t)(code + MCO_RADIUS);
            } else {
                codes[v] = 0;
                if (k < cap) { out_idx[k] = (int32_t)v; put_val(out_val, dtype, k, x, v); }
                ++k;
            }
        }
    }
    *n_out = k;
    return k > cap ? MCO_ERR_CAPACITY : MCO_OK;
}

/* Residual decoder and recomposition x' = g(x1') + x2' (Alg. 4): outliers
 * take their raw value; otherwise q = code - R (+ rho_q in learned blocks)
 * and x' = (T)((double)g + q * step2). */
void mco_vertex_decode(const uint16_t* codes, const int32_t* out_idx, const void* out_val,
                       int64_t n_out, const float* gv, const mco_bound* b, int dtype,
                       int64_t nv, const int32_t* rho_q, const uint32_t* block_flags,
                       void* xout)
{
    for (int64_t v = 0; v < nv; ++v) {
        int32_t q = (int32_t)codes[v] - MCO_RADIUS;
        if (rho_q && block_flags) {
            int64_t blk = v / MCO_BLOCK;
            if ((block_flags[blk / 32] >> (blk % 32)) & 1u) q += rho_q[v];
        }
        double xr = (double)gv[v] + (double)q * b->step2;
        if (dtype == MCO_F64) ((double*)xout)[v] = xr;
        else ((float*)xout)[v] = (float)xr;
    }
    for (int64_t k = 0; k < n_out; ++k) {
        int64_t v = out_idx[k];
        if (dtype == MCO_F64) ((double*)xout)[v] = ((const double*)out_val)[k];
        else ((float*)xout)[v] = ((const float*)out_val)[k];
    }
}
