/*
 * mco_interp.c -- oracle of a second grid compressor C(x1): the multilevel
 * interpolation predictor of the SZ family (Sec. II names polynomial
 * interpolation among its predictors; Sec. IV-D lets C be any
 * error-controlled compressor), run on the prequantised integer grid p of
 * the Lorenzo path, so that the bound tau1 and the code format stay as they
 * are and only the prediction of each node changes.
 *
 * TEST INFRASTRUCTURE, like the rest of this directory.
 *
 * Levels.  L is the smallest integer with 2^L >= n_d on every axis; the
 * strides are s = 2^(L-1), ..., 2, 1.  The origin node is predicted by 0.
 * Any other node, with coordinates (i_0, .., i_{D-1}), belongs to the
 * class (s, a):
 *   t = the least number of trailing zero bits among its non-zero i_d,
 *   s = 2^t, a = the highest axis whose i_a is non-zero with t trailing
 *   zeros (so i_a is an odd multiple of s).
 * Its prediction interpolates along axis a between the nodes at i_a - s
 * (always inside the grid) and i_a + s, the other coordinates unchanged:
 *   both inside, cubic and i_a - 3s, i_a + 3s inside too:
 *       floor((-p[-3s] + 9 p[-s] + 9 p[+s] - p[+3s] + 8) / 16)
 *   both inside otherwise:  floor((p[-s] + p[+s]) / 2)
 *   i_a + s outside:        p[-s]
 * The error d = p - prediction is coded as for the Lorenzo path: d + R,
 * or 0 with (index, d) listed in ascending index when |d| > R - 1.
 *
 * Decoding visits the origin, then for s from 2^(L-1) down to 1 and a from
 * 0 to D-1 every node of class (s, a).  Every node a prediction reads lies
 * in an earlier class: its i_a is an even multiple of s, so it either has a
 * lower axis with t trailing zeros (same stride, earlier axis) or only
 * coordinates with more trailing zeros (a coarser stride, or the origin).
 * The decoder below checks that claim on every read.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "mco.h"

static int tz64(int64_t v)
{
    int t = 0;
    while ((v & 1) == 0) { v >>= 1; ++t; }
    return t;
}

static int levels_of(const mco_grid* g)
{
    int L = 0;
    for (int d = 0; d < g->dim; ++d)
        while (((int64_t)1 << L) < g->n[d]) ++L;
    return L;
}

/* Class of node (i[0..dim-1]): returns 0 for the origin, else 1 with the
 * stride and axis. */
static int class_of(const int64_t* i, int dim, int64_t* s, int* a)
{
    int t = 64;
    for (int d = 0; d < dim; ++d)
        if (i[d] != 0 && tz64(i[d]) < t) t = tz64(i[d]);
    if (t == 64) return 0;
    *a = -1;
    for (int d = 0; d < dim; ++d)
        if (i[d] != 0 && tz64(i[d]) == t) *a = d;
    *s = (int64_t)1 << t;
    return 1;
}

static int64_t node_index(const mco_grid* g, const int64_t* i)
{
    int64_t j = 0;
    for (int d = g->dim - 1; d >= 0; --d) j = j * g->n[d] + i[d];
    return j;
}

/* p at the node i with axis a moved by off; *ok cleared if that node has
 * not been decoded yet (known == NULL: no check). */
static int64_t at(const int32_t* p, const unsigned char* known, const mco_grid* g, const int64_t* i, int a,
                  int64_t off, int* ok)
{
    int64_t k[3] = {i[0], i[1], i[2]};
    k[a] += off;
    const int64_t j = node_index(g, k);
    if (known && !known[j]) *ok = 0;
    return p[j];
}

static int64_t predict(const int32_t* p, const unsigned char* known, const mco_grid* g, const int64_t* i, int64_t s,
                       int a, int cubic, int* ok)
{
    const int64_t n = g->n[a], x = i[a];
    const int64_t A = at(p, known, g, i, a, -s, ok);
    if (x + s > n - 1) return A;
    const int64_t B = at(p, known, g, i, a, s, ok);
    if (cubic && x - 3 * s >= 0 && x + 3 * s <= n - 1) {
        const int64_t A3 = at(p, known, g, i, a, -3 * s, ok), B3 = at(p, known, g, i, a, 3 * s, ok);
        return (int64_t)floor((double)(-A3 + 9 * A + 9 * B - B3 + 8) / 16.0);
    }
    return (int64_t)floor((double)(A + B) / 2.0);
}

static void coords_of(const mco_grid* g, int64_t j, int64_t* i)
{
    i[0] = i[1] = i[2] = 0;
    for (int d = 0; d < g->dim; ++d) {
        i[d] = j % g->n[d];
        j /= g->n[d];
    }
}

void mco_interp_delta(const int32_t* p, const mco_grid* g, int cubic, int64_t* delta)
{
    const int64_t ng = g->n[0] * g->n[1] * g->n[2];
    for (int64_t j = 0; j < ng; ++j) {
        int64_t i[3], s = 0;
        int a = 0, ok = 1;
        coords_of(g, j, i);
        const int64_t pred = class_of(i, g->dim, &s, &a) ? predict(p, NULL, g, i, s, a, cubic, &ok) : 0;
        delta[j] = (int64_t)p[j] - pred;
    }
}

int mco_interp_codes(const int32_t* p, const mco_grid* g, int cubic, uint16_t* codes, int32_t* out_idx,
                     int32_t* out_delta, int64_t cap, int64_t* n_out)
{
    const int64_t ng = g->n[0] * g->n[1] * g->n[2];
    int64_t* delta = (int64_t*)malloc((size_t)ng * sizeof(int64_t));
    if (!delta) return MCO_ERR_ARG;
    mco_interp_delta(p, g, cubic, delta);
    int64_t k = 0;
    for (int64_t j = 0; j < ng; ++j) {
        const int64_t d = delta[j];
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

int mco_interp_decode(const uint16_t* codes, const int32_t* out_idx, const int32_t* out_delta, int64_t n_out,
                      const mco_grid* g, int cubic, int32_t* p)
{
    const int64_t ng = g->n[0] * g->n[1] * g->n[2];
    int64_t* d = (int64_t*)malloc((size_t)ng * sizeof(int64_t));
    unsigned char* known = (unsigned char*)calloc((size_t)ng, 1);
    if (!d || !known) { free(d); free(known); return MCO_ERR_ARG; }
    for (int64_t j = 0; j < ng; ++j) d[j] = (int64_t)codes[j] - MCO_RADIUS;
    for (int64_t k = 0; k < n_out; ++k) {
        const int64_t j = out_idx[k];
        if (j < 0 || j >= ng || codes[j] != 0) { free(d); free(known); return MCO_ERR_ARG; }
        d[j] = out_delta[k];
    }
    for (int64_t j = 0; j < ng; ++j) p[j] = 0;
    p[0] = (int32_t)d[0];
    known[0] = 1;
    int ok = 1;
    for (int64_t s = (int64_t)1 << (levels_of(g) - 1); s >= 1 && ok; s /= 2)
        for (int a = 0; a < g->dim && ok; ++a)
            for (int64_t j = 1; j < ng; ++j) {
                int64_t i[3], sj = 0;
                int aj = 0;
                coords_of(g, j, i);
                if (!class_of(i, g->dim, &sj, &aj) || sj != s || aj != a) continue;
                p[j] = (int32_t)(predict(p, known, g, i, s, a, cubic, &ok) + d[j]);
                known[j] = 1;
            }
    for (int64_t j = 0; j < ng && ok; ++j)
        if (!known[j]) ok = 0;
    free(d);
    free(known);
    return ok ? MCO_OK : MCO_ERR_ARG;
}
