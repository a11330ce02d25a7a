/*
 * mco_grid_init.c -- oracle of the grid initialisation (Alg. 1, Sec. IV-C):
 * the grid spacing of each axis is a low percentile of the distances
 * between the vertices of the mesh's cells along that axis, and the grid
 * spans the vertices' bounding box.
 *
 * TEST INFRASTRUCTURE, like the rest of this directory.
 *
 *   distances  s = |p_a,d - p_b,d| (FP32) for every edge (a, b) of every
 *              cell: 3 per triangle, 6 per tetrahedron (an edge shared by
 *              several cells counts once per cell)
 *   percentile the value of rank ceil(k N / 100) (1-based, at least 1) of
 *              the N sorted distances (nearest rank)
 *   G_max      while (max_d - min_d) / gs_d >= G_max, k grows by one
 *              percentage point, at most to 100 (then MCO_ERR_ARG)
 *   grid       origin min_d, spacing gs_d, n_d = ceil((max_d - min_d) / gs_d) + 1
 *              (at least 2), as a grid given by its spacing
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "mco.h"

static int cmp_float(const void* a, const void* b)
{
    const float x = *(const float*)a, y = *(const float*)b;
    return (x > y) - (x < y);
}

static float percentile_of(const float* sorted, int64_t n, double k)
{
    double r = ceil((k * (double)n) / 100.0);
    if (r < 1.0) r = 1.0;
    if (r > (double)n) r = (double)n;
    return sorted[(int64_t)r - 1];
}

int mco_grid_init(const float* coords, const int32_t* cells, int dim, int64_t nv, int64_t nc, double k0,
                  int64_t g_max, mco_grid* g, double k_used[3])
{
    static const int e2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    static const int e3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    if ((dim != 2 && dim != 3) || nv <= 0 || nc <= 0 || !(k0 >= 0.0) || !(k0 <= 100.0) || g_max < 2)
        return MCO_ERR_ARG;
    const int ne = dim == 2 ? 3 : 6;
    const int64_t n = nc * ne;
    float* s = (float*)malloc((size_t)n * sizeof(float));
    if (!s) return MCO_ERR_ARG;
    float lo[3], hi[3];
    mco_bbox(coords, dim, nv, lo, hi);
    memset(g, 0, sizeof *g);
    g->dim = dim;
    for (int d = 0; d < 3; ++d) {
        g->n[d] = 1;
        g->o[d] = 0.0;
        g->h[d] = 1.0;
        if (k_used) k_used[d] = 0.0;
    }
    for (int d = 0; d < dim; ++d) {
        for (int64_t c = 0; c < nc; ++c)
            for (int e = 0; e < ne; ++e) {
                const int ia = dim == 2 ? e2[e][0] : e3[e][0], ib = dim == 2 ? e2[e][1] : e3[e][1];
                const int32_t a = cells[(int64_t)ia * nc + c], b = cells[(int64_t)ib * nc + c];
                if (a < 0 || a >= nv || b < 0 || b >= nv) { free(s); return MCO_ERR_ARG; }
                s[c * ne + e] = fabsf(coords[(int64_t)d * nv + a] - coords[(int64_t)d * nv + b]);
            }
        qsort(s, (size_t)n, sizeof(float), cmp_float);
        const double extent = (double)hi[d] - (double)lo[d];
        double k = k0;
        double gs = (double)percentile_of(s, n, k);
        while (!(extent / gs < (double)g_max)) {            /* also when gs = 0 */
            if (k >= 100.0) { free(s); return MCO_ERR_ARG; }
            k = k + 1.0 > 100.0 ? 100.0 : k + 1.0;
            gs = (double)percentile_of(s, n, k);
        }
        double nd = ceil(extent / gs) + 1.0;
        if (nd < 2.0) nd = 2.0;
        g->n[d] = (int64_t)nd;
        g->o[d] = (double)lo[d];
        g->h[d] = gs;
        if (k_used) k_used[d] = k;
    }
    free(s);
    return MCO_OK;
}
