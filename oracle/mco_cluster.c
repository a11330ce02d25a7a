/*
 * mco_cluster.c -- oracle of the paper's own operator pair: the
 * nearest-node back-interpolation g and the cluster-mean resampling f
 * (Sec. IV-C: each vertex approximated by its closest grid node m_k;
 * Sec. IV-D: a node's value is the mean of the vertices assigned to it),
 * with the residual of Alg. 3 taken against the uncompressed grid x1
 * (open loop) or, as an option, against the reconstructed grid x1'.
 *
 * TEST INFRASTRUCTURE, like the rest of this directory.
 *
 *   m_k   = per axis rint((p_d - o_d) / h_d), clamped to [0, n_d - 1]
 *   x1[j] = (sum of x_k over m_k = j, in FP64, ascending k) / count_j;
 *           a node no vertex maps to holds c (prequantised value 0)
 *   p[j]  = rint((x1[j] - c) / (2 tau1)), Lorenzo-coded as for the linear pair
 *   x1'[j] = (float)(c + p[j] 2 tau1), the grid decoder's FP32 output
 *   open:   q_k = rint((x_k - x1[m_k]) / (2 tau2)), bound tau1 + tau2 = tau
 *   closed: q_k = rint((x_k - x1'[m_k]) / (2 tau2)), bound tau2
 *   x'_k = (T)(x1'[m_k] + q_k 2 tau2); code q + R when |q| <= R - 1 and
 *   |x_k - x'_k| <= bound, else 0 with x_k stored raw.
 * With g the nearest node (one weight of 1), Sec. III's bound reads
 * tau1 + tau2 <= tau for the open loop; the per-vertex check makes it hold
 * after rounding too.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "mco.h"

static double val_at(const void* x, int dtype, int64_t i)
{
    return dtype == MCO_F64 ? ((const double*)x)[i] : (double)((const float*)x)[i];
}

void mco_nearest_nodes(const float* coords, int dim, int64_t nv, const mco_grid* g, int32_t* m)
{
    for (int64_t k = 0; k < nv; ++k) {
        int64_t idx[3] = {0, 0, 0};
        for (int d = 0; d < dim; ++d) {
            double t = rint(((double)coords[d * nv + k] - g->o[d]) / g->h[d]);
            if (!(t >= 0.0)) t = 0.0;                       /* also catches NaN */
            if (t > (double)(g->n[d] - 1)) t = (double)(g->n[d] - 1);
            idx[d] = (int64_t)t;
        }
        m[k] = (int32_t)(idx[0] + g->n[0] * (idx[1] + g->n[1] * idx[2]));
    }
}

void mco_cluster_mean(const void* x, int dtype, int64_t nv, const int32_t* m, int64_t ng, double c,
                      double* x1, int32_t* count)
{
    for (int64_t j = 0; j < ng; ++j) {
        x1[j] = 0.0;
        count[j] = 0;
    }
    for (int64_t k = 0; k < nv; ++k) {          /* ascending k: the sum order */
        x1[m[k]] = x1[m[k]] + val_at(x, dtype, k);
        count[m[k]] += 1;
    }
    for (int64_t j = 0; j < ng; ++j) x1[j] = count[j] > 0 ? x1[j] / (double)count[j] : c;
}

int mco_residual_nearest(const void* x, int dtype, int64_t nv, const int32_t* m, const double* x1,
                         const float* xhat, const mco_bound* b, int open, uint16_t* codes, int32_t* out_idx,
                         void* out_val, int64_t cap, int64_t* n_out)
{
    const double bound = open ? b->tau : b->tau2;
    int64_t k = 0;
    for (int64_t i = 0; i < nv; ++i) {
        const double xi = val_at(x, dtype, i);
        const double xh = (double)xhat[m[i]];
        const double ref = open ? x1[m[i]] : xh;
        const double q = rint((xi - ref) * b->inv2);
        const double sum = xh + q * b->step2;
        const double xr = dtype == MCO_F64 ? sum : (double)(float)sum;
        if (fabs(q) <= (double)(MCO_RADIUS - 1) && fabs(xi - xr) <= bound) {
            codes[i] = (uint16_t)((int)q + MCO_RADIUS);
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

void mco_vertex_decode_nearest(const uint16_t* codes, const int32_t* out_idx, const void* out_val, int64_t n_out,
                               const int32_t* m, const float* xhat, const mco_bound* b, int dtype, int64_t nv,
                               void* xout)
{
    int64_t k = 0;
    for (int64_t i = 0; i < nv; ++i) {
        double v;
        if (codes[i] == 0) {
            while (k < n_out && out_idx[k] < i) ++k;
            v = (k < n_out && out_idx[k] == i) ? val_at(out_val, dtype, k) : 0.0;
        } else {
            v = (double)xhat[m[i]] + (double)((int)codes[i] - MCO_RADIUS) * b->step2;
        }
        if (dtype == MCO_F64) ((double*)xout)[i] = v;
        else ((float*)xout)[i] = (float)v;
    }
}

/* Grid_Coarsen (Alg. 2) for the nearest-node g: a grid plane (all nodes
 * with one coordinate fixed along one axis) that no vertex maps to is
 * dropped, axis by axis; an axis left with fewer than two planes keeps all
 * of its planes.  keep[off_d + i] is plane i's index on the coarsened axis
 * d, or -1 when dropped (off_0 = 0, off_1 = n_0, off_2 = n_0 + n_1);
 * new_n the coarsened extents; m_out the vertices' nodes on the coarsened
 * grid.  Only the node indices change: every vertex keeps its node. */
void mco_grid_coarsen(const int32_t* m, int64_t nv, const mco_grid* g, int32_t* keep, int64_t new_n[3],
                      int32_t* m_out)
{
    const int64_t n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    const int64_t off[3] = {0, n0, n0 + n1};
    for (int64_t i = 0; i < n0 + n1 + n2; ++i) keep[i] = 0;
    for (int64_t k = 0; k < nv; ++k) {            /* visited planes */
        const int64_t j = m[k];
        keep[off[0] + j % n0] = 1;
        keep[off[1] + (j / n0) % n1] = 1;
        keep[off[2] + j / (n0 * n1)] = 1;
    }
    for (int d = 0; d < 3; ++d) {
        int64_t cnt = 0;
        for (int64_t i = 0; i < g->n[d]; ++i) cnt += keep[off[d] + i];
        if (cnt < 2 && g->n[d] >= 2)
            for (int64_t i = 0; i < g->n[d]; ++i) keep[off[d] + i] = 1;
        int64_t next = 0;
        for (int64_t i = 0; i < g->n[d]; ++i) keep[off[d] + i] = keep[off[d] + i] ? (int32_t)next++ : -1;
        new_n[d] = next;
    }
    for (int64_t k = 0; k < nv; ++k) {
        const int64_t j = m[k];
        const int64_t a = keep[off[0] + j % n0], b = keep[off[1] + (j / n0) % n1], c = keep[off[2] + j / (n0 * n1)];
        m_out[k] = (int32_t)(a + new_n[0] * (b + new_n[1] * c));
    }
}
