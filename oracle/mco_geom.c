/*
 * mco_geom.c -- oracle geometry: grid description, point location,
 * barycentric resampling f (mesh -> grid) and multilinear back-interpolation
 * g (grid -> mesh).
 *
 * TEST INFRASTRUCTURE (see mco.h).  Plain loops, no acceleration beyond the
 * per-cell bounding-box filter of mco_locate_raster, which is checked
 * against the brute-force definition mco_locate_brute by the tests.
 */
#include "mco.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Bounding box of the vertex coordinates (Alg. 1 takes the grid corners
 * from the minimum and maximum vertex coordinate along each axis). */
void mco_bbox(const float* coords, int dim, int64_t nv, float lo[3], float hi[3])
{
    for (int d = 0; d < 3; ++d) { lo[d] = 0.0f; hi[d] = 0.0f; }
    for (int d = 0; d < dim; ++d) {
        float a = coords[(int64_t)d * nv], b = a;
        for (int64_t i = 1; i < nv; ++i) {
            float c = coords[(int64_t)d * nv + i];
            if (c < a) a = c;
            if (c > b) b = c;
        }
        lo[d] = a;
        hi[d] = b;
    }
}

/* Grid spanning the vertex bounding box with the given number of nodes per
 * axis: origin = box minimum, spacing = extent / (n - 1). */
int mco_grid_from_dims(const float* coords, int dim, int64_t nv, const int64_t dims[3],
                       mco_grid* g)
{
    if ((dim != 2 && dim != 3) || nv <= 0) return MCO_ERR_ARG;
    float lo[3], hi[3];
    mco_bbox(coords, dim, nv, lo, hi);
    memset(g, 0, sizeof *g);
    g->dim = dim;
    for (int d = 0; d < 3; ++d) {
        if (d < dim) {
            if (dims[d] < 2 || !(hi[d] > lo[d])) return MCO_ERR_ARG;
            g->n[d] = dims[d];
            g->o[d] = (double)lo[d];
            g->h[d] = ((double)hi[d] - (double)lo[d]) / (double)(dims[d] - 1);
        } else {
            g->n[d] = 1;
            g->o[d] = 0.0;
            g->h[d] = 1.0;
        }
    }
    return MCO_OK;
}

/* Node coordinate in FP32: y = (float)o + (float)i * (float)h. */
void mco_grid_node(const mco_grid* g, int64_t j, float y[3])
{
    int64_t i0 = j % g->n[0];
    int64_t i1 = (j / g->n[0]) % g->n[1];
    int64_t i2 = j / (g->n[0] * g->n[1]);
    int64_t ii[3] = {i0, i1, i2};
    for (int d = 0; d < 3; ++d) {
        if (d < g->dim)
            y[d] = (float)g->o[d] + (float)ii[d] * (float)g->h[d];
        else
            y[d] = 0.0f;
    }
}

static float fmax4(float a, float b, float c, float d)
{
    float m = a;
    if (b > m) m = b;
    if (c > m) m = c;
    if (d > m) m = d;
    return m;
}

/* Barycentric coordinates of y in the simplex verts[(dim+1)*dim] (vertex
 * k at verts[k*dim .. k*dim+dim-1]).
 *
 * Triangle (a,b,c): e1 = b-a, e2 = c-a, q = y-a,
 *   det = e1x*e2y - e2x*e1y, lb = (qx*e2y - e2x*qy)/det,
 *   lc = (e1x*qy - qx*e1y)/det, la = (1 - lb) - lc.
 * Tetrahedron (a,b,c,d): e3 = d-a, m = e2 x e3, det = e1.m,
 *   lb = q.m/det, lc = e1.(q x e3)/det, ld = e1.(e2 x q)/det,
 *   la = ((1 - lb) - lc) - ld, dot products summed (x + y) + z.
 * Evaluated in FP32.  Near-degenerate cells -- |det| <= 2^-10 * L^dim with
 * L the largest absolute edge-vector component -- are recomputed from the
 * exact double conversion of the coordinates with the same formulas in
 * FP64; the inside test then uses the FP64 values, which are rounded to
 * FP32 for storage.  A zero FP64 determinant never contains a point.
 * Inside: min_k lambda_k >= -2^-20.  Returns 1 if inside. */
int mco_bary(int dim, const float* verts, const float* y, float* lam, int* near_degenerate)
{
    const float tol = -0x1p-20f;
    *near_degenerate = 0;
    if (dim == 2) {
        const float *a = verts, *b = verts + 2, *c = verts + 4;
        float e1x = b[0] - a[0], e1y = b[1] - a[1];
        float e2x = c[0] - a[0], e2y = c[1] - a[1];
        float qx = y[0] - a[0], qy = y[1] - a[1];
        float det = e1x * e2y - e2x * e1y;
        float L = fmax4(fabsf(e1x), fabsf(e1y), fabsf(e2x), fabsf(e2y));
        if (fabsf(det) <= 0x1p-10f * (L * L)) {
            *near_degenerate = 1;
            double E1x = (double)b[0] - (double)a[0], E1y = (double)b[1] - (double)a[1];
            double E2x = (double)c[0] - (double)a[0], E2y = (double)c[1] - (double)a[1];
            double Qx = (double)y[0] - (double)a[0], Qy = (double)y[1] - (double)a[1];
            double D = E1x * E2y - E2x * E1y;
            if (D == 0.0) { lam[0] = lam[1] = lam[2] = 0.0f; return 0; }
            double lb = (Qx * E2y - E2x * Qy) / D;
            double lc = (E1x * Qy - Qx * E1y) / D;
            double la = (1.0 - lb) - lc;
            lam[0] = (float)la; lam[1] = (float)lb; lam[2] = (float)lc;
            double mn = la;
            if (lb < mn) mn = lb;
            if (lc < mn) mn = lc;
            return mn >= -0x1p-20;
        }
        float lb = (qx * e2y - e2x * qy) / det;
        float lc = (e1x * qy - qx * e1y) / det;
        float la = (1.0f - lb) - lc;
        lam[0] = la; lam[1] = lb; lam[2] = lc;
        float mn = la;
        if (lb < mn) mn = lb;
        if (lc < mn) mn = lc;
        return mn >= tol;
    }
    const float *a = verts, *b = verts + 3, *c = verts + 6, *d = verts + 9;
    float e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
    float e2x = c[0] - a[0], e2y = c[1] - a[1], e2z = c[2] - a[2];
    float e3x = d[0] - a[0], e3y = d[1] - a[1], e3z = d[2] - a[2];
    float qx = y[0] - a[0], qy = y[1] - a[1], qz = y[2] - a[2];
    float mx = e2y * e3z - e2z * e3y;
    float my = e2z * e3x - e2x * e3z;
    float mz = e2x * e3y - e2y * e3x;
    float det = (e1x * mx + e1y * my) + e1z * mz;
    float L = fmax4(fmax4(fabsf(e1x), fabsf(e1y), fabsf(e1z), fabsf(e2x)),
                    fmax4(fabsf(e2y), fabsf(e2z), fabsf(e3x), fabsf(e3y)), fabsf(e3z), 0.0f);
    if (fabsf(det) <= 0x1p-10f * ((L * L) * L)) {
        *near_degenerate = 1;
        double E1x = (double)b[0] - (double)a[0], E1y = (double)b[1] - (double)a[1],
               E1z = (double)b[2] - (double)a[2];
        double E2x = (double)c[0] - (double)a[0], E2y = (double)c[1] - (double)a[1],
               E2z = (double)c[2] - (double)a[2];
        double E3x = (double)d[0] - (double)a[0], E3y = (double)d[1] - (double)a[1],
               E3z = (double)d[2] - (double)a[2];
        double Qx = (double)y[0] - (double)a[0], Qy = (double)y[1] - (double)a[1],
               Qz = (double)y[2] - (double)a[2];
        double Mx = E2y * E3z - E2z * E3y;
        double My = E2z * E3x - E2x * E3z;
        double Mz = E2x * E3y - E2y * E3x;
        double D = (E1x * Mx + E1y * My) + E1z * Mz;
        if (D == 0.0) { lam[0] = lam[1] = lam[2] = lam[3] = 0.0f; return 0; }
        double Nx = Qy * E3z - Qz * E3y, Ny = Qz * E3x - Qx * E3z, Nz = Qx * E3y - Qy * E3x;
        double Kx = E2y * Qz - E2z * Qy, Ky = E2z * Qx - E2x * Qz, Kz = E2x * Qy - E2y * Qx;
        double lb = ((Qx * Mx + Qy * My) + Qz * Mz) / D;
        double lc = ((E1x * Nx + E1y * Ny) + E1z * Nz) / D;
        double ld = ((E1x * Kx + E1y * Ky) + E1z * Kz) / D;
        double la = ((1.0 - lb) - lc) - ld;
        lam[0] = (float)la; lam[1] = (float)lb; lam[2] = (float)lc; lam[3] = (float)ld;
        double mn = la;
        if (lb < mn) mn = lb;
        if (lc < mn) mn = lc;
        if (ld < mn) mn = ld;
        return mn >= -0x1p-20;
    }
    float nx = qy * e3z - qz * e3y, ny = qz * e3x - qx * e3z, nz = qx * e3y - qy * e3x;
    float kx = e2y * qz - e2z * qy, ky = e2z * qx - e2x * qz, kz = e2x * qy - e2y * qx;
    float lb = ((qx * mx + qy * my) + qz * mz) / det;
    float lc = ((e1x * nx + e1y * ny) + e1z * nz) / det;
    float ld = ((e1x * kx + e1y * ky) + e1z * kz) / det;
    float la = ((1.0f - lb) - lc) - ld;
    lam[0] = la; lam[1] = lb; lam[2] = lc; lam[3] = ld;
    float mn = la;
    if (lb < mn) mn = lb;
    if (lc < mn) mn = lc;
    if (ld < mn) mn = ld;
    return mn >= tol;
}

static void gather_cell(const float* coords, const int32_t* cells, int dim, int64_t nv,
                        int64_t nc, int64_t c, float* verts)
{
    for (int k = 0; k <= dim; ++k) {
        int32_t v = cells[(int64_t)k * nc + c];
        for (int d = 0; d < dim; ++d) verts[k * dim + d] = coords[(int64_t)d * nv + v];
    }
}

static void store_hit(int dim, int64_t ng, int64_t j, const int32_t* cells, int64_t nc,
                      int64_t c, const float* lam, int32_t* cell_of_node, int32_t* vid,
                      float* w)
{
    cell_of_node[j] = (int32_t)c;
    for (int k = 0; k <= dim; ++k) {
        vid[(int64_t)k * ng + j] = cells[(int64_t)k * nc + c];
        w[(int64_t)k * ng + j] = lam[k];
    }
}

static int64_t grid_count(const mco_grid* g) { return g->n[0] * g->n[1] * g->n[2]; }

/* Point location by definition: every grid node is tested against every
 * cell; the chosen cell is the lowest cell id whose barycentric test
 * passes.  Unlocated nodes get cell -1, vid -1, w 0.  Returns the number of
 * unlocated nodes. */
int64_t mco_locate_brute(const float* coords, const int32_t* cells, int dim, int64_t nv,
                         int64_t nc, const mco_grid* g, int32_t* cell_of_node,
                         int32_t* vid, float* w)
{
    int64_t ng = grid_count(g), unresolved = 0;
    float verts[12], lam[4], y[3];
    for (int64_t j = 0; j < ng; ++j) {
        mco_grid_node(g, j, y);
        cell_of_node[j] = -1;
        for (int k = 0; k <= dim; ++k) { vid[(int64_t)k * ng + j] = -1; w[(int64_t)k * ng + j] = 0.0f; }
        for (int64_t c = 0; c < nc; ++c) {
            int nd;
            gather_cell(coords, cells, dim, nv, nc, c, verts);
            if (mco_bary(dim, verts, y, lam, &nd)) {
                store_hit(dim, ng, j, cells, nc, c, lam, cell_of_node, vid, w);
                break;
            }
        }
        if (cell_of_node[j] < 0) ++unresolved;
    }
    return unresolved;
}

/* The same result as mco_locate_brute, visiting cells in ascending id and
 * testing only the nodes inside the cell's bounding box widened by L/8 (L =
 * largest absolute edge-vector component).  A node that passes the
 * barycentric test lies within the box widened by (dim+1) * 2^-20 * L plus
 * rounding, far inside that margin.  A node keeps the first (lowest-id)
 * cell that contains it. */
int64_t mco_locate_raster(const float* coords, const int32_t* cells, int dim, int64_t nv,
                          int64_t nc, const mco_grid* g, int32_t* cell_of_node,
                          int32_t* vid, float* w)
{
    int64_t ng = grid_count(g);
    for (int64_t j = 0; j < ng; ++j) {
        cell_of_node[j] = -1;
        for (int k = 0; k <= dim; ++k) { vid[(int64_t)k * ng + j] = -1; w[(int64_t)k * ng + j] = 0.0f; }
    }
    float verts[12], lam[4], y[3];
    for (int64_t c = 0; c < nc; ++c) {
        gather_cell(coords, cells, dim, nv, nc, c, verts);
        float L = 0.0f;
        for (int k = 1; k <= dim; ++k)
            for (int d = 0; d < dim; ++d) {
                float e = fabsf(verts[k * dim + d] - verts[d]);
                if (e > L) L = e;
            }
        int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        int empty = 0;
        for (int d = 0; d < dim; ++d) {
            double mn = verts[d], mx = verts[d];
            for (int k = 1; k <= dim; ++k) {
                double v = verts[k * dim + d];
                if (v < mn) mn = v;
                if (v > mx) mx = v;
            }
            double m = 0.125 * (double)L;
            double a = ceil((mn - m - g->o[d]) / g->h[d]);
            double b = floor((mx + m - g->o[d]) / g->h[d]);
            if (a < 0) a = 0;
            if (b > (double)(g->n[d] - 1)) b = (double)(g->n[d] - 1);
            if (a > b) empty = 1;
            lo[d] = (int64_t)a;
            hi[d] = (int64_t)b;
        }
        if (empty) continue;
        for (int64_t i2 = lo[2]; i2 <= hi[2]; ++i2)
            for (int64_t i1 = lo[1]; i1 <= hi[1]; ++i1)
                for (int64_t i0 = lo[0]; i0 <= hi[0]; ++i0) {
                    int64_t j = i0 + g->n[0] * (i1 + g->n[1] * i2);
                    if (cell_of_node[j] >= 0) continue;
                    int nd;
                    mco_grid_node(g, j, y);
                    if (mco_bary(dim, verts, y, lam, &nd))
                        store_hit(dim, ng, j, cells, nc, c, lam, cell_of_node, vid, w);
                }
    }
    int64_t unresolved = 0;
    for (int64_t j = 0; j < ng; ++j) unresolved += cell_of_node[j] < 0;
    return unresolved;
}

/* Grid nodes outside every cell (hollow regions, outside the hull; Fig. 1
 * of the paper fills holes with a constant).  nearest != 0: the node takes
 * the value of the vertex with the smallest FP32 squared distance
 * ((dx*dx + dy*dy) + dz*dz), lowest vertex id on ties, encoded as weights
 * (1, 0, ..) on that vertex.  nearest == 0: vid stays -1 and the resampler
 * writes the mid-range value c. */
void mco_fill_unresolved(const float* coords, int dim, int64_t nv, const mco_grid* g,
                         const int32_t* cell_of_node, int nearest, int32_t* vid, float* w)
{
    int64_t ng = grid_count(g);
    float y[3];
    for (int64_t j = 0; j < ng; ++j) {
        if (cell_of_node[j] >= 0) continue;
        if (!nearest) {
            for (int k = 0; k <= dim; ++k) { vid[(int64_t)k * ng + j] = -1; w[(int64_t)k * ng + j] = 0.0f; }
            continue;
        }
        mco_grid_node(g, j, y);
        int64_t best = -1;
        float bd = 0.0f;
        for (int64_t v = 0; v < nv; ++v) {
            float dx = coords[v] - y[0];
            float dy = coords[nv + v] - y[1];
            float dd = dx * dx + dy * dy;
            if (dim == 3) {
                float dz = coords[2 * nv + v] - y[2];
                dd = dd + dz * dz;
            }
            if (best < 0 || dd < bd) { best = v; bd = dd; }
        }
        for (int k = 0; k <= dim; ++k) {
            vid[(int64_t)k * ng + j] = (int32_t)best;
            w[(int64_t)k * ng + j] = k == 0 ? 1.0f : 0.0f;
        }
    }
}

/* Nearest-vertex fill of selected nodes (Sec. 8 reading of Fig. 1: a node
 * outside every cell takes the value of its nearest vertex), the same FP32
 * metric and lowest-id tie-break as mco_fill_unresolved, each node's
 * minimum taken over its own candidate vertices only:
 * cand[cand_ptr[i] .. cand_ptr[i+1]) for node nodes[i].  Equal to the
 * definition whenever every candidate list holds all vertices that can
 * attain that node's minimum.  Writes vid/w of the full grid arrays
 * (k * ng + node). */
void mco_fill_candidates(const float* coords, int dim, int64_t nv, const mco_grid* g, const int64_t* nodes,
                         int64_t nn, const int64_t* cand_ptr, const int32_t* cand, int32_t* vid, float* w)
{
    int64_t ng = grid_count(g);
    float y[3];
    for (int64_t i = 0; i < nn; ++i) {
        int64_t j = nodes[i];
        mco_grid_node(g, j, y);
        int64_t best = -1;
        float bd = 0.0f;
        for (int64_t k = cand_ptr[i]; k < cand_ptr[i + 1]; ++k) {
            int64_t v = cand[k];
            float dx = coords[v] - y[0];
            float dy = coords[nv + v] - y[1];
            float dd = dx * dx + dy * dy;
            if (dim == 3) {
                float dz = coords[2 * nv + v] - y[2];
                dd = dd + dz * dz;
            }
            if (best < 0 || dd < bd || (dd == bd && v < best)) { best = v; bd = dd; }
        }
        for (int k = 0; k <= dim; ++k) {
            vid[(int64_t)k * ng + j] = (int32_t)best;
            w[(int64_t)k * ng + j] = k == 0 ? 1.0f : 0.0f;
        }
    }
}

/* Point location of selected grid nodes (the definition above, restricted):
 * node nodes[i] is tested against the cells cand[i * ncand .. + ncand - 1]
 * (cell ids, ascending; -1 entries are skipped), takes the lowest id that
 * contains it, and otherwise the nearest-vertex fill (nearest != 0) or the
 * mid-range marker.  Exact when the caller's candidate set holds every cell
 * that can contain the node.  Outputs per listed node: cell_out[i],
 * vid_out[k * nn + i], w_out[k * nn + i]. */
void mco_locate_nodes(const float* coords, const int32_t* cells, int dim, int64_t nv, int64_t nc,
                      const mco_grid* g, const int64_t* nodes, int64_t nn, const int32_t* cand, int ncand,
                      int nearest, int32_t* cell_out, int32_t* vid_out, float* w_out)
{
    float y[3], verts[12], lam[4];
    for (int64_t i = 0; i < nn; ++i) {
        const int64_t j = nodes[i];
        mco_grid_node(g, j, y);
        int32_t hit = -1;
        for (int q = 0; q < ncand && hit < 0; ++q) {
            const int32_t c = cand[i * ncand + q];
            if (c < 0 || c >= nc) continue;
            gather_cell(coords, cells, dim, nv, nc, c, verts);
            int nd = 0;
            if (mco_bary(dim, verts, y, lam, &nd)) {
                hit = c;
                for (int k = 0; k <= dim; ++k) {
                    vid_out[k * nn + i] = cells[(int64_t)k * nc + c];
                    w_out[k * nn + i] = lam[k];
                }
            }
        }
        cell_out[i] = hit;
        if (hit >= 0) continue;
        int64_t best = -1;
        float bd = 0.0f;
        if (nearest)
            for (int64_t v = 0; v < nv; ++v) {
                float dx = coords[v] - y[0];
                float dy = coords[nv + v] - y[1];
                float dd = dx * dx + dy * dy;
                if (dim == 3) {
                    float dz = coords[2 * nv + v] - y[2];
                    dd = dd + dz * dz;
                }
                if (best < 0 || dd < bd) { best = v; bd = dd; }
            }
        for (int k = 0; k <= dim; ++k) {
            vid_out[k * nn + i] = (int32_t)best;
            w_out[k * nn + i] = (nearest && k == 0) ? 1.0f : 0.0f;
        }
    }
}

static float field_as_float(const void* x, int dtype, int64_t i)
{
    return dtype == MCO_F64 ? (float)((const double*)x)[i] : ((const float*)x)[i];
}

/* f: mesh -> grid.  v_j = ((w0*f0 + w1*f1) + w2*f2) [+ w3*f3] in FP32 with
 * f_k = (float)x[vid_k]; an unlocated node in mid-range mode (vid -1) takes
 * (float)c. */
void mco_resample(const int32_t* vid, const float* w, int dim, int64_t ng, const void* x,
                  int dtype, double c, float* v)
{
    for (int64_t j = 0; j < ng; ++j) {
        if (vid[j] < 0) { v[j] = (float)c; continue; }
        float acc = w[j] * field_as_float(x, dtype, vid[j]);
        for (int k = 1; k <= dim; ++k)
            acc = acc + w[(int64_t)k * ng + j] * field_as_float(x, dtype, vid[(int64_t)k * ng + j]);
        v[j] = acc;
    }
}

/* Grid cell and in-cell offset of vertex v: u = (P - (float)o) * (float)(1/h),
 * i = clamp(floor(u), 0, n-2), t = clamp(u - i, 0, 1), all FP32. */
void mco_vertex_cell(const float* coords, int dim, int64_t nv, const mco_grid* g,
                     int64_t v, int32_t idx[3], float t[3])
{
    for (int d = 0; d < 3; ++d) { idx[d] = 0; t[d] = 0.0f; }
    for (int d = 0; d < dim; ++d) {
        float of = (float)g->o[d];
        float ihf = (float)(1.0 / g->h[d]);
        float u = (coords[(int64_t)d * nv + v] - of) * ihf;
        float fl = floorf(u);
        int64_t i;
        if (fl < 0.0f) i = 0;
        else if (fl > (float)(g->n[d] - 2)) i = g->n[d] - 2;
        else i = (int64_t)fl;
        float tt = u - (float)i;
        if (tt < 0.0f) tt = 0.0f;
        if (tt > 1.0f) tt = 1.0f;
        idx[d] = (int32_t)i;
        t[d] = tt;
    }
}

static float lerp(float a, float b, float t) { return (1.0f - t) * a + t * b; }

/* g: grid -> mesh, multilinear interpolation of the reconstructed grid at
 * each vertex: lerp along x on the 2^(dim-1) cell edges, then along y, then
 * along z, lerp(a, b, t) = (1 - t)*a + t*b in FP32.  The 2^dim weights are
 * non-negative and sum to one (the piece-wise linear case of Sec. III). */
void mco_back_interp(const float* coords, int dim, int64_t nv, const mco_grid* g,
                     const float* xhat, float* gv)
{
    int64_t n0 = g->n[0], n01 = g->n[0] * g->n[1];
    for (int64_t v = 0; v < nv; ++v) {
        int32_t idx[3];
        float t[3];
        mco_vertex_cell(coords, dim, nv, g, v, idx, t);
        int64_t j = idx[0] + n0 * idx[1] + n01 * idx[2];
        float c00 = lerp(xhat[j], xhat[j + 1], t[0]);
        float c10 = lerp(xhat[j + n0], xhat[j + n0 + 1], t[0]);
        float c0 = lerp(c00, c10, t[1]);
        if (dim == 2) { gv[v] = c0; continue; }
        float c01 = lerp(xhat[j + n01], xhat[j + n01 + 1], t[0]);
        float c11 = lerp(xhat[j + n01 + n0], xhat[j + n01 + n0 + 1], t[0]);
        float c1 = lerp(c01, c11, t[1]);
        gv[v] = lerp(c0, c1, t[2]);
    }
}
