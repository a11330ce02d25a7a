// k_plan.hip -- field-independent plan on gfx950: the reusable mesh-grid
// mapping of the paper (Sec. IV-B/IV-C), here barycentric weights of every
// grid node in the lowest-numbered cell that contains it.
//   k_bbox            vertex bounding box (ordered-integer keys)
//   k_bins_count/fill uniform bin index in grid-index space: every cell is
//                     listed in the bins its bounding box (widened by 1/8 of
//                     its largest edge component) overlaps
//   k_scan            exclusive scan of counts (decoupled look-back)
//   k_locate          per node: barycentric test against the candidates of
//                     its bin, lowest containing cell id wins; FP64 recompute
//                     for near-degenerate cells
//   k_vbins_*         vertex bins for the nearest-vertex fill
//   k_fill_nearest    unlocated nodes: nearest vertex by a ring search over
//                     vertex bins with a conservative stopping distance
#include "mc_dev.h"
#include "mc_kernels.h"

__device__ __forceinline__ unsigned fkey(float f)
{
    unsigned b = __float_as_uint(f);
    if (f == 0.0f) b = 0u;
    return (b >> 31) ? ~b : (b | 0x80000000u);
}

__global__ __launch_bounds__(256) void k_bbox(const float* __restrict__ coords, int dim, long long nv,
                                              unsigned int* __restrict__ keys)
{
    for (int d = 0; d < dim; ++d) {
        unsigned mn = ~0u, mx = 0u;
        for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < nv; i += (long long)gridDim.x * 256) {
            const unsigned k = fkey(coords[(long long)d * nv + i]);
            mn = k < mn ? k : mn;
            mx = k > mx ? k : mx;
        }
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            const unsigned a = __shfl_xor(mn, s, 64), b = __shfl_xor(mx, s, 64);
            mn = a < mn ? a : mn;
            mx = b > mx ? b : mx;
        }
        if (lane_id() == 0) {
            atomicMin(&keys[2 * d], mn);
            atomicMax(&keys[2 * d + 1], mx);
        }
    }
}

// Node index range covered by a cell's widened bounding box along one axis.
struct CellBox {
    int lo[3], hi[3];
    bool empty;
};

template <int D>
__device__ __forceinline__ CellBox cell_box(const float* __restrict__ coords, const int32_t* __restrict__ cells,
                                            long long nv, long long nc, long long c, const GridGeom& gg,
                                            const double* o, const double* h, bool& bad)
{
    CellBox cb;
    int vv[D + 1];
    bad = false;
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        vv[k] = cells[k * nc + c];
        if (vv[k] < 0 || vv[k] >= nv) bad = true;
    }
    cb.empty = true;
    if (bad) return cb;
    float mn[D], mx[D], a[D];
    float L = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        a[d] = coords[d * nv + vv[0]];
        mn[d] = a[d];
        mx[d] = a[d];
    }
#pragma unroll
    for (int k = 1; k <= D; ++k)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float q = coords[d * nv + vv[k]];
            mn[d] = fminf(mn[d], q);
            mx[d] = fmaxf(mx[d], q);
            L = fmaxf(L, fabsf(q - a[d]));
        }
    const double m = 0.125 * (double)L;
    const int nn[3] = {gg.n0, gg.n1, gg.n2};
    cb.empty = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d >= D) { cb.lo[d] = 0; cb.hi[d] = 0; continue; }
        double lo = ceil(((double)mn[d] - m - o[d]) / h[d]);
        double hi = floor(((double)mx[d] + m - o[d]) / h[d]);
        if (lo < 0.0) lo = 0.0;
        if (hi > (double)(nn[d] - 1)) hi = (double)(nn[d] - 1);
        if (lo > hi) cb.empty = true;
        cb.lo[d] = (int)lo;
        cb.hi[d] = (int)hi;
    }
    return cb;
}

struct Dd3 { double o[3], h[3]; };

template <int D>
__global__ __launch_bounds__(256) void k_bins_count(const float* __restrict__ coords, const int32_t* __restrict__ cells,
                                                    long long nv, long long nc, GridGeom gg, Dd3 oh, int B, int nb0,
                                                    int nb1, unsigned int* __restrict__ cnt,
                                                    unsigned int* __restrict__ bad_cells)
{
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    bool bad;
    const CellBox cb = cell_box<D>(coords, cells, nv, nc, c, gg, oh.o, oh.h, bad);
    if (bad) { atomicAdd(bad_cells, 1u); return; }
    if (cb.empty) return;
    for (int b2 = cb.lo[2] / B; b2 <= cb.hi[2] / B; ++b2)
        for (int b1 = cb.lo[1] / B; b1 <= cb.hi[1] / B; ++b1)
            for (int b0 = cb.lo[0] / B; b0 <= cb.hi[0] / B; ++b0)
                atomicAdd(&cnt[b0 + (long long)nb0 * (b1 + (long long)nb1 * b2)], 1u);
}

template <int D>
__global__ __launch_bounds__(256) void k_bins_fill(const float* __restrict__ coords, const int32_t* __restrict__ cells,
                                                   long long nv, long long nc, GridGeom gg, Dd3 oh, int B, int nb0,
                                                   int nb1, const long long* __restrict__ start,
                                                   unsigned int* __restrict__ cursor, int32_t* __restrict__ list)
{
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    bool bad;
    const CellBox cb = cell_box<D>(coords, cells, nv, nc, c, gg, oh.o, oh.h, bad);
    if (bad || cb.empty) return;
    for (int b2 = cb.lo[2] / B; b2 <= cb.hi[2] / B; ++b2)
        for (int b1 = cb.lo[1] / B; b1 <= cb.hi[1] / B; ++b1)
            for (int b0 = cb.lo[0] / B; b0 <= cb.hi[0] / B; ++b0) {
                const long long b = b0 + (long long)nb0 * (b1 + (long long)nb1 * b2);
                const unsigned k = atomicAdd(&cursor[b], 1u);
                list[start[b] + k] = (int32_t)c;
            }
}

// Exclusive scan of n counts into out[0..n] (out[n] = total), 4096 per tile,
// 16 consecutive values per thread.
__global__ __launch_bounds__(256) void k_scan(const unsigned int* __restrict__ in, long long n,
                                              long long* __restrict__ out, unsigned long long* __restrict__ st,
                                              unsigned int* __restrict__ ticket, long long ntiles)
{
    __shared__ long long s_slot;
    __shared__ long long s_w[4];
    const long long tile = take_ticket(ticket, &s_slot);
    const long long base = tile * MC_TILE + (long long)threadIdx.x * MC_IPT;
    long long v[MC_IPT];
    long long run = 0;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        v[i] = (base + i < n) ? (long long)in[base + i] : 0;
        run += v[i];
    }
    const long long inc = wave_incl_scan(run);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) s_w[w] = inc;
    __syncthreads();
    long long off = 0;
    for (int k = 0; k < w; ++k) off += s_w[k];
    const long long ttot = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
    const long long excl = (long long)tile_prefix(st, tile, (unsigned long long)ttot, &s_slot);
    long long acc = excl + off + inc - run;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (base + i < n) out[base + i] = acc;
        acc += v[i];
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) out[n] = excl + ttot;
}

// Barycentric coordinates of node y in cell (FP32; FP64 recompute when
// |det| <= 2^-10 L^D with L the largest absolute edge-vector component).
// Triangle: det = e1x*e2y - e2x*e1y, lb = (qx*e2y - e2x*qy)/det,
// lc = (e1x*qy - qx*e1y)/det, la = (1 - lb) - lc.  Tetrahedron: m = e2 x e3,
// det = e1.m, lb = q.m/det, lc = e1.(q x e3)/det, ld = e1.(e2 x q)/det,
// la = ((1 - lb) - lc) - ld; dot products summed (x + y) + z.  Inside iff the
// smallest coordinate is >= -2^-20 (in the precision it was computed in).
template <typename F>
__device__ __forceinline__ bool bary2(const F* a, const F* b, const F* c, const F* y, F* lam)
{
    const F e1x = b[0] - a[0], e1y = b[1] - a[1];
    const F e2x = c[0] - a[0], e2y = c[1] - a[1];
    const F qx = y[0] - a[0], qy = y[1] - a[1];
    const F det = e1x * e2y - e2x * e1y;
    if (det == (F)0) return false;
    const F lb = (qx * e2y - e2x * qy) / det;
    const F lc = (e1x * qy - qx * e1y) / det;
    const F la = ((F)1 - lb) - lc;
    lam[0] = la; lam[1] = lb; lam[2] = lc;
    F mnv = la < lb ? la : lb;
    mnv = mnv < lc ? mnv : lc;
    return mnv >= (F)(-0x1p-20);
}

template <typename F>
__device__ __forceinline__ bool bary3(const F* a, const F* b, const F* c, const F* d, const F* y, F* lam)
{
    const F e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
    const F e2x = c[0] - a[0], e2y = c[1] - a[1], e2z = c[2] - a[2];
    const F e3x = d[0] - a[0], e3y = d[1] - a[1], e3z = d[2] - a[2];
    const F qx = y[0] - a[0], qy = y[1] - a[1], qz = y[2] - a[2];
    const F mx = e2y * e3z - e2z * e3y, my = e2z * e3x - e2x * e3z, mz = e2x * e3y - e2y * e3x;
    const F det = (e1x * mx + e1y * my) + e1z * mz;
    if (det == (F)0) return false;
    const F nx = qy * e3z - qz * e3y, ny = qz * e3x - qx * e3z, nz = qx * e3y - qy * e3x;
    const F kx = e2y * qz - e2z * qy, ky = e2z * qx - e2x * qz, kz = e2x * qy - e2y * qx;
    const F lb = ((qx * mx + qy * my) + qz * mz) / det;
    const F lc = ((e1x * nx + e1y * ny) + e1z * nz) / det;
    const F ld = ((e1x * kx + e1y * ky) + e1z * kz) / det;
    const F la = (((F)1 - lb) - lc) - ld;
    lam[0] = la; lam[1] = lb; lam[2] = lc; lam[3] = ld;
    F mnv = la < lb ? la : lb;
    mnv = mnv < lc ? mnv : lc;
    mnv = mnv < ld ? mnv : ld;
    return mnv >= (F)(-0x1p-20);
}

template <int D>
__device__ __forceinline__ bool near_degenerate(const float (*P)[3])
{
    float L = 0.0f;
#pragma unroll
    for (int k = 1; k <= D; ++k)
#pragma unroll
        for (int d = 0; d < D; ++d) L = fmaxf(L, fabsf(P[k][d] - P[0][d]));
    float det;
    if (D == 2) {
        const float e1x = P[1][0] - P[0][0], e1y = P[1][1] - P[0][1];
        const float e2x = P[2][0] - P[0][0], e2y = P[2][1] - P[0][1];
        det = e1x * e2y - e2x * e1y;
        return fabsf(det) <= 0x1p-10f * (L * L);
    } else {
        const float e1x = P[1][0] - P[0][0], e1y = P[1][1] - P[0][1], e1z = P[1][2] - P[0][2];
        const float e2x = P[2][0] - P[0][0], e2y = P[2][1] - P[0][1], e2z = P[2][2] - P[0][2];
        const float e3x = P[3][0] - P[0][0], e3y = P[3][1] - P[0][1], e3z = P[3][2] - P[0][2];
        const float mx = e2y * e3z - e2z * e3y, my = e2z * e3x - e2x * e3z, mz = e2x * e3y - e2y * e3x;
        det = (e1x * mx + e1y * my) + e1z * mz;
        return fabsf(det) <= 0x1p-10f * ((L * L) * L);
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_locate(const float* __restrict__ coords, const int32_t* __restrict__ cells,
                                                long long nv, long long nc, GridGeom gg, int B, int nb0, int nb1,
                                                const long long* __restrict__ start, const int32_t* __restrict__ list,
                                                int32_t* __restrict__ vid, float* __restrict__ w,
                                                int32_t* __restrict__ cell_out, int32_t* __restrict__ unres,
                                                unsigned int* __restrict__ n_unres,
                                                unsigned int* __restrict__ n_neardeg)
{
    const long long ng = (long long)gg.n0 * gg.n1 * gg.n2;
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (j >= ng) return;
    const int i0 = (int)(j % gg.n0);
    const long long r = j / gg.n0;
    const int i1 = (int)(r % gg.n1);
    const int i2 = (int)(r / gg.n1);
    float y[3];
    y[0] = gg.of[0] + (float)i0 * gg.hf[0];
    y[1] = gg.of[1] + (float)i1 * gg.hf[1];
    y[2] = D == 3 ? gg.of[2] + (float)i2 * gg.hf[2] : 0.0f;
    const long long b = (i0 / B) + (long long)nb0 * ((i1 / B) + (long long)nb1 * (i2 / B));
    const long long s0 = start[b], s1 = start[b + 1];
    int best = 0x7fffffff;
    float lam_best[4] = {0.f, 0.f, 0.f, 0.f};
    bool best_nd = false;
    for (long long k = s0; k < s1; ++k) {
        const int c = list[k];
        if (c >= best) continue;
        float P[D + 1][3];
#pragma unroll
        for (int q = 0; q <= D; ++q) {
            const int v = cells[q * nc + c];
#pragma unroll
            for (int d = 0; d < 3; ++d) P[q][d] = d < D ? coords[d * nv + v] : 0.0f;
        }
        const bool nd = near_degenerate<D>(P);
        bool inside;
        float lam[4];
        if (!nd) {
            if (D == 2) inside = bary2<float>(P[0], P[1], P[2], y, lam);
            else inside = bary3<float>(P[0], P[1], P[2], P[3], y, lam);
        } else {
            double Q[D + 1][3], Y[3] = {(double)y[0], (double)y[1], (double)y[2]}, L64[4];
#pragma unroll
            for (int q = 0; q <= D; ++q)
#pragma unroll
                for (int d = 0; d < 3; ++d) Q[q][d] = (double)P[q][d];
            if (D == 2) inside = bary2<double>(Q[0], Q[1], Q[2], Y, L64);
            else inside = bary3<double>(Q[0], Q[1], Q[2], Q[3], Y, L64);
#pragma unroll
            for (int q = 0; q <= D; ++q) lam[q] = (float)L64[q];
        }
        if (inside) {
            best = c;
            best_nd = nd;
#pragma unroll
            for (int q = 0; q <= D; ++q) lam_best[q] = lam[q];
        }
    }
    const bool un = best == 0x7fffffff;
    if (un) {
        cell_out[j] = -1;
#pragma unroll
        for (int q = 0; q <= D; ++q) { vid[q * ng + j] = -1; w[q * ng + j] = 0.0f; }
    } else {
        cell_out[j] = best;
#pragma unroll
        for (int q = 0; q <= D; ++q) {
            vid[q * ng + j] = cells[q * nc + best];
            w[q * ng + j] = lam_best[q];
        }
    }
    // unresolved ids compacted per wave: one atomic reserves the wave's run
    // of the list, ballot ranks place its nodes (in ascending id within the
    // run; the fill treats every listed node on its own, so the order of the
    // runs is free); the near-degenerate count likewise one atomic per wave
    const unsigned long long mu = __ballot(un), mn = __ballot(!un && best_nd);
    if (mu) {
        const int lead = __ffsll((long long)mu) - 1;
        unsigned base = 0;
        if (lane_id() == lead) base = atomicAdd(n_unres, (unsigned)__popcll(mu));
        base = __shfl(base, lead, 64);
        if (un) unres[base + (unsigned)mbcnt64(mu)] = (int32_t)j;
    }
    if (mn && lane_id() == __ffsll((long long)mn) - 1) atomicAdd(n_neardeg, (unsigned)__popcll(mn));
}

// ---- vertex bins --------------------------------------------------------
template <int D>
__device__ __forceinline__ long long vbin_of(const float* __restrict__ coords, long long nv, long long v,
                                             const Dd3& oh, int VB, int nb0, int nb1, int nb2)
{
    const int nb[3] = {nb0, nb1, nb2};
    long long b[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double u = floor(((double)coords[d * nv + v] - oh.o[d]) / (oh.h[d] * (double)VB));
        if (u < 0.0) u = 0.0;
        if (u > (double)(nb[d] - 1)) u = (double)(nb[d] - 1);
        b[d] = (long long)u;
    }
    return b[0] + (long long)nb0 * (b[1] + (long long)nb1 * b[2]);
}

template <int D>
__global__ __launch_bounds__(256) void k_vbins_count(const float* __restrict__ coords, long long nv, Dd3 oh, int VB,
                                                     int nb0, int nb1, int nb2, unsigned int* __restrict__ cnt)
{
    const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    atomicAdd(&cnt[vbin_of<D>(coords, nv, v, oh, VB, nb0, nb1, nb2)], 1u);
}

template <int D>
__global__ __launch_bounds__(256) void k_vbins_fill(const float* __restrict__ coords, long long nv, Dd3 oh, int VB,
                                                    int nb0, int nb1, int nb2, const long long* __restrict__ start,
                                                    unsigned int* __restrict__ cursor, int32_t* __restrict__ list)
{
    const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    const long long b = vbin_of<D>(coords, nv, v, oh, VB, nb0, nb1, nb2);
    const unsigned k = atomicAdd(&cursor[b], 1u);
    list[start[b] + k] = (int32_t)v;
}

// Nearest vertex to an unlocated node: FP32 squared distance
// ((dx*dx + dy*dy) + dz*dz), ties to the lowest vertex id.  Rings of vertex
// bins (Chebyshev distance r from the node's bin) are searched until every
// unsearched vertex is provably farther: a vertex r+1 or more bins away is
// at least r*VB*h_min away along some axis (less a rounding allowance).
template <int D>
__global__ __launch_bounds__(256) void k_fill_nearest(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                      Dd3 oh, int VB, int nb0, int nb1, int nb2,
                                                      const long long* __restrict__ start,
                                                      const int32_t* __restrict__ list, const int32_t* __restrict__ unres,
                                                      long long n_unres, int32_t* __restrict__ vid,
                                                      float* __restrict__ w, long long ng, double hmin, double eps)
{
    const long long u = (long long)blockIdx.x * 256 + threadIdx.x;
    if (u >= n_unres) return;
    const long long j = unres[u];
    const int i0 = (int)(j % gg.n0);
    const long long r0 = j / gg.n0;
    const int i1 = (int)(r0 % gg.n1);
    const int i2 = (int)(r0 / gg.n1);
    float y[3];
    y[0] = gg.of[0] + (float)i0 * gg.hf[0];
    y[1] = gg.of[1] + (float)i1 * gg.hf[1];
    y[2] = D == 3 ? gg.of[2] + (float)i2 * gg.hf[2] : 0.0f;
    const int c0 = i0 / VB, c1 = i1 / VB, c2 = D == 3 ? i2 / VB : 0;
    const int rmax = max(max(nb0, nb1), nb2);
    float bd = 0.0f;
    long long bv = -1;
    for (int r = 0; r <= rmax; ++r) {
        // the ring's bins inside the bin grid only: (dz, dy) over the ring's
        // cross-section clamped to the grid; dx over the whole clamped row
        // where (dz, dy) is on the ring already, else only dx = -r and +r
        // (a ring scanned as a full cube costs (2r + 1)^3 steps, far too many
        // on a grid much finer along one axis, where many rings are needed)
        const int zr = D == 3 ? r : 0;
        const int z0 = max(-zr, -c2), z1 = min(zr, nb2 - 1 - c2);
        const int y0 = max(-r, -c1), y1 = min(r, nb1 - 1 - c1);
        const int x0 = max(-r, -c0), x1 = min(r, nb0 - 1 - c0);
        for (int dz = z0; dz <= z1; ++dz)
            for (int dy = y0; dy <= y1; ++dy) {
                const bool edge = max(abs(dy), abs(dz)) == r;
                const int xs = edge ? 1 : 2 * r;                   // step: every dx, or -r then +r
                for (int dx = edge ? x0 : -r; dx <= (edge ? x1 : r); dx += (xs > 0 ? xs : 1)) {
                    if (dx < x0 || dx > x1) continue;
                    const int b0 = c0 + dx, b1 = c1 + dy, b2 = c2 + dz;
                    const long long b = b0 + (long long)nb0 * (b1 + (long long)nb1 * b2);
                    for (long long k = start[b]; k < start[b + 1]; ++k) {
                        const long long v = list[k];
                        const float ddx = coords[v] - y[0];
                        const float ddy = coords[nv + v] - y[1];
                        float dd = ddx * ddx + ddy * ddy;
                        if (D == 3) {
                            const float ddz = coords[2 * nv + v] - y[2];
                            dd = dd + ddz * ddz;
                        }
                        if (bv < 0 || dd < bd || (dd == bd && v < bv)) { bd = dd; bv = v; }
                    }
                }
            }
        if (bv >= 0) {
            double lb = (double)r * VB * hmin - eps;
            if (lb > 0.0 && (double)bd < lb * lb * (1.0 - 1e-5)) break;
        }
    }
    for (int q = 0; q <= D; ++q) {
        vid[q * ng + j] = (int32_t)bv;
        w[q * ng + j] = q == 0 ? 1.0f : 0.0f;
    }
}

__global__ void k_fill_midrange(int dim, const int32_t* __restrict__ unres, long long n_unres,
                                int32_t* __restrict__ vid, float* __restrict__ w, long long ng)
{
    const long long u = (long long)blockIdx.x * 256 + threadIdx.x;
    if (u >= n_unres) return;
    const long long j = unres[u];
    for (int q = 0; q <= dim; ++q) { vid[q * ng + j] = -1; w[q * ng + j] = 0.0f; }
}

// ---------------------------------------------------------------------------
namespace mck {

static Dd3 mkdd(const double* o, const double* h)
{
    Dd3 r;
    for (int d = 0; d < 3; ++d) { r.o[d] = o[d]; r.h[d] = h[d]; }
    return r;
}

static dim3 blocks_for(long long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t bbox(const float* coords, int dim, long long nv, unsigned int* keys, hipStream_t s)
{
    ProfScope ps("k_bbox", s);
    long long nb = (nv + 255) / 256;
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(k_bbox, dim3((unsigned)nb), dim3(256), 0, s, coords, dim, nv, keys);
    return hipGetLastError();
}

hipError_t bins_count(const float* coords, const int32_t* cells, int dim, long long nv, long long nc, GridGeom gg,
                      const double* o, const double* h, int B, int nb0, int nb1, int nb2, unsigned int* bin_count,
                      unsigned int* bad_cells, hipStream_t s)
{
    ProfScope ps("k_bins_count", s);
    (void)nb2;
    if (dim == 2)
        hipLaunchKernelGGL(k_bins_count<2>, blocks_for(nc), dim3(256), 0, s, coords, cells, nv, nc, gg, mkdd(o, h), B,
                           nb0, nb1, bin_count, bad_cells);
    else
        hipLaunchKernelGGL(k_bins_count<3>, blocks_for(nc), dim3(256), 0, s, coords, cells, nv, nc, gg, mkdd(o, h), B,
                           nb0, nb1, bin_count, bad_cells);
    return hipGetLastError();
}

hipError_t bins_fill(const float* coords, const int32_t* cells, int dim, long long nv, long long nc, GridGeom gg,
                     const double* o, const double* h, int B, int nb0, int nb1, int nb2, const long long* bin_start,
                     unsigned int* cursor, int32_t* list, hipStream_t s)
{
    ProfScope ps("k_bins_fill", s);
    (void)nb2;
    if (dim == 2)
        hipLaunchKernelGGL(k_bins_fill<2>, blocks_for(nc), dim3(256), 0, s, coords, cells, nv, nc, gg, mkdd(o, h), B,
                           nb0, nb1, bin_start, cursor, list);
    else
        hipLaunchKernelGGL(k_bins_fill<3>, blocks_for(nc), dim3(256), 0, s, coords, cells, nv, nc, gg, mkdd(o, h), B,
                           nb0, nb1, bin_start, cursor, list);
    return hipGetLastError();
}

hipError_t scan_u32(const unsigned int* in, long long n, long long* out, unsigned long long* st, unsigned int* ticket,
                    hipStream_t s)
{
    ProfScope ps("k_scan", s);
    long long ntiles = (n + MC_TILE - 1) / MC_TILE;
    if (ntiles == 0) ntiles = 1;
    hipLaunchKernelGGL(k_scan, dim3((unsigned)ntiles), dim3(256), 0, s, in, n, out, st, ticket, ntiles);
    return hipGetLastError();
}

hipError_t locate(const float* coords, const int32_t* cells, int dim, long long nv, long long nc, GridGeom gg, int B,
                  int nb0, int nb1, const long long* bin_start, const int32_t* list, int32_t* vid, float* w,
                  int32_t* cell, int32_t* unres, unsigned int* n_unres, unsigned int* n_neardeg, hipStream_t s)
{
    ProfScope ps("k_locate", s);
    long long ng = (long long)gg.n0 * gg.n1 * gg.n2;
    if (dim == 2)
        hipLaunchKernelGGL(k_locate<2>, blocks_for(ng), dim3(256), 0, s, coords, cells, nv, nc, gg, B, nb0, nb1,
                           bin_start, list, vid, w, cell, unres, n_unres, n_neardeg);
    else
        hipLaunchKernelGGL(k_locate<3>, blocks_for(ng), dim3(256), 0, s, coords, cells, nv, nc, gg, B, nb0, nb1,
                           bin_start, list, vid, w, cell, unres, n_unres, n_neardeg);
    return hipGetLastError();
}

hipError_t vbins_count(const float* coords, int dim, long long nv, const double* o, const double* h, int VB, int nb0,
                       int nb1, int nb2, unsigned int* cnt, hipStream_t s)
{
    ProfScope ps("k_vbins_count", s);
    if (dim == 2)
        hipLaunchKernelGGL(k_vbins_count<2>, blocks_for(nv), dim3(256), 0, s, coords, nv, mkdd(o, h), VB, nb0, nb1, nb2,
                           cnt);
    else
        hipLaunchKernelGGL(k_vbins_count<3>, blocks_for(nv), dim3(256), 0, s, coords, nv, mkdd(o, h), VB, nb0, nb1, nb2,
                           cnt);
    return hipGetLastError();
}

hipError_t vbins_fill(const float* coords, int dim, long long nv, const double* o, const double* h, int VB, int nb0,
                      int nb1, int nb2, const long long* start, unsigned int* cursor, int32_t* list, hipStream_t s)
{
    ProfScope ps("k_vbins_fill", s);
    if (dim == 2)
        hipLaunchKernelGGL(k_vbins_fill<2>, blocks_for(nv), dim3(256), 0, s, coords, nv, mkdd(o, h), VB, nb0, nb1, nb2,
                           start, cursor, list);
    else
        hipLaunchKernelGGL(k_vbins_fill<3>, blocks_for(nv), dim3(256), 0, s, coords, nv, mkdd(o, h), VB, nb0, nb1, nb2,
                           start, cursor, list);
    return hipGetLastError();
}

hipError_t fill_nearest(const float* coords, int dim, long long nv, GridGeom gg, const double* o, const double* h,
                        int VB, int nb0, int nb1, int nb2, const long long* vstart, const int32_t* vlist,
                        const int32_t* unres, long long n_unres, int32_t* vid, float* w, long long ng, hipStream_t s)
{
    if (n_unres <= 0) return hipSuccess;
    ProfScope ps("k_fill_nearest", s);
    double hmin = h[0], ext = fabs(o[0]) + h[0] * gg.n0;
    for (int d = 1; d < dim; ++d) {
        hmin = h[d] < hmin ? h[d] : hmin;
        double e = fabs(o[d]) + h[d] * (d == 1 ? gg.n1 : gg.n2);
        ext = e > ext ? e : ext;
    }
    const double eps = 1e-5 * ext;
    if (dim == 2)
        hipLaunchKernelGGL(k_fill_nearest<2>, blocks_for(n_unres), dim3(256), 0, s, coords, nv, gg, mkdd(o, h), VB, nb0,
                           nb1, nb2, vstart, vlist, unres, n_unres, vid, w, ng, hmin, eps);
    else
        hipLaunchKernelGGL(k_fill_nearest<3>, blocks_for(n_unres), dim3(256), 0, s, coords, nv, gg, mkdd(o, h), VB, nb0,
                           nb1, nb2, vstart, vlist, unres, n_unres, vid, w, ng, hmin, eps);
    return hipGetLastError();
}

hipError_t fill_midrange(int dim, const int32_t* unres, long long n_unres, int32_t* vid, float* w, long long ng,
                         hipStream_t s)
{
    if (n_unres <= 0) return hipSuccess;
    ProfScope ps("k_fill_midrange", s);
    hipLaunchKernelGGL(k_fill_midrange, blocks_for(n_unres), dim3(256), 0, s, dim, unres, n_unres, vid, w, ng);
    return hipGetLastError();
}

}  // namespace mck
