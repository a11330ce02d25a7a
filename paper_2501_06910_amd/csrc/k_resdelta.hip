// k_resdelta.hip -- residual codes with a 1-D Lorenzo predictor along the
// vertex order on gfx950 (the residuals serialised as a 1-D array and
// compressed predictively, Sec. IV-B):
//   q_i = rint((x_i - g_i) / (2 tau2)), x'_i = (T)(g_i + q_i 2 tau2),
//   code_i = (q_i - q_{i-1}) + R when |x_i - x'_i| <= tau2 and the
//   difference is within R - 1, else 0 with x_i stored raw.
// g is the multilinear back-interpolation (the linear pair) or the value of
// the vertex's nearest node (the paper's pair, closed loop).
// Compression keeps the usual tile layout (vertex tile*1024 + i*256 + t) and
// stages the tile's q in LDS to take the differences; the vertex before a
// tile is back-interpolated once more by the tile's first thread.
// Decompression is a segmented running sum over the codes that restarts at
// every raw value from rint((raw - g) / (2 tau2)):
//   k_resd_tot     per-tile aggregate (restart seen, running value)
//   seg_carry      exclusive segmented scan of the aggregates
//   k_vdecode_delta  back-interpolation, in-tile scan, x'
#include "mc_dev.h"
#include "mc_kernels.h"
#include "mc_seg.h"

// g of N vertices: multilinear back-interpolation (the linear pair) or the
// nearest node's value (the paper's pair, m = node of every vertex).
template <int D, bool NEAR, int N>
__device__ __forceinline__ void g_of(const float* __restrict__ coords, long long nv, const GridGeom& gg,
                                     const float* __restrict__ xh, const int32_t* __restrict__ m,
                                     const long long (&v)[N], const bool (&act)[N], float (&g)[N])
{
    if (NEAR) {
        int32_t j[N];
#pragma unroll
        for (int i = 0; i < N; ++i) j[i] = m[act[i] ? v[i] : 0];
#pragma unroll
        for (int i = 0; i < N; ++i) g[i] = xh[j[i]];
    } else {
        back_interp_n<D, N>(coords, nv, gg, xh, v, act, g);
    }
}

template <typename T, int D, bool NEAR>
__global__ __launch_bounds__(256) void k_residual_delta(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                        const float* __restrict__ xh, const int32_t* __restrict__ m,
                                                        const T* __restrict__ x,
                                                        const DevBound* __restrict__ bnd, uint16_t* __restrict__ codes,
                                                        float* __restrict__ dbg_g, unsigned int* __restrict__ count,
                                                        unsigned int* __restrict__ vsum, unsigned int* __restrict__ err)
{
    __shared__ int s_q[MC_TILE];
    __shared__ int s_qb;
    __shared__ int s_cnt[4];
    const DevBound b = *bnd;
    const long long tile = blockIdx.x;
    long long v[MC_IPT];
    bool act[MC_IPT];
    T xv[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        v[i] = tile * MC_TILE + i * MC_WG + threadIdx.x;
        act[i] = v[i] < nv && b.ok;
        xv[i] = x[act[i] ? v[i] : 0];
    }
    float g[MC_IPT];
    g_of<D, NEAR, MC_IPT>(coords, nv, gg, xh, m, v, act, g);
    int q[MC_IPT];
    bool ok[MC_IPT];
    bool range_bad = false;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        const double s = ((double)xv[i] - (double)g[i]) * b.inv2;
        const bool inr = fabs(s) < 134217728.0;
        q[i] = inr ? (int)rint(s) : 0;
        range_bad |= act[i] && !inr;
        const T xr = (T)((double)g[i] + (double)q[i] * b.step2);
        ok[i] = inr && fabs((double)xv[i] - (double)xr) <= b.tau2;
        s_q[i * MC_WG + threadIdx.x] = q[i];
        if (dbg_g && act[i]) dbg_g[v[i]] = g[i];
    }
    if (threadIdx.x == 0) {                     // q of the vertex before the tile
        int qb = 0;
        if (tile > 0 && b.ok) {
            const long long vb[1] = {tile * MC_TILE - 1};
            const bool ab[1] = {true};
            float gb[1];
            g_of<D, NEAR, 1>(coords, nv, gg, xh, m, vb, ab, gb);
            const double s = ((double)x[vb[0]] - (double)gb[0]) * b.inv2;
            qb = fabs(s) < 134217728.0 ? (int)rint(s) : 0;
        }
        s_qb = qb;
    }
    __syncthreads();
    int nout = 0;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (!act[i]) continue;
        const int e = i * MC_WG + threadIdx.x;
        const int d = q[i] - (e > 0 ? s_q[e - 1] : s_qb);
        const bool c = ok[i] && d >= -(MC_R - 1) && d <= MC_R - 1;
        codes[v[i]] = c ? (uint16_t)(d + MC_R) : (uint16_t)0;
        nout += c ? 0 : 1;
    }
    if (range_bad) atomicOr(err, MC_EBIT_RANGE);
    nout = wave_sum(nout);
    if (lane_id() == 0) s_cnt[threadIdx.x >> 6] = nout;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned c = (unsigned)(s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3]);
        if (c) atomicAdd(&vsum[tile / MC_SC_TILES], c);
        count[tile] = c;
    }
}

__device__ __forceinline__ long long rd_find(const int32_t* __restrict__ oidx, long long n, long long j)
{
    long long lo = 0, hi = n;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if ((long long)oidx[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && (long long)oidx[lo] == j) ? lo : -1;
}

// Raw value and restart q of a code-0 vertex (g computed here: such
// vertices are rare).
template <typename T, int D, bool NEAR>
__device__ __forceinline__ int restart_q(const float* __restrict__ coords, long long nv, const GridGeom& gg,
                                         const float* __restrict__ xh, const int32_t* __restrict__ m,
                                         const int32_t* __restrict__ oidx,
                                         const T* __restrict__ oval, long long nout, long long vtx, double inv2,
                                         const float* g_known, T* raw_out)
{
    const long long k = rd_find(oidx, nout, vtx);
    const T raw = k >= 0 ? oval[k] : (T)0;
    float g;
    if (g_known) {
        g = *g_known;
    } else {
        const long long vb[1] = {vtx};
        const bool ab[1] = {true};
        float gb[1];
        g_of<D, NEAR, 1>(coords, nv, gg, xh, m, vb, ab, gb);
        g = gb[0];
    }
    if (raw_out) *raw_out = raw;
    return (int)rint(((double)raw - (double)g) * inv2);
}

// Segments of the tile in vertex order: element e of the tile is vertex
// tile*1024 + e, owned by thread e % 256 (slot e / 256); thread t folds
// elements 4t..4t+3 from LDS.
template <typename T, int D, bool NEAR>
__global__ __launch_bounds__(256) void k_resd_tot(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                  const float* __restrict__ xh, const int32_t* __restrict__ m,
                                                  const uint16_t* __restrict__ codes,
                                                  const int32_t* __restrict__ oidx, const T* __restrict__ oval,
                                                  const mc_result* __restrict__ res, long long vcap,
                                                  int2* __restrict__ agg)
{
    __shared__ Seg s_seg[MC_TILE];
    __shared__ Seg s_w[4];
    const long long tile = blockIdx.x;
    const double inv2 = 1.0 / (2.0 * res->tau2);
    const long long nout = res->n_vertex_outliers < vcap ? res->n_vertex_outliers : vcap;
    int code[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        const long long vi = tile * MC_TILE + i * MC_WG + threadIdx.x;
        code[i] = vi < nv ? (int)codes[vi] : MC_R;               // past the end: a zero difference
    }
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        const long long vi = tile * MC_TILE + i * MC_WG + threadIdx.x;
        Seg sg{0, code[i] - MC_R};
        if (code[i] == 0)
            sg = Seg{1, restart_q<T, D, NEAR>(coords, nv, gg, xh, m, oidx, oval, nout, vi, inv2, nullptr, nullptr)};
        s_seg[i * MC_WG + threadIdx.x] = sg;
    }
    __syncthreads();
    Seg s{0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) s = seg_op(s, s_seg[4 * threadIdx.x + k]);
    Seg total;
    (void)block_seg_excl<4>(s, Seg{0, 0}, s_w, &total);
    if (threadIdx.x == 0) agg[tile] = make_int2(total.f, total.v);
}

template <typename T, int D, bool NEAR>
__global__ __launch_bounds__(256) void k_vdecode_delta(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                       const float* __restrict__ xh, const int32_t* __restrict__ m,
                                                       const uint16_t* __restrict__ codes,
                                                       const int32_t* __restrict__ oidx, const T* __restrict__ oval,
                                                       const mc_result* __restrict__ res, long long vcap,
                                                       const int* __restrict__ carry, T* __restrict__ xout)
{
    __shared__ Seg s_seg[MC_TILE];
    __shared__ Seg s_w[4];
    const long long tile = blockIdx.x;
    const double step2 = 2.0 * res->tau2, inv2 = 1.0 / (2.0 * res->tau2);
    const long long nout = res->n_vertex_outliers < vcap ? res->n_vertex_outliers : vcap;
    long long v[MC_IPT];
    bool act[MC_IPT];
    int code[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        v[i] = tile * MC_TILE + i * MC_WG + threadIdx.x;
        act[i] = v[i] < nv;
        code[i] = act[i] ? (int)codes[v[i]] : MC_R;
    }
    float g[MC_IPT];
    g_of<D, NEAR, MC_IPT>(coords, nv, gg, xh, m, v, act, g);
    T raw[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        Seg sg{0, code[i] - MC_R};
        raw[i] = (T)0;
        if (code[i] == 0)
            sg = Seg{1, restart_q<T, D, NEAR>(coords, nv, gg, xh, m, oidx, oval, nout, v[i], inv2, &g[i], &raw[i])};
        s_seg[i * MC_WG + threadIdx.x] = sg;
    }
    __syncthreads();
    Seg e4[4];
    Seg s{0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        e4[k] = s_seg[4 * threadIdx.x + k];
        s = seg_op(s, e4[k]);
    }
    Seg total;
    Seg run = block_seg_excl<4>(s, Seg{1, carry[tile]}, s_w, &total);
    __syncthreads();                              // every thread has read its elements
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        run = seg_op(run, e4[k]);
        s_seg[4 * threadIdx.x + k].v = run.v;     // q of the element
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (!act[i]) continue;
        const int qv = s_seg[i * MC_WG + threadIdx.x].v;
        xout[v[i]] = code[i] == 0 ? raw[i] : (T)((double)g[i] + (double)qv * step2);
    }
}

namespace mck {

hipError_t residual_delta(const float* coords, long long nv, GridGeom gg, const float* xh, const int32_t* m,
                          const void* x, int dtype, const DevBound* bnd, uint16_t* codes, float* dbg_g,
                          unsigned* count, unsigned* vsum, unsigned* err, hipStream_t s)
{
    ProfScope ps("k_residual_delta", s);
    const dim3 grid((unsigned)((nv + MC_TILE - 1) / MC_TILE));
#define MC_RD(T, D, NR) hipLaunchKernelGGL((k_residual_delta<T, D, NR>), grid, dim3(256), 0, s, coords, nv, gg, xh, \
                                           m, (const T*)x, bnd, codes, dbg_g, count, vsum, err)
#define MC_RD2(T) do { if (m) MC_RD(T, 3, true); else if (gg.dim == 2) MC_RD(T, 2, false); \
                       else MC_RD(T, 3, false); } while (0)
    if (dtype == MC_F64) MC_RD2(double);
    else MC_RD2(float);
#undef MC_RD2
#undef MC_RD
    return hipGetLastError();
}

hipError_t vertex_decode_delta(const float* coords, long long nv, GridGeom gg, const float* xh, const int32_t* m,
                               const uint16_t* codes,
                               const int32_t* oidx, const void* oval, long long vcap, const mc_result* res,
                               int2* agg, int* carry, void* xout, int dtype, hipStream_t s)
{
    const long long ntiles = (nv + MC_TILE - 1) / MC_TILE;
    const dim3 grid((unsigned)ntiles);
    hipError_t e;
    {
        ProfScope ps("k_resd_tot", s);
#define MC_RT(T, D, NR) hipLaunchKernelGGL((k_resd_tot<T, D, NR>), grid, dim3(256), 0, s, coords, nv, gg, xh, m, codes, \
                                           oidx, (const T*)oval, res, vcap, agg)
#define MC_RT2(T) do { if (m) MC_RT(T, 3, true); else if (gg.dim == 2) MC_RT(T, 2, false); \
                       else MC_RT(T, 3, false); } while (0)
        if (dtype == MC_F64) MC_RT2(double);
        else MC_RT2(float);
#undef MC_RT2
#undef MC_RT
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        ProfScope ps("k_resd_carry", s);
        if ((e = seg_carry(agg, ntiles, carry, s)) != hipSuccess) return e;
    }
    ProfScope ps("k_vdecode_delta", s);
#define MC_VD(T, D, NR) hipLaunchKernelGGL((k_vdecode_delta<T, D, NR>), grid, dim3(256), 0, s, coords, nv, gg, xh, m, \
                                           codes, oidx, (const T*)oval, res, vcap, carry, (T*)xout)
#define MC_VD2(T) do { if (m) MC_VD(T, 3, true); else if (gg.dim == 2) MC_VD(T, 2, false); \
                       else MC_VD(T, 3, false); } while (0)
    if (dtype == MC_F64) MC_VD2(double);
    else MC_VD2(float);
#undef MC_VD2
#undef MC_VD
    return hipGetLastError();
}

}  // namespace mck
