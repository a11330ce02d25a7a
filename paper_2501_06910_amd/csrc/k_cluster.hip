// k_cluster.hip -- the paper's own operator pair on gfx950: the nearest
// grid node as back-interpolation g (Sec. IV-C) and the mean of the
// vertices assigned to a node as resampling f (Sec. IV-D), with the
// residual of Alg. 3 taken against the uncompressed grid (open loop) or the
// reconstructed one (closed loop).
//   plan:        k_nearest_node (node of every vertex, counts per node)
//                -> scan of the counts -> stable LSD radix sort of (node,
//                vertex) pairs (k_rs_*): each node's vertices in ascending
//                id order
//   compress:    k_cluster_mean (one thread per node sums its vertices in
//                FP64 in ascending id order, prequantises) -> Lorenzo ->
//                k_residual_nearest -> scatter
//   decompress:  grid decode -> k_vdecode_nearest
#include <cstring>

#include "mc_dev.h"
#include "mc_kernels.h"

// m_k = per axis rint((p_d - o_d) / h_d) clamped to [0, n_d - 1] (FP64, IEEE
// division, as the definition reads).
__global__ __launch_bounds__(256) void k_nearest_node(const float* __restrict__ coords, int dim, long long nv,
                                                      mck::NodeGeom ng_, int32_t* __restrict__ m,
                                                      unsigned int* __restrict__ count)
{
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= nv) return;
    long long idx[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        double t = rint(((double)coords[d * nv + k] - ng_.o[d]) / ng_.h[d]);
        if (!(t >= 0.0)) t = 0.0;
        if (t > (double)(ng_.n[d] - 1)) t = (double)(ng_.n[d] - 1);
        idx[d] = (long long)t;
    }
    const long long j = idx[0] + ng_.n[0] * (idx[1] + ng_.n[1] * idx[2]);
    m[k] = (int32_t)j;
    atomicAdd(&count[j], 1u);
}

// Nodes no vertex maps to.
// Grid_Coarsen (Alg. 2): every plane holding a vertex's node is marked
// (flags: axis 0, then 1, then 2; each mark writes the same 1).
__global__ __launch_bounds__(256) void k_mark_planes(const int32_t* __restrict__ m, long long nv, int n0, int n1, int n2,
                                                     int* __restrict__ flags)
{
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= nv) return;
    const unsigned j = (unsigned)m[k], r = j / (unsigned)n0;
    flags[j - r * (unsigned)n0] = 1;
    flags[n0 + (int)(r % (unsigned)n1)] = 1;
    flags[n0 + n1 + (int)(r / (unsigned)n1)] = 1;
    (void)n2;
}

// Every vertex's node on the coarsened grid (c0 x c1 x ...) from the kept
// planes' new indices, and the vertex count per coarsened node.
__global__ __launch_bounds__(256) void k_remap_nodes(int32_t* __restrict__ m, long long nv, int n0, int n1,
                                                     const int* __restrict__ keep, int c0, int c1,
                                                     unsigned int* __restrict__ count)
{
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= nv) return;
    const unsigned j = (unsigned)m[k], r = j / (unsigned)n0;
    const int a = keep[j - r * (unsigned)n0], b = keep[n0 + (int)(r % (unsigned)n1)],
              c = keep[n0 + n1 + (int)(r / (unsigned)n1)];
    const int jn = a + c0 * (b + c1 * c);
    m[k] = jn;
    atomicAdd(&count[jn], 1u);
}

__global__ __launch_bounds__(256) void k_count_empty(const unsigned int* __restrict__ count, long long ng,
                                                     unsigned int* __restrict__ out)
{
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    int e = j < ng && count[j] == 0 ? 1 : 0;
    e = wave_sum(e);
    if (lane_id() == 0 && e) atomicAdd(out, (unsigned)e);
}

// One thread per node: x1 = FP64 sum of its vertices' values in ascending
// vertex order / count (c for a node without vertices), prequantised with
// tau1; x1' = (float)(c + p 2 tau1).  Also clears the grid tile counts and
// writes the result header.
template <typename T>
__global__ __launch_bounds__(256) void k_cluster_mean(const long long* __restrict__ noff,
                                                      const int32_t* __restrict__ vlist, long long ng,
                                                      const T* __restrict__ x, const DevBound* __restrict__ bnd,
                                                      int32_t* __restrict__ p, float* __restrict__ xh,
                                                      double* __restrict__ x1,
                                                      float* __restrict__ dbg_v, unsigned int* __restrict__ err,
                                                      mc_result* __restrict__ res, int dtype,
                                                      unsigned int* __restrict__ gcount, long long ntg)
{
    const DevBound b = *bnd;
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (j < ntg) gcount[j] = 0u;
    if (j == 0) {
        res->status = b.ok ? 0 : 1;
        res->dtype = dtype;
        res->tau = b.tau;
        res->tau1 = b.tau1;
        res->tau2 = b.tau2;
        res->c = b.c;
        res->xmin = b.xmin;
        res->xmax = b.xmax;
        if (!b.ok) atomicOr(err, (b.flags & MC_EBIT_NONFINITE) ? MC_EBIT_NONFINITE : MC_EBIT_TAU);
    }
    if (!b.ok || j >= ng) return;
    const long long a = noff[j], e = noff[j + 1];
    double sum = 0.0;
    long long k = a;
    for (; k + 4 <= e; k += 4) {               // four gathers in flight, added in order
        const int32_t v0 = vlist[k], v1 = vlist[k + 1], v2 = vlist[k + 2], v3 = vlist[k + 3];
        const double x0 = (double)x[v0], xa = (double)x[v1], xb = (double)x[v2], xc = (double)x[v3];
        sum = sum + x0;
        sum = sum + xa;
        sum = sum + xb;
        sum = sum + xc;
    }
    for (; k < e; ++k) sum = sum + (double)x[vlist[k]];
    const double mean = e > a ? sum / (double)(e - a) : b.c;
    const double s = (mean - b.c) * b.inv1;
    int32_t q = 0;
    if (!(fabs(s) < 134217728.0)) atomicOr(err, MC_EBIT_RANGE);
    else q = (int32_t)rint(s);
    p[j] = q;
    xh[j] = xhat_of(q, b.c, b.step1);      // the grid decoder's FP32 output
    if (x1) x1[j] = mean;
    if (dbg_v) dbg_v[j] = (float)mean;
}

// Residual codes against the nearest node: ref = x1[m] (open loop, bound
// tau) or x1'[m] (closed loop, bound tau2); x' = (T)(x1'[m] + q 2 tau2).
template <typename T>
__global__ __launch_bounds__(256) void k_residual_nearest(const int32_t* __restrict__ m, long long nv,
                                                          const T* __restrict__ x, const double* __restrict__ x1,
                                                          const float* __restrict__ xhat,
                                                          const DevBound* __restrict__ bnd,
                                                          uint16_t* __restrict__ codes, float* __restrict__ dbg_g,
                                                          unsigned int* __restrict__ count,
                                                          unsigned int* __restrict__ vsum)
{
    __shared__ int s_cnt[4];
    const DevBound b = *bnd;
    const long long tile = blockIdx.x;
    const bool open = x1 != nullptr;
    const double bound = open ? b.tau : b.tau2;
    long long v[MC_IPT];
    bool act[MC_IPT];
    T xv[MC_IPT];
    int32_t mi[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        v[i] = tile * MC_TILE + i * MC_WG + threadIdx.x;
        act[i] = v[i] < nv && b.ok;
        const long long vc = act[i] ? v[i] : 0;
        xv[i] = x[vc];
        mi[i] = m[vc];
    }
    float xq[MC_IPT];
    double ref[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        xq[i] = xhat[mi[i]];
        ref[i] = open ? x1[mi[i]] : 0.0;
    }
    int nout = 0;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (!act[i]) continue;
        const double xi = (double)xv[i];
        const double xh = (double)xq[i];
        const double r = open ? ref[i] : xh;
        const double q = rint((xi - r) * b.inv2);
        const T xr = (T)(xh + q * b.step2);
        const bool ok = fabs(q) <= (double)(MC_R - 1) && fabs(xi - (double)xr) <= bound;
        if (dbg_g) dbg_g[v[i]] = (float)r;
        codes[v[i]] = ok ? (uint16_t)((int)q + MC_R) : (uint16_t)0;
        nout += ok ? 0 : 1;
    }
    nout = wave_sum(nout);
    if (lane_id() == 0) s_cnt[threadIdx.x >> 6] = nout;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned c = (unsigned)(s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3]);
        if (c) atomicAdd(&vsum[tile / MC_SC_TILES], c);
        count[tile] = c;
    }
}

__device__ __forceinline__ long long cl_find(const int32_t* __restrict__ oidx, long long n, long long j)
{
    long long lo = 0, hi = n;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if ((long long)oidx[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && (long long)oidx[lo] == j) ? lo : -1;
}

template <typename T>
__global__ __launch_bounds__(256) void k_vdecode_nearest(const int32_t* __restrict__ m, long long nv,
                                                         const float* __restrict__ xhat,
                                                         const uint16_t* __restrict__ codes,
                                                         const int32_t* __restrict__ oidx, const T* __restrict__ oval,
                                                         const mc_result* __restrict__ res, long long vcap,
                                                         T* __restrict__ xout)
{
    const long long tile = blockIdx.x;
    const double step2 = 2.0 * res->tau2;
    long long v[MC_IPT];
    bool act[MC_IPT];
    int code[MC_IPT];
    int32_t mi[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        v[i] = tile * MC_TILE + i * MC_WG + threadIdx.x;
        act[i] = v[i] < nv;
        const long long vc = act[i] ? v[i] : 0;
        code[i] = codes[vc];
        mi[i] = m[vc];
    }
    float xq[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) xq[i] = xhat[mi[i]];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (!act[i]) continue;
        if (code[i] == 0) {
            const long long n = res->n_vertex_outliers < vcap ? res->n_vertex_outliers : vcap;
            const long long k = cl_find(oidx, n, v[i]);
            xout[v[i]] = k >= 0 ? oval[k] : (T)0;
        } else {
            xout[v[i]] = (T)((double)xq[i] + (double)(code[i] - MC_R) * step2);
        }
    }
}

namespace mck {

hipError_t nearest_nodes(const float* coords, int dim, long long nv, NodeGeom g, int32_t* m, unsigned* count,
                         hipStream_t s)
{
    ProfScope ps("k_nearest_node", s);
    hipLaunchKernelGGL(k_nearest_node, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, coords, dim, nv, g, m,
                       count);
    return hipGetLastError();
}

hipError_t mark_planes(const int32_t* m, long long nv, int n0, int n1, int n2, int* flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_mark_planes, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, m, nv, n0, n1, n2, flags);
    return hipGetLastError();
}

hipError_t remap_nodes(int32_t* m, long long nv, int n0, int n1, const int* keep, int c0, int c1, unsigned* count,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_remap_nodes, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, m, nv, n0, n1, keep, c0, c1,
                       count);
    return hipGetLastError();
}

hipError_t count_empty(const unsigned* count, long long ng, unsigned* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_empty, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, count, ng, out);
    return hipGetLastError();
}

// Stable LSD radix sort of (key, index) pairs, 8-bit digits, tiles of
// RS_TILE keys per workgroup (4 waves x 1024 consecutive keys):
//   k_rs_count    digit histogram of every tile, stored digit-major, so the
//                 exclusive scan of the array gives each (digit, tile) its
//                 first output position
//   k_rs_scatter  per wave, its digit counts offset by the earlier waves'
//                 of the tile; then 64 keys at a time in order, each key's
//                 rank among the lanes with the same digit from eight
//                 ballots, and a running per-digit position in LDS
#define RS_TILE 4096

__global__ __launch_bounds__(256) void k_rs_count(const uint32_t* __restrict__ keys, long long n, int shift,
                                                  unsigned* __restrict__ hist, unsigned nblk)
{
    __shared__ unsigned s_h[256];
    s_h[threadIdx.x] = 0u;
    __syncthreads();
    const long long base = (long long)blockIdx.x * RS_TILE;
    for (int i = threadIdx.x; i < RS_TILE; i += 256) {
        const long long k = base + i;
        if (k < n) atomicAdd(&s_h[(keys[k] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblk + blockIdx.x] = s_h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_rs_scatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                    long long n, int shift, const long long* __restrict__ off,
                                                    unsigned nblk, uint32_t* __restrict__ kout,
                                                    int32_t* __restrict__ vout)
{
    __shared__ unsigned s_cnt[4][256];
    __shared__ long long s_base[256];
    const int w = threadIdx.x >> 6, l = lane_id();
    for (int i = threadIdx.x; i < 4 * 256; i += 256) (&s_cnt[0][0])[i] = 0u;
    __syncthreads();
    const long long wb = (long long)blockIdx.x * RS_TILE + (long long)w * (RS_TILE / 4);
    for (int r = 0; r < RS_TILE / 4 / 64; ++r) {
        const long long k = wb + r * 64 + l;
        if (k < n) atomicAdd(&s_cnt[w][(kin[k] >> shift) & 255u], 1u);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        unsigned run = 0u;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const unsigned c = s_cnt[v][d];
            s_cnt[v][d] = run;
            run += c;
        }
        s_base[d] = off[(size_t)d * nblk + blockIdx.x];
    }
    __syncthreads();
    const unsigned long long lt = (1ull << l) - 1ull;
    for (int r = 0; r < RS_TILE / 4 / 64; ++r) {
        const long long k = wb + r * 64 + l;
        const bool valid = k < n;
        const uint32_t key = valid ? kin[k] : 0u;
        const int32_t val = valid ? (vin ? vin[k] : (int32_t)k) : 0;
        const unsigned d = (key >> shift) & 255u;
        unsigned long long eq = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            eq &= bit ? bb : ~bb;
        }
        const unsigned rank = (unsigned)__popcll(eq & lt);
        const unsigned run = s_cnt[w][d];      // read by every lane before the group's update below
        if (valid) {
            const long long pos = s_base[d] + run + rank;
            kout[pos] = key;
            vout[pos] = val;
            if (rank == 0u) s_cnt[w][d] = run + (unsigned)__popcll(eq);
        }
    }
}

static size_t rs_align(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace: temp_bytes is set when temp is NULL.  keys_out[i] and vlist[i]
// get the i-th (key, index) pair in key order, equal keys by index.
hipError_t sort_by_node(const int32_t* m, long long nv, long long ng, uint32_t* keys_out, int32_t* vlist,
                        void* temp, size_t* temp_bytes, hipStream_t s)
{
    const unsigned nblk = (unsigned)((nv + RS_TILE - 1) / RS_TILE > 0 ? (nv + RS_TILE - 1) / RS_TILE : 1);
    const long long nh = 256ll * nblk;
    const long long nst = (nh + MC_TILE - 1) / MC_TILE;
    const size_t b_kt = rs_align((size_t)nv * 4), b_vt = b_kt, b_h = rs_align((size_t)nh * 4),
                 b_off = rs_align((size_t)(nh + 1) * 8), b_st = rs_align((size_t)nst * 8), b_tk = 256;
    const size_t need = b_kt + b_vt + b_h + b_off + b_st + b_tk;
    if (!temp) {
        *temp_bytes = need;
        return hipSuccess;
    }
    if (*temp_bytes < need) return hipErrorInvalidValue;
    if (nv <= 0) return hipSuccess;
    char* q = (char*)temp;
    uint32_t* kt = (uint32_t*)q;
    int32_t* vt = (int32_t*)(q + b_kt);
    unsigned* hist = (unsigned*)(q + b_kt + b_vt);
    long long* off = (long long*)(q + b_kt + b_vt + b_h);
    unsigned long long* st = (unsigned long long*)(q + b_kt + b_vt + b_h + b_off);
    unsigned* ticket = (unsigned*)(q + b_kt + b_vt + b_h + b_off + b_st);
    int bits = 1;
    while (bits < 32 && (1ll << bits) < ng) ++bits;
    const int passes = (bits + 7) / 8;
    const uint32_t* kin = (const uint32_t*)m;
    const int32_t* vin = nullptr;                   // pass 0: the indices themselves
    for (int p = 0; p < passes; ++p) {
        // the last pass writes the caller's arrays
        const bool to_out = ((passes - 1 - p) & 1) == 0;
        uint32_t* ko = to_out ? keys_out : kt;
        int32_t* vo = to_out ? vlist : vt;
        hipError_t e = hipMemsetAsync(st, 0, b_st + b_tk, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_count, dim3(nblk), dim3(256), 0, s, kin, nv, 8 * p, hist, nblk);
        e = scan_u32(hist, nh, off, st, ticket, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(256), 0, s, kin, vin, nv, 8 * p, off, nblk, ko, vo);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        kin = ko;
        vin = vo;
    }
    return hipSuccess;
}

hipError_t cluster_mean(const long long* noff, const int32_t* vlist, long long ng, const void* x, int dtype,
                        const DevBound* bnd, int32_t* p, float* xh, double* x1, float* dbg_v, unsigned* err,
                        mc_result* res, unsigned* gcount, long long ntg, hipStream_t s)
{
    ProfScope ps("k_cluster_mean", s);
    const long long need = ng > ntg ? ng : ntg;
    dim3 grid((unsigned)((need + 255) / 256));
    if (dtype == MC_F64)
        hipLaunchKernelGGL(k_cluster_mean<double>, grid, dim3(256), 0, s, noff, vlist, ng, (const double*)x, bnd, p, xh,
                           x1, dbg_v, err, res, dtype, gcount, ntg);
    else
        hipLaunchKernelGGL(k_cluster_mean<float>, grid, dim3(256), 0, s, noff, vlist, ng, (const float*)x, bnd, p, xh,
                           x1, dbg_v, err, res, dtype, gcount, ntg);
    return hipGetLastError();
}

hipError_t residual_nearest(const int32_t* m, long long nv, const void* x, int dtype, const double* x1,
                            const float* xhat, const DevBound* bnd, uint16_t* codes, float* dbg_g, unsigned* count,
                            unsigned* vsum, hipStream_t s)
{
    ProfScope ps("k_residual_nearest", s);
    dim3 grid((unsigned)((nv + MC_TILE - 1) / MC_TILE));
    if (dtype == MC_F64)
        hipLaunchKernelGGL(k_residual_nearest<double>, grid, dim3(256), 0, s, m, nv, (const double*)x, x1, xhat, bnd,
                           codes, dbg_g, count, vsum);
    else
        hipLaunchKernelGGL(k_residual_nearest<float>, grid, dim3(256), 0, s, m, nv, (const float*)x, x1, xhat, bnd,
                           codes, dbg_g, count, vsum);
    return hipGetLastError();
}

hipError_t vertex_decode_nearest(const int32_t* m, long long nv, const float* xhat, const uint16_t* codes,
                                 const int32_t* oidx, const void* oval, long long vcap, const mc_result* res,
                                 void* xout, int dtype, hipStream_t s)
{
    ProfScope ps("k_vdecode_nearest", s);
    dim3 grid((unsigned)((nv + MC_TILE - 1) / MC_TILE));
    if (dtype == MC_F64)
        hipLaunchKernelGGL(k_vdecode_nearest<double>, grid, dim3(256), 0, s, m, nv, xhat, codes, oidx,
                           (const double*)oval, res, vcap, (double*)xout);
    else
        hipLaunchKernelGGL(k_vdecode_nearest<float>, grid, dim3(256), 0, s, m, nv, xhat, codes, oidx,
                           (const float*)oval, res, vcap, (float*)xout);
    return hipGetLastError();
}

}  // namespace mck
