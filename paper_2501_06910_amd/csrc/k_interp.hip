// k_interp.hip -- the multilevel interpolation and the time-axis grid
// predictors on gfx950 (alternative grid compressors C(x1): the SZ family's
// interpolation predictor, Sec. II; Sec. IV-D admits any compressor).  The
// classes, their order and the prediction rules are stated in mc_interp.h.
// The time-axis predictor codes and decodes every node on its own, one pass
// each way.
//
// Encoder: the predictions read the prequantised grid p, which the encoder
// holds whole, so every node is coded independently in one pass (thread per
// node, codes and per-tile outlier counts; the outlier gather of
// k_compress.hip recomputes the errors of the outliers).  Encoder and class
// passes take their 256-node tiles in XCD-contiguous order, so that the rows
// and planes a prediction reads are mostly in the same XCD's L2.
//
// Decoder: classes in order.  The coarse classes (every node whose
// coordinates are all multiples of SC, at most MC_IP_COARSE of them) are
// decoded by one workgroup in LDS: the nodes of that sub-lattice keep the
// class order and the rules (a stride s >= SC becomes s / SC there, and the
// neighbour tests hold on the sub-lattice's extents).  Each finer class is
// one launch, thread per node, neighbours read from p in HBM; every launch
// writes p and x1' = (float)(c + p * 2 tau1) of its own nodes.
#include "mc_dev.h"
#include "mc_interp.h"
#include "mc_kernels.h"

#define MC_IP_COARSE 4096      // nodes decoded in LDS by the coarse workgroup

// Multiples of s in [0, m - 1], and the odd ones among them.
__host__ __device__ __forceinline__ int ip_mult(int m, int s) { return (m - 1) / s + 1; }
__host__ __device__ __forceinline__ int ip_odd(int m, int s) { return ((m - 1) / s + 1) / 2; }

// MC_IP_NPT nodes per thread, 256-node chunks: short-lived waves are
// otherwise dispatch-bound.  Indices past the grid are clamped for the
// loads (every load of the chunk issued together) and masked for the stores.
#define MC_IP_NPT 8
template <bool CUBIC>
__global__ __launch_bounds__(256) void k_ip_codes(const int32_t* __restrict__ p, int n0, int n1, int n2, unsigned ng,
                                                  uint16_t* __restrict__ codes, unsigned int* __restrict__ count,
                                                  unsigned int* __restrict__ gsum)
{
    const unsigned j0 = xcd_tile(blockIdx.x, gridDim.x) * (256u * MC_IP_NPT) + threadIdx.x;
    long long d[MC_IP_NPT];
#pragma unroll
    for (int u = 0; u < MC_IP_NPT; ++u) {
        const unsigned j = min(j0 + 256u * u, ng - 1u);
        const unsigned r = j / (unsigned)n0;
        const int i0 = (int)(j - r * (unsigned)n0), i1 = (int)(r % (unsigned)n1), i2 = (int)(r / (unsigned)n1);
        d[u] = ip_delta<CUBIC>(p, (int)j, i0, i1, i2, n0, n1, n2);
    }
#pragma unroll
    for (int u = 0; u < MC_IP_NPT; ++u) {
        const unsigned j = j0 + 256u * u;
        const bool out = j < ng && !(d[u] >= -(MC_R - 1) && d[u] <= MC_R - 1);
        if (j < ng) codes[j] = out ? (uint16_t)0 : (uint16_t)(d[u] + MC_R);
        // the 64 lanes of a wave lie in one MC_TILE tile (256-aligned chunks)
        const unsigned long long m = __ballot(out);
        if (m != 0ull && lane_id() == 0) {
            const unsigned t = j / MC_TILE;
            atomicAdd(&count[t], (unsigned)__popcll(m));
            atomicAdd(&gsum[t / MC_SC_TILES], (unsigned)__popcll(m));
        }
    }
}

// Coarse classes in LDS: sub-lattice of extents m0 x m1 x m2 (node b at
// grid coordinates b * SC); strides 2^(L-1) / SC .. 1 on it.
template <bool CUBIC>
__global__ __launch_bounds__(1024) void k_ip_coarse(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                    const int32_t* __restrict__ odelta,
                                                    const mc_result* __restrict__ res, long long gcap, int n0, int n1,
                                                    int dim, int top, int SC, int m0, int m1, int m2,
                                                    int32_t* __restrict__ p, float* __restrict__ xh)
{
    __shared__ int32_t q[MC_IP_COARSE];
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const int mm = m0 * m1 * m2;
    const int mdim[3] = {m0, m1, m2};
    auto flat = [&](int b0, int b1, int b2) {
        return (long long)b0 * SC + (long long)n0 * ((long long)b1 * SC + (long long)n1 * ((long long)b2 * SC));
    };
    // every code load in flight before any is used (at most 4 per thread)
    constexpr int PER = MC_IP_COARSE / 1024;
    int cv[PER];
    long long jv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int k = threadIdx.x + 1024 * u;
        const int b0 = k % m0, r = k / m0;
        jv[u] = k < mm ? flat(b0, r % m1, r / m1) : 0;
        cv[u] = k < mm ? (int)codes[jv[u]] : MC_R;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int k = threadIdx.x + 1024 * u;
        if (k >= mm) continue;
        int e = cv[u] - MC_R;
        if (cv[u] == 0) {
            const long long o = find_outlier(oidx, nout, jv[u]);
            e = o >= 0 ? odelta[o] : 0;
        }
        q[k] = e;
    }
    __syncthreads();
    // q holds the errors; each class pass turns its nodes into values (the
    // origin's error is its value)
    for (int s = top; s >= 1; s >>= 1) {
        for (int a = 0; a < dim; ++a) {
            int c[3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                c[d] = d == a ? ip_odd(mdim[d], s) : ip_mult(mdim[d], d < a ? s : 2 * s);
            const int tot = c[0] * c[1] * c[2];
            const int st = a == 0 ? 1 : (a == 1 ? m0 : m0 * m1);
            for (int k = threadIdx.x; k < tot; k += 1024) {
                int b[3];
                b[0] = k % c[0];
                const int r = k / c[0];
                b[1] = r % c[1];
                b[2] = r / c[1];
#pragma unroll
                for (int d = 0; d < 3; ++d) b[d] = d == a ? (2 * b[d] + 1) * s : b[d] * (d < a ? s : 2 * s);
                const int kk = b[0] + m0 * (b[1] + m1 * b[2]);
                q[kk] = (int32_t)(ip_predict<CUBIC>(q, kk, b[a], mdim[a], st * s, s) + q[kk]);
            }
            __syncthreads();
        }
    }
    const double cc = res->c, step1 = 2.0 * res->tau1;
    for (int k = threadIdx.x; k < mm; k += 1024) {
        const int b0 = k % m0, r = k / m0;
        const long long j = flat(b0, r % m1, r / m1);
        p[j] = q[k];
        xh[j] = xhat_of(q[k], cc, step1);
    }
}

// One finer class (s, a): c0 x c1 x c2 nodes, MC_IP_PPT per thread in
// 256-node chunks (loads first, indices past the class clamped).
#define MC_IP_PPT 4
template <bool CUBIC>
__global__ __launch_bounds__(256) void k_ip_pass(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                 const int32_t* __restrict__ odelta, const mc_result* __restrict__ res,
                                                 long long gcap, int n0, int n1, int n2, int s, int a, int c0, int c1,
                                                 unsigned tot, int32_t* __restrict__ p, float* __restrict__ xh)
{
    const unsigned k0 = xcd_tile(blockIdx.x, gridDim.x) * (256u * MC_IP_PPT) + threadIdx.x;
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const double cc = res->c, step1 = 2.0 * res->tau1;
    const int st = a == 0 ? 1 : (a == 1 ? n0 : n0 * n1);
    const int n = a == 0 ? n0 : (a == 1 ? n1 : n2);
    int jv[MC_IP_PPT], cv[MC_IP_PPT];
    long long pred[MC_IP_PPT];
#pragma unroll
    for (int u = 0; u < MC_IP_PPT; ++u) {
        const unsigned k = min(k0 + 256u * u, tot - 1u);
        const unsigned r = k / (unsigned)c0;
        int b[3] = {(int)(k - r * (unsigned)c0), (int)(r % (unsigned)c1), (int)(r / (unsigned)c1)};
#pragma unroll
        for (int d = 0; d < 3; ++d) b[d] = d == a ? (2 * b[d] + 1) * s : b[d] * (d < a ? s : 2 * s);
        jv[u] = b[0] + n0 * (b[1] + n1 * b[2]);
        cv[u] = codes[jv[u]];
        pred[u] = ip_predict<CUBIC>(p, jv[u], b[a], n, st * s, s);
    }
#pragma unroll
    for (int u = 0; u < MC_IP_PPT; ++u) {
        if (k0 + 256u * u >= tot) break;
        int e = cv[u] - MC_R;
        if (cv[u] == 0) {       // an outlier: its error from the list
            const long long o = find_outlier(oidx, nout, jv[u]);
            e = o >= 0 ? odelta[o] : 0;
        }
        const int32_t v = (int32_t)(pred[u] + e);
        p[jv[u]] = v;
        xh[jv[u]] = xhat_of(v, cc, step1);
    }
}

// Time-axis predictor: every node on its own (MC_IP_NPT per thread).
__global__ __launch_bounds__(256) void k_tp_codes(const int32_t* __restrict__ p, const float* __restrict__ ref,
                                                  const DevBound* __restrict__ bnd, unsigned ng,
                                                  uint16_t* __restrict__ codes, unsigned int* __restrict__ count,
                                                  unsigned int* __restrict__ gsum)
{
    const double c = bnd->c, inv1 = bnd->inv1;
    const unsigned j0 = xcd_tile(blockIdx.x, gridDim.x) * (256u * MC_IP_NPT) + threadIdx.x;
    int pv[MC_IP_NPT];
    float rv[MC_IP_NPT];
#pragma unroll
    for (int u = 0; u < MC_IP_NPT; ++u) {
        const unsigned j = min(j0 + 256u * u, ng - 1u);
        pv[u] = p[j];
        rv[u] = ref[j];
    }
#pragma unroll
    for (int u = 0; u < MC_IP_NPT; ++u) {
        const unsigned j = j0 + 256u * u;
        const long long d = (long long)pv[u] - tp_pred(rv[u], c, inv1);
        const bool out = j < ng && !(d >= -(MC_R - 1) && d <= MC_R - 1);
        if (j < ng) codes[j] = out ? (uint16_t)0 : (uint16_t)(d + MC_R);
        const unsigned long long m = __ballot(out);
        if (m != 0ull && lane_id() == 0) {
            const unsigned t = j / MC_TILE;
            atomicAdd(&count[t], (unsigned)__popcll(m));
            atomicAdd(&gsum[t / MC_SC_TILES], (unsigned)__popcll(m));
        }
    }
}

__global__ __launch_bounds__(256) void k_tp_decode(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                   const int32_t* __restrict__ odelta,
                                                   const mc_result* __restrict__ res, long long gcap,
                                                   const float* __restrict__ ref, unsigned ng, int32_t* __restrict__ p,
                                                   float* __restrict__ xh)
{
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const double c = res->c, step1 = 2.0 * res->tau1, inv1 = 1.0 / (2.0 * res->tau1);
    const unsigned j0 = xcd_tile(blockIdx.x, gridDim.x) * (256u * MC_IP_NPT) + threadIdx.x;
    int cv[MC_IP_NPT];
    float rv[MC_IP_NPT];
#pragma unroll
    for (int u = 0; u < MC_IP_NPT; ++u) {
        const unsigned j = min(j0 + 256u * u, ng - 1u);
        cv[u] = codes[j];
        rv[u] = ref[j];
    }
#pragma unroll
    for (int u = 0; u < MC_IP_NPT; ++u) {
        const unsigned j = j0 + 256u * u;
        if (j >= ng) break;
        int e = cv[u] - MC_R;
        if (cv[u] == 0) {
            const long long o = find_outlier(oidx, nout, j);
            e = o >= 0 ? odelta[o] : 0;
        }
        const int32_t v = (int32_t)(tp_pred(rv[u], c, inv1) + e);
        p[j] = v;
        xh[j] = xhat_of(v, c, step1);
    }
}

namespace mck {

hipError_t temporal_codes(const int32_t* p, const float* ref, const DevBound* bnd, long long ng, uint16_t* codes,
                          unsigned int* count, unsigned int* gsum, hipStream_t s)
{
    ProfScope ps("k_tp_codes", s);
    const dim3 grid((unsigned)((ng + 256 * MC_IP_NPT - 1) / (256 * MC_IP_NPT)));
    hipLaunchKernelGGL(k_tp_codes, grid, dim3(256), 0, s, p, ref, bnd, (unsigned)ng, codes, count, gsum);
    return hipGetLastError();
}

hipError_t temporal_decode(const uint16_t* codes, const int32_t* oidx, const int32_t* odelta, long long gcap,
                           const mc_result* res, const float* ref, long long ng, int32_t* p, float* xh, hipStream_t s)
{
    ProfScope ps("k_tp_decode", s);
    const dim3 grid((unsigned)((ng + 256 * MC_IP_NPT - 1) / (256 * MC_IP_NPT)));
    hipLaunchKernelGGL(k_tp_decode, grid, dim3(256), 0, s, codes, oidx, odelta, res, gcap, ref, (unsigned)ng, p, xh);
    return hipGetLastError();
}

hipError_t interp_codes(const int32_t* p, int n0, int n1, int n2, long long ng, bool cubic, uint16_t* codes,
                        unsigned int* count, unsigned int* gsum, hipStream_t s)
{
    ProfScope ps("k_ip_codes", s);
    const dim3 grid((unsigned)((ng + 256 * MC_IP_NPT - 1) / (256 * MC_IP_NPT)));
    if (cubic) hipLaunchKernelGGL(k_ip_codes<true>, grid, dim3(256), 0, s, p, n0, n1, n2, (unsigned)ng, codes, count, gsum);
    else hipLaunchKernelGGL(k_ip_codes<false>, grid, dim3(256), 0, s, p, n0, n1, n2, (unsigned)ng, codes, count, gsum);
    return hipGetLastError();
}

hipError_t interp_decode(const uint16_t* codes, const int32_t* oidx, const int32_t* odelta, long long gcap,
                         const mc_result* res, int dim, int n0, int n1, int n2, bool cubic, int32_t* p, float* xh,
                         hipStream_t s)
{
    const int n[3] = {n0, n1, n2};
    int L = 0;
    for (int d = 0; d < dim; ++d)
        while ((1 << L) < n[d]) ++L;
    // coarsest sub-lattice spacing SC whose nodes fit in LDS
    int SC = 1;
    for (;;) {
        long long mm = 1;
        for (int d = 0; d < 3; ++d) mm *= ip_mult(n[d], SC);
        if (mm <= MC_IP_COARSE) break;
        SC *= 2;
    }
    const int m0 = ip_mult(n0, SC), m1 = ip_mult(n1, SC), m2 = ip_mult(n2, SC);
    const int top = (1 << (L - 1)) >= SC ? (1 << (L - 1)) / SC : 0;
    {
        ProfScope ps("k_ip_coarse", s);
        if (cubic)
            hipLaunchKernelGGL(k_ip_coarse<true>, dim3(1), dim3(1024), 0, s, codes, oidx, odelta, res, gcap, n0, n1,
                               dim, top, SC, m0, m1, m2, p, xh);
        else
            hipLaunchKernelGGL(k_ip_coarse<false>, dim3(1), dim3(1024), 0, s, codes, oidx, odelta, res, gcap, n0, n1,
                               dim, top, SC, m0, m1, m2, p, xh);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ProfScope ps("k_ip_pass", s);
    for (int st = SC / 2; st >= 1; st >>= 1)
        for (int a = 0; a < dim; ++a) {
            int c[3];
            for (int d = 0; d < 3; ++d) c[d] = d == a ? ip_odd(n[d], st) : ip_mult(n[d], d < a ? st : 2 * st);
            const unsigned tot = (unsigned)((long long)c[0] * c[1] * c[2]);
            if (tot == 0) continue;
            const dim3 grid((tot + 256 * MC_IP_PPT - 1) / (256 * MC_IP_PPT));
            if (cubic)
                hipLaunchKernelGGL(k_ip_pass<true>, grid, dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, n1, n2,
                                   st, a, c[0], c[1], tot, p, xh);
            else
                hipLaunchKernelGGL(k_ip_pass<false>, grid, dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, n1, n2,
                                   st, a, c[0], c[1], tot, p, xh);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace mck
