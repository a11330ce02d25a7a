// k_decode.hip -- decompression on gfx950 (paper Alg. 4).
//   k_dec_xy   Lorenzo inverse within each z-plane: d = code - R (outliers
//              by binary search in the ascending outlier list), running
//              column sums over a chunk of rows plus a workgroup scan along
//              x per row; chunks of one plane chain their column totals
//              through a decoupled look-back (vector payload per chunk)
//   k_dec_z    (3-D) inclusive prefix along z, chunks of planes chained by
//              the same look-back; in place
//   k_vdecode  g(x1') at each vertex from the decoded grid, dequantisation
//              x' = (T)(g + q * 2 tau2), learned shift in learned blocks,
//              raw values for outliers
#include "mc_dev.h"
#include "mc_kernels.h"

__device__ __forceinline__ long long find_outlier(const int32_t* __restrict__ oidx, long long n, long long j)
{
    long long lo = 0, hi = n;           // first index with oidx >= j
    while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        if ((long long)oidx[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && (long long)oidx[lo] == j) ? lo : -1;
}

__device__ __forceinline__ int delta_at(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                        const int32_t* __restrict__ odelta, long long nout, long long j)
{
    const int c = codes[j];
    if (c != 0) return c - MC_R;
    const long long k = find_outlier(oidx, nout, j);
    return k >= 0 ? odelta[k] : 0;
}

__device__ __forceinline__ int ld_coherent(const int* a)
{
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits for a chunk's flag and returns it (thread 0 only).
__device__ __forceinline__ unsigned wait_flag(unsigned int* f)
{
    unsigned v;
    while ((v = __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) == 0u)
        __builtin_amdgcn_s_sleep(1);
    return v;
}

__device__ __forceinline__ void set_flag(unsigned int* f, unsigned v)
{
    __hip_atomic_store(f, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive scan of a workgroup's per-thread totals (256 threads); s needs 5.
__device__ __forceinline__ int block_excl_scan(int v, int* s, int& total)
{
    const int inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) s[w] = inc;
    __syncthreads();
    int off = 0;
    for (int k = 0; k < w; ++k) off += s[k];
    total = s[0] + s[1] + s[2] + s[3];
    __syncthreads();
    return off + inc - v;
}

template <int CPT>
__global__ __launch_bounds__(256) void k_dec_xy(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                const int32_t* __restrict__ odelta, const mc_result* __restrict__ res,
                                                long long gcap, int n0, int n1, int n2, int rows, int nyc,
                                                int32_t* __restrict__ out,
                                                int* __restrict__ agg, int* __restrict__ incl,
                                                unsigned int* __restrict__ flags, unsigned int* __restrict__ ticket)
{
    __shared__ long long s_slot;
    __shared__ int s_sc[5];
    __shared__ unsigned s_f;
    const long long tile = take_ticket(ticket, &s_slot);
    const int z = (int)(tile / nyc), yc = (int)(tile % nyc);
    const int y0 = yc * rows, y1 = min(n1, y0 + rows);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const int c0 = threadIdx.x * CPT;
    const long long plane = (long long)z * n1 * n0;
    int tot[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) tot[k] = 0;
    for (int y = y0; y < y1; ++y) {
        const long long base = plane + (long long)y * n0;
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (c0 + k < n0) tot[k] += delta_at(codes, oidx, odelta, nout, base + c0 + k);
    }
    const long long slot = tile;           // == z * nyc + yc
    int carry[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) carry[k] = 0;
    if (yc == 0) {
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (c0 + k < n0) incl[slot * n0 + c0 + k] = tot[k];
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) set_flag(&flags[slot], 2u);
    } else {
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (c0 + k < n0) agg[slot * n0 + c0 + k] = tot[k];
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) set_flag(&flags[slot], 1u);
        long long kk = slot - 1;
        for (;;) {
            if (threadIdx.x == 0) s_f = wait_flag(&flags[kk]);
            __syncthreads();
            const unsigned f = s_f;
            const int* src = (f == 2u ? incl : agg) + kk * n0;
#pragma unroll
            for (int k = 0; k < CPT; ++k)
                if (c0 + k < n0) carry[k] += ld_coherent(src + c0 + k);
            __syncthreads();
            if (f == 2u) break;
            --kk;
        }
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (c0 + k < n0) incl[slot * n0 + c0 + k] = carry[k] + tot[k];
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) set_flag(&flags[slot], 2u);
    }
    // second pass: column sums from the carry, one x-scan per row
    int col[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) col[k] = carry[k];
    for (int y = y0; y < y1; ++y) {
        const long long base = plane + (long long)y * n0;
        int s[CPT];
        int run = 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            if (c0 + k < n0) col[k] += delta_at(codes, oidx, odelta, nout, base + c0 + k);
            run += (c0 + k < n0) ? col[k] : 0;
            s[k] = run;
        }
        int total;
        const int off = block_excl_scan(run, s_sc, total);
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (c0 + k < n0) out[base + c0 + k] = off + s[k];
    }
}

#define ZPT 4
__global__ __launch_bounds__(256) void k_dec_z(int32_t* __restrict__ s, long long nxy, int n2, int zplanes, int nxyb,
                                               int* __restrict__ agg, int* __restrict__ incl,
                                               unsigned int* __restrict__ flags, unsigned int* __restrict__ ticket)
{
    __shared__ long long s_slot;
    __shared__ unsigned s_f;
    const long long tile = take_ticket(ticket, &s_slot);
    const int zc = (int)(tile / nxyb), xb = (int)(tile % nxyb);
    const int z0 = zc * zplanes, z1 = min(n2, z0 + zplanes);
    const int W = 256 * ZPT;
    long long pos[ZPT];
    int tot[ZPT], carry[ZPT];
#pragma unroll
    for (int k = 0; k < ZPT; ++k) {
        pos[k] = (long long)xb * W + k * 256 + threadIdx.x;
        tot[k] = 0;
        carry[k] = 0;
    }
    for (int z = z0; z < z1; ++z)
#pragma unroll
        for (int k = 0; k < ZPT; ++k)
            if (pos[k] < nxy) tot[k] += s[(long long)z * nxy + pos[k]];
    const long long slot = tile;
    if (zc == 0) {
#pragma unroll
        for (int k = 0; k < ZPT; ++k) incl[slot * W + k * 256 + threadIdx.x] = tot[k];
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) set_flag(&flags[slot], 2u);
    } else {
#pragma unroll
        for (int k = 0; k < ZPT; ++k) agg[slot * W + k * 256 + threadIdx.x] = tot[k];
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) set_flag(&flags[slot], 1u);
        long long kk = slot - nxyb;
        for (;;) {
            if (threadIdx.x == 0) s_f = wait_flag(&flags[kk]);
            __syncthreads();
            const unsigned f = s_f;
            const int* src = (f == 2u ? incl : agg) + kk * W;
#pragma unroll
            for (int k = 0; k < ZPT; ++k) carry[k] += ld_coherent(src + k * 256 + threadIdx.x);
            __syncthreads();
            if (f == 2u) break;
            kk -= nxyb;
        }
#pragma unroll
        for (int k = 0; k < ZPT; ++k) incl[slot * W + k * 256 + threadIdx.x] = carry[k] + tot[k];
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) set_flag(&flags[slot], 2u);
    }
    int run[ZPT];
#pragma unroll
    for (int k = 0; k < ZPT; ++k) run[k] = carry[k];
    for (int z = z0; z < z1; ++z)
#pragma unroll
        for (int k = 0; k < ZPT; ++k)
            if (pos[k] < nxy) {
                const long long j = (long long)z * nxy + pos[k];
                run[k] += s[j];
                s[j] = run[k];
            }
}

template <typename T, int D, bool LEARNED>
__global__ __launch_bounds__(256) void k_vdecode(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                 const int32_t* __restrict__ p, const uint16_t* __restrict__ codes,
                                                 const int32_t* __restrict__ oidx, const T* __restrict__ oval,
                                                 const mc_result* __restrict__ res, long long vcap,
                                                 const int32_t* __restrict__ rho_q,
                                                 const uint32_t* __restrict__ bflags, T* __restrict__ xout)
{
    const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    const double c = res->c, step1 = 2.0 * res->tau1, step2 = 2.0 * res->tau2;
    const int code = codes[v];
    if (code == 0) {
        const long long n = res->n_vertex_outliers < vcap ? res->n_vertex_outliers : vcap;
        const long long k = find_outlier(oidx, n, v);
        xout[v] = k >= 0 ? oval[k] : (T)0;
        return;
    }
    int i0, i1, i2 = 0;
    float t0, t1, t2 = 0.0f;
    axis_cell(coords[v], gg.of[0], gg.ihf[0], gg.n0, i0, t0);
    axis_cell(coords[nv + v], gg.of[1], gg.ihf[1], gg.n1, i1, t1);
    if (D == 3) axis_cell(coords[2 * nv + v], gg.of[2], gg.ihf[2], gg.n2, i2, t2);
    const long long n0 = gg.n0, n01 = (long long)gg.n0 * gg.n1;
    const long long j = i0 + n0 * i1 + n01 * i2;
    const float c00 = lerpf_(xhat_of(p[j], c, step1), xhat_of(p[j + 1], c, step1), t0);
    const float c10 = lerpf_(xhat_of(p[j + n0], c, step1), xhat_of(p[j + n0 + 1], c, step1), t0);
    float g = lerpf_(c00, c10, t1);
    if (D == 3) {
        const float c01 = lerpf_(xhat_of(p[j + n01], c, step1), xhat_of(p[j + n01 + 1], c, step1), t0);
        const float c11 = lerpf_(xhat_of(p[j + n01 + n0], c, step1), xhat_of(p[j + n01 + n0 + 1], c, step1), t0);
        g = lerpf_(g, lerpf_(c01, c11, t1), t2);
    }
    int q = code - MC_R;
    if (LEARNED) {
        const long long blk = v / MC_BLOCK;
        if ((bflags[blk >> 5] >> (blk & 31)) & 1u) q += rho_q[v];
    }
    xout[v] = (T)((double)g + (double)q * step2);
}

__global__ void k_zero_u32(unsigned int* a, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = 0u;
}

namespace mck {

hipError_t zero_u32(unsigned int* a, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    ProfScope ps("k_zero", s);
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n);
    return hipGetLastError();
}

hipError_t grid_decode(const uint16_t* codes, const int32_t* oidx, const int32_t* odelta, long long gcap,
                       const mc_result* res, int dim, int n0, int n1, int n2, int32_t* p, const DecodeWs& ws, hipStream_t s)
{
    hipError_t e;
    {
        ProfScope ps("k_dec_xy", s);
        const int cpt = (n0 + 255) / 256;
        dim3 grid((unsigned)((long long)ws.nyc * n2));
#define MC_DXY(C) hipLaunchKernelGGL(k_dec_xy<C>, grid, dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, n1, n2, ws.rows, \
                                     ws.nyc, p, ws.agg_xy, ws.incl_xy, ws.flag_xy, ws.tickets)
        if (cpt <= 1) MC_DXY(1);
        else if (cpt <= 2) MC_DXY(2);
        else if (cpt <= 4) MC_DXY(4);
        else if (cpt <= 8) MC_DXY(8);
        else if (cpt <= 16) MC_DXY(16);
        else MC_DXY(32);
#undef MC_DXY
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (dim == 3) {
        ProfScope ps("k_dec_z", s);
        const long long nxy = (long long)n0 * n1;
        dim3 grid((unsigned)((long long)ws.nzc * ws.nxyb));
        hipLaunchKernelGGL(k_dec_z, grid, dim3(256), 0, s, p, nxy, n2, ws.zplanes, ws.nxyb, ws.agg_z, ws.incl_z,
                           ws.flag_z, ws.tickets + 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t vertex_decode(const float* coords, long long nv, GridGeom gg, const int32_t* p, const uint16_t* codes,
                         const int32_t* oidx, const void* oval, long long vcap, const mc_result* res,
                         const int32_t* rho_q, const uint32_t* bflags, void* xout, int dtype, hipStream_t s)
{
    ProfScope ps(rho_q ? "k_vdecode_learned" : "k_vdecode", s);
    dim3 grid((unsigned)((nv + 255) / 256));
#define MC_VD(T, D, L) hipLaunchKernelGGL((k_vdecode<T, D, L>), grid, dim3(256), 0, s, coords, nv, gg, p, codes, oidx, \
                                          (const T*)oval, res, vcap, rho_q, bflags, (T*)xout)
    const bool L = rho_q != nullptr;
    if (dtype == MC_F64) {
        if (gg.dim == 2) { if (L) MC_VD(double, 2, true); else MC_VD(double, 2, false); }
        else { if (L) MC_VD(double, 3, true); else MC_VD(double, 3, false); }
    } else {
        if (gg.dim == 2) { if (L) MC_VD(float, 2, true); else MC_VD(float, 2, false); }
        else { if (L) MC_VD(float, 3, true); else MC_VD(float, 3, false); }
    }
#undef MC_VD
    return hipGetLastError();
}

}  // namespace mck
