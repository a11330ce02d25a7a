// k_decode.hip -- decompression on gfx950 (paper Alg. 4).
//   k_dec_xy_* Lorenzo inverse within each z-plane: d = code - R (outliers
//              by binary search in the ascending outlier list); column
//              totals per chunk of rows, their prefix over the plane's
//              chunks, then running column sums plus a wave scan along x
//   k_dec_z_*  (3-D) inclusive prefix along z in chunks of planes: totals,
//              prefix over the chunks, apply; in place
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

// Exclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ int wave_excl_scan(int v)
{
    return wave_incl_scan(v) - v;
}

// The grid decoder is the inclusive prefix sum of the Lorenzo errors along
// every axis.  In 3-D the z prefix runs first (on the decoded errors), then
// the 2-D prefix of each plane; the last pass writes x1' = (float)(c + p *
// 2 tau1) directly.  Tiles: (chunk of rows) x (all x) per plane for the xy
// part, (chunk of planes) x (the same chunk of rows) for the z part, so the
// z pass can also emit the xy column totals.
//   k_dec_xy_tot    2-D: column totals of each (plane, row chunk) tile
//   k_dec_xy_carry  per (plane, column): exclusive prefix over row chunks
//   k_dec_xy_apply  running column sums from the carry, x-scan of each row,
//                   x1' written (input: codes in 2-D, z-prefixed errors in 3-D)
//   k_dec_z_tot     3-D: per (plane chunk, position): sum of the errors
//   k_dec_z_carry   per position: exclusive prefix over plane chunks
//   k_dec_z_apply   z-prefixed errors + xy column totals of every tile
template <int CPT>
__global__ __launch_bounds__(256) void k_dec_xy_tot(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                    const int32_t* __restrict__ odelta,
                                                    const mc_result* __restrict__ res, long long gcap, int n0, int n1,
                                                    int rows, int nyc, long long ntiles, int* __restrict__ agg)
{
    const long long tile = (long long)xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const int z = (int)(tile / nyc), yc = (int)(tile % nyc);
    const int y0 = yc * rows, y1 = min(n1, y0 + rows);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const int c0 = lane_id() * CPT;
    const long long plane = (long long)z * n1 * n0;
    int tot[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) tot[k] = 0;
    for (int y = y0; y < y1; ++y) {
        const long long base_r = plane + (long long)y * n0;
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (c0 + k < n0) tot[k] += delta_at(codes, oidx, odelta, nout, base_r + c0 + k);
    }
#pragma unroll
    for (int k = 0; k < CPT; ++k)
        if (c0 + k < n0) agg[tile * n0 + c0 + k] = tot[k];
}

__global__ __launch_bounds__(256) void k_dec_xy_carry(int* __restrict__ agg, int n0, int n2, int nyc)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n0 * n2) return;
    const long long z = i / n0, c = i % n0;
    int run = 0;
    int yc = 0;
    for (; yc + 8 <= nyc; yc += 8) {
        int t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = agg[(z * nyc + yc + u) * n0 + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            agg[(z * nyc + yc + u) * n0 + c] = run;
            run += t[u];
        }
    }
    for (; yc < nyc; ++yc) {
        const long long k = (z * nyc + yc) * n0 + c;
        const int t = agg[k];
        agg[k] = run;
        run += t;
    }
}

template <int CPT, bool FROM_CODES>
__global__ __launch_bounds__(256) void k_dec_xy_apply(const uint16_t* __restrict__ codes,
                                                      const int32_t* __restrict__ oidx,
                                                      const int32_t* __restrict__ odelta,
                                                      const int32_t* __restrict__ pz,
                                                      const mc_result* __restrict__ res, long long gcap, int n0,
                                                      int n1, int rows, int nyc, long long ntiles,
                                                      const int* __restrict__ carry, float* __restrict__ xh)
{
    const long long tile = (long long)xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const int z = (int)(tile / nyc), yc = (int)(tile % nyc);
    const int y0 = yc * rows, y1 = min(n1, y0 + rows);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const double c = res->c, step1 = 2.0 * res->tau1;
    const int c0 = lane_id() * CPT;
    const long long plane = (long long)z * n1 * n0;
    int col[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) col[k] = c0 + k < n0 ? carry[tile * n0 + c0 + k] : 0;
    for (int y = y0; y < y1; ++y) {
        const long long base_r = plane + (long long)y * n0;
        int s[CPT];
        int run = 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            if (c0 + k < n0)
                col[k] += FROM_CODES ? delta_at(codes, oidx, odelta, nout, base_r + c0 + k) : pz[base_r + c0 + k];
            run += (c0 + k < n0) ? col[k] : 0;
            s[k] = run;
        }
        const int off = wave_excl_scan(run);
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (c0 + k < n0) xh[base_r + c0 + k] = xhat_of(off + s[k], c, step1);
    }
}

// 3-D z part.  Workgroup tile = (chunk of ZC planes) x (rows [y0, y1)) x
// (all x); thread t owns columns t, t+256, ... (CX of them).
template <int CX>
__global__ __launch_bounds__(256) void k_dec_z_tot(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                   const int32_t* __restrict__ odelta,
                                                   const mc_result* __restrict__ res, long long gcap, int n0, int n1,
                                                   int n2, int rows, int nyc, int zplanes, int* __restrict__ aggz)
{
    const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);
    const int zc = tile / nyc, yc = tile % nyc;
    const int y0 = yc * rows, y1 = min(n1, y0 + rows);
    const int z0 = zc * zplanes, z1 = min(n2, z0 + zplanes);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const long long nxy = (long long)n0 * n1;
    for (int y = y0; y < y1; ++y)
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            const int x = threadIdx.x + 256 * k;
            if (x >= n0) continue;
            int t = 0;
#pragma unroll 4
            for (int z = z0; z < z1; ++z) t += delta_at(codes, oidx, odelta, nout, (long long)z * nxy + (long long)y * n0 + x);
            aggz[(long long)zc * nxy + (long long)y * n0 + x] = t;
        }
}

__global__ __launch_bounds__(256) void k_dec_z_carry(int* __restrict__ aggz, long long nxy, int nzc)
{
    const long long pos = (long long)blockIdx.x * 256 + threadIdx.x;
    if (pos >= nxy) return;
    int run = 0;
    int zc = 0;
    for (; zc + 8 <= nzc; zc += 8) {
        int t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = aggz[(long long)(zc + u) * nxy + pos];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            aggz[(long long)(zc + u) * nxy + pos] = run;
            run += t[u];
        }
    }
    for (; zc < nzc; ++zc) {
        const long long k = (long long)zc * nxy + pos;
        const int t = aggz[k];
        aggz[k] = run;
        run += t;
    }
}

template <int CX>
__global__ __launch_bounds__(256) void k_dec_z_apply(const uint16_t* __restrict__ codes,
                                                     const int32_t* __restrict__ oidx,
                                                     const int32_t* __restrict__ odelta,
                                                     const mc_result* __restrict__ res, long long gcap, int n0, int n1,
                                                     int n2, int rows, int nyc, int zplanes,
                                                     const int* __restrict__ carryz, int32_t* __restrict__ pz,
                                                     int* __restrict__ agg_xy)
{
    const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);
    const int zc = tile / nyc, yc = tile % nyc;
    const int y0 = yc * rows, y1 = min(n1, y0 + rows);
    const int z0 = zc * zplanes, z1 = min(n2, z0 + zplanes);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const long long nxy = (long long)n0 * n1;
    constexpr int RMAX = (32 / CX) > 16 ? 16 : (32 / CX);     // rows per tile never exceed this
    int run[RMAX][CX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            const int x = threadIdx.x + 256 * k, y = y0 + r;
            run[r][k] = (x < n0 && y < y1) ? carryz[(long long)zc * nxy + (long long)y * n0 + x] : 0;
        }
    for (int z = z0; z < z1; ++z) {
        int colsum[CX];
#pragma unroll
        for (int k = 0; k < CX; ++k) colsum[k] = 0;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int y = y0 + r;
            if (y >= y1) continue;
#pragma unroll
            for (int k = 0; k < CX; ++k) {
                const int x = threadIdx.x + 256 * k;
                if (x >= n0) continue;
                const long long j = (long long)z * nxy + (long long)y * n0 + x;
                run[r][k] += delta_at(codes, oidx, odelta, nout, j);
                pz[j] = run[r][k];
                colsum[k] += run[r][k];
            }
        }
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            const int x = threadIdx.x + 256 * k;
            if (x < n0) agg_xy[((long long)z * nyc + yc) * n0 + x] = colsum[k];
        }
    }
}

template <typename T, int D, bool LEARNED>
__global__ __launch_bounds__(256) void k_vdecode(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                 const float* __restrict__ xh, const uint16_t* __restrict__ codes,
                                                 const int32_t* __restrict__ oidx, const T* __restrict__ oval,
                                                 const mc_result* __restrict__ res, long long vcap,
                                                 const int32_t* __restrict__ rho_q,
                                                 const uint32_t* __restrict__ bflags, T* __restrict__ xout)
{
    const long long v = (long long)xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (v >= nv) return;
    const int code = codes[v];
    if (code == 0) {
        const long long n = res->n_vertex_outliers < vcap ? res->n_vertex_outliers : vcap;
        const long long k = find_outlier(oidx, n, v);
        xout[v] = k >= 0 ? oval[k] : (T)0;
        return;
    }
    const double step2 = 2.0 * res->tau2;
    int i0, i1, i2 = 0;
    float t0, t1, t2 = 0.0f;
    axis_cell(coords[v], gg.of[0], gg.ihf[0], gg.n0, i0, t0);
    axis_cell(coords[nv + v], gg.of[1], gg.ihf[1], gg.n1, i1, t1);
    if (D == 3) axis_cell(coords[2 * nv + v], gg.of[2], gg.ihf[2], gg.n2, i2, t2);
    const int n0 = gg.n0;
    const unsigned n01 = (unsigned)gg.n0 * (unsigned)gg.n1;
    const unsigned j = (unsigned)i0 + (unsigned)n0 * (unsigned)i1 + n01 * (unsigned)i2;
    const float c00 = lerpf_(xh[j], xh[j + 1], t0);
    const float c10 = lerpf_(xh[j + n0], xh[j + n0 + 1], t0);
    float g = lerpf_(c00, c10, t1);
    if (D == 3) {
        const float c01 = lerpf_(xh[j + n01], xh[j + n01 + 1], t0);
        const float c11 = lerpf_(xh[j + n01 + n0], xh[j + n01 + n0 + 1], t0);
        g = lerpf_(g, lerpf_(c01, c11, t1), t2);
    }
    int q = code - MC_R;
    if (LEARNED) {
        const long long blk = v / MC_LBLOCK;
        if ((bflags[blk >> 5] >> (blk & 31)) & 1u) q += rho_q[v];
    }
    xout[v] = (T)((double)g + (double)q * step2);
}

namespace mck {

hipError_t grid_decode(const uint16_t* codes, const int32_t* oidx, const int32_t* odelta, long long gcap,
                       const mc_result* res, int dim, int n0, int n1, int n2, int32_t* pz, float* xh, DecodeWs& ws,
                       hipStream_t s)
{
    hipError_t e;
    const int cpt = (n0 + 63) / 64;
    const unsigned nb_xy = (unsigned)((ws.ntiles_xy + 3) / 4);
    if (dim == 2) {
        ProfScope ps("k_dec_xy_tot", s);
#define MC_DXT(C) hipLaunchKernelGGL(k_dec_xy_tot<C>, dim3(nb_xy), dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, \
                                     n1, ws.rows, ws.nyc, ws.ntiles_xy, ws.agg_xy)
        if (cpt <= 1) MC_DXT(1);
        else if (cpt <= 2) MC_DXT(2);
        else if (cpt <= 4) MC_DXT(4);
        else if (cpt <= 8) MC_DXT(8);
        else if (cpt <= 16) MC_DXT(16);
        else if (cpt <= 32) MC_DXT(32);
        else if (cpt <= 64) MC_DXT(64);
        else MC_DXT(128);
#undef MC_DXT
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        const long long nxy = (long long)n0 * n1;
        const int cx = (n0 + 255) / 256;
        const unsigned nb_z = (unsigned)(ws.nzc * ws.nyc);
        {
            ProfScope ps("k_dec_z_tot", s);
#define MC_DZT(C) hipLaunchKernelGGL(k_dec_z_tot<C>, dim3(nb_z), dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, n1, \
                                     n2, ws.rows, ws.nyc, ws.zplanes, ws.agg_z)
            if (cx <= 1) MC_DZT(1);
            else if (cx <= 2) MC_DZT(2);
            else if (cx <= 4) MC_DZT(4);
            else if (cx <= 8) MC_DZT(8);
            else if (cx <= 16) MC_DZT(16);
            else MC_DZT(32);
#undef MC_DZT
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        {
            ProfScope ps("k_dec_z_carry", s);
            hipLaunchKernelGGL(k_dec_z_carry, dim3((unsigned)((nxy + 255) / 256)), dim3(256), 0, s, ws.agg_z, nxy,
                               ws.nzc);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        {
            ProfScope ps("k_dec_z_apply", s);
#define MC_DZA(C) hipLaunchKernelGGL(k_dec_z_apply<C>, dim3(nb_z), dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, \
                                     n1, n2, ws.rows, ws.nyc, ws.zplanes, ws.agg_z, pz, ws.agg_xy)
            if (cx <= 1) MC_DZA(1);
            else if (cx <= 2) MC_DZA(2);
            else if (cx <= 4) MC_DZA(4);
            else if (cx <= 8) MC_DZA(8);
            else if (cx <= 16) MC_DZA(16);
            else MC_DZA(32);
#undef MC_DZA
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    {
        ProfScope ps("k_dec_xy_carry", s);
        hipLaunchKernelGGL(k_dec_xy_carry, dim3((unsigned)(((long long)n0 * n2 + 255) / 256)), dim3(256), 0, s,
                           ws.agg_xy, n0, n2, ws.nyc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        ProfScope ps("k_dec_xy_apply", s);
#define MC_DXA(C, F) hipLaunchKernelGGL((k_dec_xy_apply<C, F>), dim3(nb_xy), dim3(256), 0, s, codes, oidx, odelta, pz, res, \
                                        gcap, n0, n1, ws.rows, ws.nyc, ws.ntiles_xy, ws.agg_xy, xh)
#define MC_DXA2(C) do { if (dim == 2) MC_DXA(C, true); else MC_DXA(C, false); } while (0)
        if (cpt <= 1) MC_DXA2(1);
        else if (cpt <= 2) MC_DXA2(2);
        else if (cpt <= 4) MC_DXA2(4);
        else if (cpt <= 8) MC_DXA2(8);
        else if (cpt <= 16) MC_DXA2(16);
        else if (cpt <= 32) MC_DXA2(32);
        else if (cpt <= 64) MC_DXA2(64);
        else MC_DXA2(128);
#undef MC_DXA2
#undef MC_DXA
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t vertex_decode(const float* coords, long long nv, GridGeom gg, const float* xh, const uint16_t* codes,
                         const int32_t* oidx, const void* oval, long long vcap, const mc_result* res,
                         const int32_t* rho_q, const uint32_t* bflags, void* xout, int dtype, hipStream_t s)
{
    ProfScope ps(rho_q ? "k_vdecode_learned" : "k_vdecode", s);
    dim3 grid((unsigned)((nv + 255) / 256));
#define MC_VD(T, D, L) hipLaunchKernelGGL((k_vdecode<T, D, L>), grid, dim3(256), 0, s, coords, nv, gg, xh, codes, oidx, \
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
