// k_compress.hip -- the compression hot path on gfx950 (paper Alg. 3 with
// the residual taken against the reconstructed grid):
//   k_range(_final)  field min/max (ordered integer keys: per-block partials,
//                    then one workgroup) and non-finite check; clears the
//                    per-call state of the kernels after it
//   k_resample       f: v_j = sum_k w_kj * x[vid_kj] (FP32, fixed order), the
//                    prequantised grid p_j = rint((v_j - c) / (2 tau1)) and,
//                    when a consumer reads it, the reconstructed grid
//                    x1'_j = (float)(c + p_j * 2 tau1)
//   k_lorenzo        Lorenzo prediction error of p, uint16 codes, per-tile
//                    outlier counts
//   k_residual       g: multilinear x1' at each vertex (corners read from x1',
//                    or from p and converted as the decoder does), residual
//                    quantisation with the per-vertex bound check, per-tile
//                    outlier counts
//   k_scatter        outlier lists in index order (wave ballots)
#include "mc_dev.h"
#include "mc_interp.h"
#include "mc_kernels.h"

// ---------------------------------------------------------------------------
// Block b of nb: min/max keys and non-finite flag of its share of x (a
// grid-stride loop over nb blocks), written to partial[3b..3b+2]; the
// blocks also clear zero[0, nzero).
template <typename T, bool VEC>
__device__ __forceinline__ void range_block(unsigned b, unsigned nb, const T* __restrict__ x, long long n,
                                            unsigned long long* __restrict__ partial, unsigned int* __restrict__ zero,
                                            long long nzero)
{
    __shared__ unsigned long long s_mn[4], s_mx[4];
    __shared__ unsigned int s_fl[4];
    const long long stride = (long long)nb * 256;
    const long long gid = (long long)b * 256 + threadIdx.x;
    for (long long i = gid; i < nzero; i += stride) zero[i] = 0u;
    // running extremes in the field's own type (min and max are exact, so
    // widening the two results gives the same keys as widening every value)
    T mn = (T)__builtin_inf(), mx = -(T)__builtin_inf();
    bool bad = false;
    if (VEC) {
        // quads of 16-byte aligned values, 4 quads per thread in flight
        const long long nq = n / 4;
        constexpr int UQ = 8;
        long long q = gid;
        for (; q + (UQ - 1) * stride < nq; q += UQ * stride) {
            Quad<T> v[UQ];
#pragma unroll
            for (int u = 0; u < UQ; ++u) v[u] = load_quad(x + 4 * (q + u * stride));
#pragma unroll
            for (int u = 0; u < UQ; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const T d = v[u].v[e];
                    bad |= !isfinite(d);
                    mn = fmin(mn, d);
                    mx = fmax(mx, d);
                }
        }
        for (; q < nq; q += stride) {
            const Quad<T> v = load_quad(x + 4 * q);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const T d = v.v[e];
                bad |= !isfinite(d);
                mn = fmin(mn, d);
                mx = fmax(mx, d);
            }
        }
        if (gid < n - 4 * nq) {
            const T d = x[4 * nq + gid];
            bad |= !isfinite(d);
            mn = fmin(mn, d);
            mx = fmax(mx, d);
        }
    }
    constexpr int U = 8;
    long long i = VEC ? n : gid;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = x[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T d = v[u];
            bad |= !isfinite(d);
            mn = fmin(mn, d);
            mx = fmax(mx, d);
        }
    }
    for (; i < n; i += stride) {
        const T d = x[i];
        bad |= !isfinite(d);
        mn = fmin(mn, d);
        mx = fmax(mx, d);
    }
    // keys of the per-thread extremes (-0 and +0 share a key; an empty
    // thread contributes the neutral keys)
    unsigned long long kmn = mn <= mx ? dkey((double)mn) : ~0ull;
    unsigned long long kmx = mn <= mx ? dkey((double)mx) : 0ull;
    unsigned int fl = bad ? MC_EBIT_NONFINITE : 0u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long a = __shfl_xor(kmn, d, 64), b = __shfl_xor(kmx, d, 64);
        fl |= __shfl_xor(fl, d, 64);
        kmn = a < kmn ? a : kmn;
        kmx = b > kmx ? b : kmx;
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) { s_mn[w] = kmn; s_mx[w] = kmx; s_fl[w] = fl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            kmn = s_mn[k] < kmn ? s_mn[k] : kmn;
            kmx = s_mx[k] > kmx ? s_mx[k] : kmx;
            fl |= s_fl[k];
        }
        partial[3 * b] = kmn;
        partial[3 * b + 1] = kmx;
        partial[3 * b + 2] = fl;
    }
}

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_range(const T* __restrict__ x, long long n,
                                               unsigned long long* __restrict__ partial,
                                               unsigned int* __restrict__ zero, long long nzero)
{
    range_block<T, VEC>(blockIdx.x, gridDim.x, x, n, partial, zero, nzero);
}

// One workgroup folds the per-block partials into the range slot and
// computes the error split once.
__device__ __forceinline__ void range_final_block(const unsigned long long* __restrict__ partial, int nparts,
                                                  RangeOut* __restrict__ out, BoundParams bp,
                                                  DevBound* __restrict__ bout)
{
    __shared__ unsigned long long s_mn[4], s_mx[4];
    __shared__ unsigned int s_fl[4];
    unsigned long long kmn = ~0ull, kmx = 0ull;
    unsigned int fl = 0;
    for (int i0 = threadIdx.x; i0 < nparts; i0 += 256 * 8) {      // 8 partials per thread in flight
        unsigned long long a[8], b[8], f[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = min(i0 + 256 * u, nparts - 1);
            a[u] = partial[3 * i];
            b[u] = partial[3 * i + 1];
            f[u] = partial[3 * i + 2];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            kmn = a[u] < kmn ? a[u] : kmn;
            kmx = b[u] > kmx ? b[u] : kmx;
            fl |= (unsigned)f[u];
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long a = __shfl_xor(kmn, d, 64), b = __shfl_xor(kmx, d, 64);
        fl |= __shfl_xor(fl, d, 64);
        kmn = a < kmn ? a : kmn;
        kmx = b > kmx ? b : kmx;
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) { s_mn[w] = kmn; s_mx[w] = kmx; s_fl[w] = fl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            kmn = s_mn[k] < kmn ? s_mn[k] : kmn;
            kmx = s_mx[k] > kmx ? s_mx[k] : kmx;
            fl |= s_fl[k];
        }
        RangeOut r;
        r.kmin = kmn;
        r.kmax = kmx;
        r.flags = fl;
        r.pad = 0;
        *out = r;
        *bout = make_bound(&r, bp);
    }
}

__global__ __launch_bounds__(256) void k_range_final(const unsigned long long* __restrict__ partial, int nparts,
                                                     RangeOut* __restrict__ out, BoundParams bp,
                                                     DevBound* __restrict__ bout)
{
    range_final_block(partial, nparts, out, bp, bout);
}

// ---------------------------------------------------------------------------
template <typename T, int D, bool NT>
__device__ __forceinline__ void resample_block(unsigned t, const int32_t* __restrict__ vid,
                                               const float* __restrict__ w, long long ng, const T* __restrict__ x,
                                               const DevBound* __restrict__ bnd, int32_t* __restrict__ p,
                                               float* __restrict__ xh, float* __restrict__ dbg_v,
                                               uint32_t* __restrict__ bflags, long long nbflags,
                                               unsigned int* __restrict__ err, mc_result* __restrict__ res,
                                               int dtype, unsigned int* __restrict__ gcount, long long ntg)
{
    const DevBound b = *bnd;
    const long long j = (long long)t * 256 + threadIdx.x;
    if (bflags && j < nbflags) bflags[j] = 0u;      // learned-block bits start clear
    if (j < ntg) gcount[j] = 0u;                    // grid outlier counts (k_lorenzo adds)
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
    // all mapping loads, then all field gathers (a node with vid < 0 is a
    // mid-range fill and gathers vertex 0 for nothing)
    int id[D + 1];
    float wk[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        id[k] = ld_s<NT>(vid + k * ng + j);
        wk[k] = ld_s<NT>(w + k * ng + j);
    }
    const bool fill = id[0] < 0;
    float f[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) f[k] = as_float(x[fill ? 0 : id[k]]);
    float acc = wk[0] * f[0];
#pragma unroll
    for (int k = 1; k <= D; ++k) acc = acc + wk[k] * f[k];
    const float v = fill ? (float)b.c : acc;
    const double s = ((double)v - b.c) * b.inv1;
    int32_t q = 0;
    if (!(fabs(s) < 134217728.0)) atomicOr(err, MC_EBIT_RANGE);
    else q = (int32_t)rint(s);
    p[j] = q;
    if (xh) xh[j] = xhat_of(q, b.c, b.step1);      // reconstructed grid x1', as the decoder rebuilds it
    if (dbg_v) dbg_v[j] = v;
}

template <typename T, int D, bool NT>
__global__ __launch_bounds__(256) void k_resample(const int32_t* __restrict__ vid, const float* __restrict__ w,
                                                  long long ng, const T* __restrict__ x,
                                                  const DevBound* __restrict__ bnd,
                                                  int32_t* __restrict__ p, float* __restrict__ xh,
                                                  float* __restrict__ dbg_v, uint32_t* __restrict__ bflags,
                                                  long long nbflags, unsigned int* __restrict__ err,
                                                  mc_result* __restrict__ res, int dtype,
                                                  unsigned int* __restrict__ gcount, long long ntg, unsigned remap)
{
    resample_block<T, D, NT>(tile_of(remap), vid, w, ng, x, bnd, p, xh, dbg_v, bflags, nbflags, err, res, dtype,
                             gcount, ntg);
}

// ---------------------------------------------------------------------------
// Lorenzo prediction error at node j (zeros outside the grid), int64.
template <int D>
__device__ __forceinline__ long long lorenzo_delta(const int32_t* __restrict__ p, long long j, int i0, int i1, int i2,
                                                   long long n0, long long n01)
{
    const long long a = i0 > 0 ? p[j - 1] : 0;
    const long long bq = i1 > 0 ? p[j - n0] : 0;
    const long long ab = (i0 > 0 && i1 > 0) ? p[j - n0 - 1] : 0;
    long long pred;
    if (D == 2) {
        pred = a + bq - ab;
    } else {
        const long long cz = i2 > 0 ? p[j - n01] : 0;
        const long long ac = (i0 > 0 && i2 > 0) ? p[j - n01 - 1] : 0;
        const long long bc = (i1 > 0 && i2 > 0) ? p[j - n01 - n0] : 0;
        const long long abc = (i0 > 0 && i1 > 0 && i2 > 0) ? p[j - n01 - n0 - 1] : 0;
        pred = a + bq + cz - ab - ac - bc + abc;
    }
    return (long long)p[j] - pred;
}

// Lorenzo codes by line sweeps.  The 3-D predictor error is the difference
// of the 2-D (x, y) errors of consecutive z planes,
//   d3(x,y,z) = d2(x,y,z) - d2(x,y,z-1),
//   d2(x,y,z) = p(x,y,z) - p(x-1,y,z) - p(x,y-1,z) + p(x-1,y-1,z),
// and the 2-D error the difference of the 1-D (x) errors of consecutive
// rows, with zero outside the grid; both regroup the terms of the Lorenzo
// formula exactly.  |p| < 2^27 keeps every partial in int32.  A wave owns
// 63 consecutive x of one row (3-D) or of a run of rows (2-D); its lane 0
// loads the column to their left, and every lane takes its x - 1
// neighbours from the lane below with a whole-wave DPP shift, so a node
// costs two loads (3-D) or one (2-D).  The wave sweeps MC_LZ_CHUNK planes
// (rows), carrying the previous plane's (row's) error in a register.  The
// launcher runs this kernel for 2-D grids; 3-D grids use k_lorenzo3 below,
// which also keeps the previous row in registers.
// Outliers are counted per 1024-node tile and per group of tiles with at
// most two atomics each per wave and row (a 63-run meets at most two
// tiles); the counts were zeroed before the kernel.
#define MC_LZ_W 63

__device__ __forceinline__ int lane_below(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);   // wave_shr:1 (lane 0 gets 0)
}

// Loads are unconditional (addresses clamped into the grid, neighbours
// outside it masked with bitwise ands, not selects) so that the compiler
// keeps a sweep's loads together instead of sinking them into branches.
template <int D>
__device__ __forceinline__ int lz_line(const int32_t* __restrict__ p, unsigned j, bool hx, bool hy, unsigned n0)
{
    const int mx = -(int)hx, my = -(int)hy;
    const int a = p[j];
    const int b = lane_below(a);
    if (D == 2) return a - (b & mx);
    const int c = p[hy ? j - n0 : j];
    const int e = lane_below(c);
    return ((a - (b & mx)) - (c & my)) + (e & (mx & my));
}

__device__ __forceinline__ void lz_count(unsigned j, bool out, bool act, unsigned int* __restrict__ count,
                                         unsigned int* __restrict__ gsum)
{
    const unsigned long long m = __ballot(out);
    if (m == 0ull) return;
    const unsigned long long live = __ballot(act);
    const int first = __builtin_ctzll(live), last = 63 - __builtin_clzll(live);
    const unsigned jf = __shfl(j, first, 64), jl = __shfl(j, last, 64);
    const unsigned tf = jf / MC_TILE, tl = jl / MC_TILE;
    const unsigned long long lo = __ballot(out && j / MC_TILE == tf), hi = m & ~lo;
    if (lane_id() == first) {
        if (lo) {
            atomicAdd(&count[tf], (unsigned)__popcll(lo));
            atomicAdd(&gsum[tf / MC_SC_TILES], (unsigned)__popcll(lo));
        }
        if (hi) {
            atomicAdd(&count[tl], (unsigned)__popcll(hi));
            atomicAdd(&gsum[tl / MC_SC_TILES], (unsigned)__popcll(hi));
        }
    }
}

template <int D>
__device__ __forceinline__ void lorenzo_block(unsigned t, const int32_t* __restrict__ p, int n0, int n1, int n2,
                                              int nxs, unsigned nunits, uint16_t* __restrict__ codes,
                                              unsigned int* __restrict__ count, unsigned int* __restrict__ gsum)
{
    const unsigned u = t * 4u + (threadIdx.x >> 6);
    if (u >= nunits) return;
    const unsigned xs = u % (unsigned)nxs, r = u / (unsigned)nxs;
    const int x = (int)(xs * MC_LZ_W) + lane_id() - 1;      // lane 0: the column to the left
    const bool act = lane_id() > 0 && x < n0, hx = x > 0;
    const unsigned xl = (unsigned)min(max(x, 0), n0 - 1);
    constexpr int CH = MC_LZ_CHUNK;
    unsigned base, step;
    int l0, l1;
    bool hy = false;
    if (D == 3) {
        const unsigned y = r % (unsigned)n1, zc = r / (unsigned)n1;
        base = xl + (unsigned)n0 * y;
        step = (unsigned)n0 * (unsigned)n1;
        l0 = (int)zc * CH;
        l1 = min(l0 + CH, n2);
        hy = y > 0;
    } else {
        base = xl;
        step = (unsigned)n0;
        l0 = (int)r * CH;
        l1 = min(l0 + CH, n1);
    }
    // plane (row) l0 - 1 for the first difference; past the end, the last
    // plane (row) is read again and ignored
    const int pz = lz_line<D>(p, base + step * (unsigned)(l0 > 0 ? l0 - 1 : 0), hx, hy, (unsigned)n0);
    int prev = l0 > 0 ? pz : 0;
    int cur[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) cur[k] = lz_line<D>(p, base + step * (unsigned)min(l0 + k, l1 - 1), hx, hy, (unsigned)n0);
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        if (l0 + k >= l1) break;
        const int d = cur[k] - prev;
        prev = cur[k];
        const unsigned j = base + step * (unsigned)(l0 + k);
        const bool in = d >= -(MC_R - 1) && d <= MC_R - 1;
        if (act) codes[j] = in ? (uint16_t)(d + MC_R) : (uint16_t)0;
        lz_count(j, act && !in, act, count, gsum);
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_lorenzo(const int32_t* __restrict__ p, int n0, int n1, int n2, int nxs,
                                                 unsigned nunits, uint16_t* __restrict__ codes,
                                                 unsigned int* __restrict__ count, unsigned int* __restrict__ gsum,
                                                 unsigned remap)
{
    lorenzo_block<D>(tile_of(remap), p, n0, n1, n2, nxs, nunits, codes, count, gsum);
}

// 3-D Lorenzo codes with MC_LZ_RY rows per wave: a wave owns 63 columns of
// MC_LZ_RY consecutive rows over MC_LZ3_CH planes and loads each row's
// MC_LZ3_CH + 1 planes once (plus the row before the first), so a node
// costs (RY + 1) / RY * (CH + 1) / CH loads instead of two; the y - 1 terms
// come from the previous row's registers.  Same regrouping as k_lorenzo:
//   line(y, z) = ((a - a_x-1) - a_y-1) + a_x-1,y-1,   d3 = line(z) - line(z-1).
// 4 x 4 measured fastest on the 256^3 grid (25.7 us; 4 x 16: 38.6 us, fewer
// waves in flight; two loads per node: 31-32 us).
#ifndef MC_LZ_RY
#define MC_LZ_RY 4
#endif
#ifndef MC_LZ3_CH
#define MC_LZ3_CH 4
#endif

__device__ __forceinline__ void lorenzo3_block(unsigned t, const int32_t* __restrict__ p, int n0, int n1, int n2,
                                               int nxs, int nyb, unsigned nunits, uint16_t* __restrict__ codes,
                                               unsigned int* __restrict__ count, unsigned int* __restrict__ gsum)
{
    constexpr int CH = MC_LZ3_CH, RY = MC_LZ_RY;
    const unsigned u = t * 4u + (threadIdx.x >> 6);
    if (u >= nunits) return;
    const unsigned xs = u % (unsigned)nxs, r = u / (unsigned)nxs;
    const unsigned yb = r % (unsigned)nyb, zc = r / (unsigned)nyb;
    const int x = (int)(xs * MC_LZ_W) + lane_id() - 1;      // lane 0: the column to the left
    const bool act = lane_id() > 0 && x < n0, hx = x > 0;
    const int mx = -(int)hx;
    const unsigned xl = (unsigned)min(max(x, 0), n0 - 1);
    const unsigned plane = (unsigned)n0 * (unsigned)n1;
    const int l0 = (int)zc * CH, l1 = min(l0 + CH, n2);
    const int y0 = (int)yb * RY;
    // planes l0 - 1 .. l0 + CH - 1 (clamped into [0, l1 - 1]; the extra ones are ignored)
    unsigned zoff[CH + 1];
#pragma unroll
    for (int k = 0; k <= CH; ++k) zoff[k] = plane * (unsigned)min(max(l0 - 1 + k, 0), l1 - 1);
    // every load first: the row before and the RY rows (rows past the grid clamped)
    int a[RY + 1][CH + 1];
#pragma unroll
    for (int rr = 0; rr <= RY; ++rr) {
        const unsigned yr = (unsigned)min(max(y0 - 1 + rr, 0), n1 - 1);
#pragma unroll
        for (int k = 0; k <= CH; ++k) a[rr][k] = p[xl + (unsigned)n0 * yr + zoff[k]];
    }
#pragma unroll
    for (int rr = 1; rr <= RY; ++rr) {
        const int y = y0 - 1 + rr;
        if (y >= n1) break;                              // uniform across the wave
        const int my = -(int)(y > 0), mxy = mx & my;
        int line[CH + 1];
#pragma unroll
        for (int k = 0; k <= CH; ++k) {
            const int c = a[rr - 1][k];
            line[k] = ((a[rr][k] - (lane_below(a[rr][k]) & mx)) - (c & my)) + (lane_below(c) & mxy);
        }
        int prev = l0 > 0 ? line[0] : 0;
#pragma unroll
        for (int k = 1; k <= CH; ++k) {
            const int z = l0 - 1 + k;
            if (z >= l1) break;
            const int d = line[k] - prev;
            prev = line[k];
            const unsigned j = xl + (unsigned)n0 * (unsigned)y + plane * (unsigned)z;
            const bool in = d >= -(MC_R - 1) && d <= MC_R - 1;
            if (act) codes[j] = in ? (uint16_t)(d + MC_R) : (uint16_t)0;
            lz_count(j, act && !in, act, count, gsum);
        }
    }
}

__global__ __launch_bounds__(256) void k_lorenzo3(const int32_t* __restrict__ p, int n0, int n1, int n2, int nxs,
                                                  int nyb, unsigned nunits, uint16_t* __restrict__ codes,
                                                  unsigned int* __restrict__ count, unsigned int* __restrict__ gsum,
                                                  unsigned remap)
{
    lorenzo3_block(tile_of(remap), p, n0, n1, n2, nxs, nyb, nunits, codes, count, gsum);
}

// ---------------------------------------------------------------------------
// Residual codes of one tile (1024 vertices) and its outlier count.
template <typename T, int D, bool FROM_P, bool NT>
__device__ __forceinline__ void residual_block(long long tile, const float* __restrict__ coords, long long nv,
                                               const GridGeom& gg, const void* __restrict__ xh,
                                               const T* __restrict__ x, const DevBound* __restrict__ bnd,
                                               uint16_t* __restrict__ codes, float* __restrict__ dbg_g,
                                               unsigned int* __restrict__ count, unsigned int* __restrict__ vsum)
{
    __shared__ int s_cnt[4];
    const DevBound b = *bnd;
    long long v[MC_IPT];
    bool act[MC_IPT];
    T xv[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        v[i] = tile * MC_TILE + i * MC_WG + threadIdx.x;
        act[i] = v[i] < nv && b.ok;
        xv[i] = ld_s<NT>(x + (act[i] ? v[i] : 0));
    }
    float g[MC_IPT];
    back_interp_n<D, MC_IPT, FROM_P, NT>(coords, nv, gg, xh, b.c, b.step1, v, act, g);
    int nout = 0;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (!act[i]) continue;
        if (dbg_g) dbg_g[v[i]] = g[i];
        int qi;
        const bool ok = quantize_residual<T>(xv[i], g[i], b, qi);
        st_s<NT>(codes + v[i], ok ? (uint16_t)(qi + MC_R) : (uint16_t)0);
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

template <typename T, int D, bool FROM_P, bool NT>
__global__ __launch_bounds__(256) void k_residual(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                  const void* __restrict__ xh, const T* __restrict__ x,
                                                  const DevBound* __restrict__ bnd, uint16_t* __restrict__ codes,
                                                  float* __restrict__ dbg_g, unsigned int* __restrict__ count,
                                                  unsigned int* __restrict__ vsum, unsigned remap)
{
    residual_block<T, D, FROM_P, NT>(tile_of(remap), coords, nv, gg, xh, x, bnd, codes, dbg_g, count, vsum);
}

// Grid codes (Lorenzo) and vertex residual codes in one launch: the two
// read the prequantised grid and write disjoint outputs, so blocks
// [0, nbl) take Lorenzo units and the rest residual tiles (nbl a multiple
// of 8, so each part keeps its own XCD order); one launch boundary less,
// and the tail of one part overlaps the other.
// At most 80 VGPRs (6 waves per SIMD, from 84 and 5): more gathers in
// flight; 64 (8 waves) leaves fewer loads per wave and is slower.
template <typename T, int D, bool FROM_P, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_codes(const int32_t* __restrict__ p, int n0, int n1, int n2, int nxs,
                                               int nyb, unsigned nunits, uint16_t* __restrict__ gcodes,
                                               unsigned int* __restrict__ gcount, unsigned int* __restrict__ gsum,
                                               unsigned nbl, const float* __restrict__ coords, long long nv,
                                               GridGeom gg, const void* __restrict__ xh, const T* __restrict__ x,
                                               const DevBound* __restrict__ bnd, uint16_t* __restrict__ vcodes,
                                               float* __restrict__ dbg_g, unsigned int* __restrict__ vcount,
                                               unsigned int* __restrict__ vsum, unsigned remap_l, unsigned remap_r)
{
    const unsigned bi = blockIdx.x;
    if (bi < nbl) {
        const unsigned t = remap_l ? xcd_tile(bi, nbl) : bi;
        if (D == 3) lorenzo3_block(t, p, n0, n1, n2, nxs, nyb, nunits, gcodes, gcount, gsum);
        else lorenzo_block<2>(t, p, n0, n1, n2, nxs, nunits, gcodes, gcount, gsum);
    } else {
        const unsigned b = bi - nbl, nbr = gridDim.x - nbl;
        residual_block<T, D, FROM_P, NT>(remap_r ? xcd_tile(b, nbr) : b, coords, nv, gg, xh, x, bnd, vcodes, dbg_g,
                                          vcount, vsum);
    }
}

// Gathers the outliers in index order, one workgroup per group of
// MC_SC_TILES tiles (grid groups first, then vertex groups): a group with
// any outlier sums the group totals before it (its list offset), scans its
// own tile counts, and ranks each tile's code-0 items with wave ballots.
// Grid outliers get their prediction error (Lorenzo or interpolation)
// recomputed, vertex outliers the raw value.  Block 0 also writes the list totals, the count of learned blocks
// and the final status (capacity overflows included).
template <typename T, int D>
__device__ __forceinline__ void scatter_block(unsigned bidx, const int32_t* __restrict__ p, int n0, int n1,
                                              long long ng, int gpred, const float* __restrict__ gref,
                                              const uint16_t* __restrict__ gcodes,
                                              const unsigned int* __restrict__ gcount,
                                              const unsigned int* __restrict__ gsum, int32_t* __restrict__ gidx,
                                              int32_t* __restrict__ gdelta, long long gcap, long long ntg,
                                              const T* __restrict__ x, long long nv,
                                              const uint16_t* __restrict__ vcodes,
                                              const unsigned int* __restrict__ vcount,
                                              const unsigned int* __restrict__ vsum, int32_t* __restrict__ vidx,
                                              T* __restrict__ vval, long long vcap,
                                              const unsigned int* __restrict__ err, mc_result* __restrict__ res)
{
    __shared__ int s_cnt[MC_IPT * 4 + 1];
    __shared__ unsigned s_c[MC_SC_TILES], s_off[MC_SC_TILES];
    __shared__ unsigned long long s_red[3][4];
    const long long ntv = (nv + MC_TILE - 1) / MC_TILE;
    const long long ngg = (ntg + MC_SC_TILES - 1) / MC_SC_TILES, ngv = (ntv + MC_SC_TILES - 1) / MC_SC_TILES;
    const int w = threadIdx.x >> 6;
    if (bidx == 0) {
        // totals of both lists and the learned-block count (bit 31 marks the
        // first tile of a learned block: every MC_LBLOCK / MC_TILE-th tile),
        // all loads of the three sums issued before any is added
        unsigned long long tg = 0, tv = 0, nl = 0;
        const long long step = MC_LBLOCK / MC_TILE;
        const long long nlb = (ntv + step - 1) / step;
        for (long long i0 = threadIdx.x; i0 < ngg || i0 < ngv || i0 < nlb; i0 += 4 * 256) {
            unsigned a[4], b[4], c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long long i = i0 + 256 * u;
                a[u] = i < ngg ? gsum[i] : 0u;
                b[u] = i < ngv ? vsum[i] : 0u;
                c[u] = i < nlb ? vcount[i * step] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                tg += a[u];
                tv += b[u];
                nl += c[u] >> 31;
            }
        }
        tg = wave_sum(tg);
        tv = wave_sum(tv);
        nl = wave_sum(nl);
        if (lane_id() == 0) { s_red[0][w] = tg; s_red[1][w] = tv; s_red[2][w] = nl; }
        __syncthreads();
        if (threadIdx.x == 0) {
            tg = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
            tv = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
            nl = s_red[2][0] + s_red[2][1] + s_red[2][2] + s_red[2][3];
            unsigned e = *err;
            if ((long long)tg > gcap) e |= MC_EBIT_GCAP;
            if ((long long)tv > vcap) e |= MC_EBIT_VCAP;
            res->n_grid_outliers = (long long)tg;
            res->n_vertex_outliers = (long long)tv;
            res->n_learned_blocks = (long long)nl;
            res->status = status_from_bits(e);
        }
        __syncthreads();                           // s_red is reused below
    }
    const bool vert = bidx >= ngg;
    const long long grp = vert ? bidx - ngg : bidx;
    const long long ntl = vert ? ntv : ntg;
    const unsigned int* cnt = vert ? vcount : gcount;
    const long long t0 = grp * MC_SC_TILES;
    // the group's tile counts and its list offset (the sum of the group
    // totals before it) are loaded together, before either is known to be
    // needed: one round trip to memory instead of two
    if (threadIdx.x < MC_SC_TILES) {
        const long long t = t0 + threadIdx.x;
        s_c[threadIdx.x] = t < ntl ? (cnt[t] & 0x7fffffffu) : 0u;
    }
    const unsigned int* sums = vert ? vsum : gsum;
    unsigned long long before = 0;
    for (long long i0 = threadIdx.x; i0 < grp; i0 += 8 * 256) {
        unsigned a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = i0 + 256 * u < grp ? sums[i0 + 256 * u] : 0u;
#pragma unroll
        for (int u = 0; u < 8; ++u) before += a[u];
    }
    before = wave_sum(before);
    if (lane_id() == 0) s_red[0][w] = before;
    __syncthreads();
    unsigned any = 0;
#pragma unroll
    for (int k = 0; k < MC_SC_TILES; ++k) any |= s_c[k];
    if (any == 0) return;                          // uniform: no outlier in the group
    if (threadIdx.x == 0) {
        unsigned long long a = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
        for (int k = 0; k < MC_SC_TILES; ++k) {
            s_off[k] = (unsigned)a;
            a += s_c[k];
        }
    }
    __syncthreads();
    const long long n = vert ? nv : ng;
    const uint16_t* codes = vert ? vcodes : gcodes;
    const long long n01 = (long long)n0 * n1;
    for (int k = 0; k < MC_SC_TILES; ++k) {
        if (s_c[k] == 0) continue;                 // uniform across the workgroup
        const long long tile = t0 + k;
        bool flag[MC_IPT];
        int rank[MC_IPT];
        T xv[MC_IPT];                              // raw values loaded with the codes (vertex tiles)
#pragma unroll
        for (int i = 0; i < MC_IPT; ++i) {
            const long long j = tile * MC_TILE + i * MC_WG + threadIdx.x;
            flag[i] = j < n && codes[j] == 0;
            xv[i] = (vert && j < n) ? x[j] : (T)0;
        }
        tile_ranks(flag, rank, s_cnt);
        const long long base = s_off[k];
#pragma unroll
        for (int i = 0; i < MC_IPT; ++i) {
            if (!flag[i]) continue;
            const long long j = tile * MC_TILE + i * MC_WG + threadIdx.x;
            const long long pos = base + rank[i];
            if (vert) {
                if (pos < vcap) { vidx[pos] = (int32_t)j; vval[pos] = xv[i]; }
            } else if (pos < gcap) {
                const int i0 = (int)(j % n0);
                const long long r = j / n0;
                const int i1 = (int)(r % n1), i2 = (int)(r / n1), n2 = (int)(ng / n01);
                gidx[pos] = (int32_t)j;
                long long d;
                if (gpred == MC_GRIDPRED_LORENZO) d = lorenzo_delta<D>(p, j, i0, i1, i2, n0, n01);
                else if (gpred == MC_GRIDPRED_INTERP_CUBIC) d = ip_delta<true>(p, (int)j, i0, i1, i2, n0, n1, n2);
                else if (gpred == MC_GRIDPRED_INTERP_LINEAR) d = ip_delta<false>(p, (int)j, i0, i1, i2, n0, n1, n2);
                else d = (long long)p[j] - tp_pred(gref[j], res->c, 1.0 / (2.0 * res->tau1));
                gdelta[pos] = (int32_t)d;
            }
        }
        __syncthreads();                           // s_cnt is reused by the next tile
    }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ p, int n0, int n1, long long ng, int gpred,
                                                 const float* __restrict__ gref, const uint16_t* __restrict__ gcodes,
                                                 const unsigned int* __restrict__ gcount,
                                                 const unsigned int* __restrict__ gsum, int32_t* __restrict__ gidx,
                                                 int32_t* __restrict__ gdelta, long long gcap, long long ntg,
                                                 const T* __restrict__ x, long long nv,
                                                 const uint16_t* __restrict__ vcodes,
                                                 const unsigned int* __restrict__ vcount,
                                                 const unsigned int* __restrict__ vsum, int32_t* __restrict__ vidx,
                                                 T* __restrict__ vval, long long vcap,
                                                 const unsigned int* __restrict__ err, mc_result* __restrict__ res)
{
    scatter_block<T, D>(blockIdx.x, p, n0, n1, ng, gpred, gref, gcodes, gcount, gsum, gidx, gdelta, gcap, ntg, x, nv,
                        vcodes, vcount, vsum, vidx, vval, vcap, err, res);
}

// x1' of the whole grid from p (for consumers that read x1' after a plain
// compression that wrote only p).
__global__ __launch_bounds__(256) void k_xhat_from_p(const int32_t* __restrict__ p, long long ng,
                                                     const DevBound* __restrict__ bnd, float* __restrict__ xh)
{
    const double c = bnd->c, step1 = bnd->step1;
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (j < ng) xh[j] = xhat_of(p[j], c, step1);
}

// ---------------------------------------------------------------------------
// Batched stages: one launch per stage over the tiles of every field of a
// batch.  Block b belongs to the field i with base[i] <= b < base[i + 1]
// (binary search in the small base table; uniform over the block, so the
// field's descriptor is read with scalar loads) and runs that field's tile
// b - base[i] with the field's own types: fields of both value types and
// dimensions share one launch.
using mck::BItemC;
using mck::MC_KNOB_NT_MAP;
using mck::MC_KNOB_NT_VERT;

__global__ __launch_bounds__(256) void k_b_range(const BItemC* __restrict__ items, const unsigned* __restrict__ base,
                                                 int n)
{
    const int i = item_of(base, n, blockIdx.x);
    const BItemC* it = items + i;
    const unsigned b = blockIdx.x - base[i];
    if (it->cls >= 2) {
        if (it->vec) range_block<double, true>(b, it->nparts, (const double*)it->x, it->nv, it->partial, it->small, it->nsmall);
        else range_block<double, false>(b, it->nparts, (const double*)it->x, it->nv, it->partial, it->small, it->nsmall);
    } else {
        if (it->vec) range_block<float, true>(b, it->nparts, (const float*)it->x, it->nv, it->partial, it->small, it->nsmall);
        else range_block<float, false>(b, it->nparts, (const float*)it->x, it->nv, it->partial, it->small, it->nsmall);
    }
}

__global__ __launch_bounds__(256) void k_b_range_final(const BItemC* __restrict__ items)
{
    const BItemC* it = items + blockIdx.x;
    range_final_block(it->partial, (int)it->nparts, it->cur, it->bp, it->bnd);
}

template <typename T, int D>
__device__ __forceinline__ void b_resample(const BItemC* it, unsigned t)
{
    const int dtype = sizeof(T) == 8 ? MC_F64 : MC_F32;
    if (it->knobs & MC_KNOB_NT_MAP)
        resample_block<T, D, true>(t, it->vid, it->w, it->ng, (const T*)it->x, it->bnd, it->p, nullptr, nullptr,
                                   it->bflags, it->nbflags, it->small + 2, it->res, dtype, it->gcount, it->ntg);
    else
        resample_block<T, D, false>(t, it->vid, it->w, it->ng, (const T*)it->x, it->bnd, it->p, nullptr, nullptr,
                                    it->bflags, it->nbflags, it->small + 2, it->res, dtype, it->gcount, it->ntg);
}

__global__ __launch_bounds__(256) void k_b_resample(const BItemC* __restrict__ items,
                                                    const unsigned* __restrict__ base, int n)
{
    const int i = item_of(base, n, blockIdx.x);
    const BItemC* it = items + i;
    const unsigned t = blockIdx.x - base[i];
    switch (it->cls) {
    case 0: b_resample<float, 2>(it, t); break;
    case 1: b_resample<float, 3>(it, t); break;
    case 2: b_resample<double, 2>(it, t); break;
    default: b_resample<double, 3>(it, t); break;
    }
}

template <typename T, int D>
__device__ __forceinline__ void b_codes(const BItemC* it, unsigned b)
{
    const long long ngg = (it->ntg + MC_SC_TILES - 1) / MC_SC_TILES;
    unsigned* gsum = it->small + 16;
    unsigned* vsum = gsum + ngg;
    if (b < it->nbl) {
        if (D == 3) lorenzo3_block(b, it->p, it->n0, it->n1, it->n2, it->nxs, it->nyb, it->nunits, it->gcodes, it->gcount, gsum);
        else lorenzo_block<2>(b, it->p, it->n0, it->n1, it->n2, it->nxs, it->nunits, it->gcodes, it->gcount, gsum);
    } else if (it->knobs & MC_KNOB_NT_VERT) {
        residual_block<T, D, true, true>(b - it->nbl, it->coords, it->nv, it->gg, it->p, (const T*)it->x, it->bnd,
                                         it->vcodes, nullptr, it->vcount, vsum);
    } else {
        residual_block<T, D, true, false>(b - it->nbl, it->coords, it->nv, it->gg, it->p, (const T*)it->x, it->bnd,
                                          it->vcodes, nullptr, it->vcount, vsum);
    }
}

// At most 80 VGPRs (6 waves per SIMD, from 91 and 5), as k_codes: the
// 64-field batch 4.795 -> 4.763 ms per step.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_b_codes(const BItemC* __restrict__ items, const unsigned* __restrict__ base,
                                                 int n)
{
    const int i = item_of(base, n, blockIdx.x);
    const BItemC* it = items + i;
    const unsigned b = blockIdx.x - base[i];
    switch (it->cls) {
    case 0: b_codes<float, 2>(it, b); break;
    case 1: b_codes<float, 3>(it, b); break;
    case 2: b_codes<double, 2>(it, b); break;
    default: b_codes<double, 3>(it, b); break;
    }
}

template <typename T, int D>
__device__ __forceinline__ void b_scatter(const BItemC* it, unsigned b)
{
    const long long ngg = (it->ntg + MC_SC_TILES - 1) / MC_SC_TILES;
    unsigned* gsum = it->small + 16;
    scatter_block<T, D>(b, it->p, it->n0, it->n1, it->ng, MC_GRIDPRED_LORENZO, nullptr, it->gcodes, it->gcount, gsum,
                        it->gidx, it->gdelta, it->gcap, it->ntg, (const T*)it->x, it->nv, it->vcodes, it->vcount,
                        gsum + ngg, it->vidx, (T*)it->vval, it->vcap, it->small + 2, it->res);
}

__global__ __launch_bounds__(256) void k_b_scatter(const BItemC* __restrict__ items, const unsigned* __restrict__ base,
                                                   int n)
{
    const int i = item_of(base, n, blockIdx.x);
    const BItemC* it = items + i;
    const unsigned b = blockIdx.x - base[i];
    switch (it->cls) {
    case 0: b_scatter<float, 2>(it, b); break;
    case 1: b_scatter<float, 3>(it, b); break;
    case 2: b_scatter<double, 2>(it, b); break;
    default: b_scatter<double, 3>(it, b); break;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace mck {

hipError_t range(const void* x, int dtype, long long n, unsigned long long* partial, RangeOut* cur, BoundParams bp,
                 DevBound* bnd, unsigned int* zero, long long nzero, unsigned knobs, hipStream_t s)
{
    const int nblocks = knob_range_blocks(knobs);   // 2048: one batch of 8 quads per thread at 16M values
    {
        ProfScope ps("k_range", s);
        const bool V = ((uintptr_t)x & 15u) == 0;
#define MC_RG(T) do { if (V) hipLaunchKernelGGL((k_range<T, true>), dim3(nblocks), dim3(256), 0, s, (const T*)x, n, \
                                                partial, zero, nzero); \
                      else hipLaunchKernelGGL((k_range<T, false>), dim3(nblocks), dim3(256), 0, s, (const T*)x, n, \
                                              partial, zero, nzero); } while (0)
        if (dtype == MC_F64) MC_RG(double);
        else MC_RG(float);
#undef MC_RG
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ProfScope ps("k_range_final", s);
    hipLaunchKernelGGL(k_range_final, dim3(1), dim3(256), 0, s, partial, nblocks, cur, bp, bnd);
    return hipGetLastError();
}

hipError_t resample(const int32_t* vid, const float* w, int dim, long long ng, const void* x, int dtype,
                    const DevBound* bnd, int32_t* p, float* xh, float* dbg_v, uint32_t* bflags,
                    long long nbflags, unsigned int* err, mc_result* res, unsigned int* gcount, long long ntg,
                    unsigned remap, hipStream_t s)
{
    ProfScope ps("k_resample", s);
    const long long need = ng > nbflags ? ng : nbflags;
    dim3 grid((unsigned)((need + 255) / 256));
    const bool nt = (remap & MC_KNOB_NT_MAP) != 0;
    remap &= MC_KNOB_RESAMPLE;
#define MC_RS0(T, D, NT) hipLaunchKernelGGL((k_resample<T, D, NT>), grid, dim3(256), 0, s, vid, w, ng, (const T*)x, \
                                            bnd, p, xh, dbg_v, bflags, nbflags, err, res, dtype, gcount, ntg, remap)
#define MC_RS(T, D) do { if (nt) MC_RS0(T, D, true); else MC_RS0(T, D, false); } while (0)
    if (dtype == MC_F64) { if (dim == 2) MC_RS(double, 2); else MC_RS(double, 3); }
    else { if (dim == 2) MC_RS(float, 2); else MC_RS(float, 3); }
#undef MC_RS
#undef MC_RS0
    return hipGetLastError();
}

hipError_t lorenzo(const int32_t* p, int dim, int n0, int n1, int n2, long long ng, uint16_t* codes,
                   unsigned int* count, unsigned int* gsum, unsigned remap, hipStream_t s)
{
    remap &= MC_KNOB_LORENZO;
    ProfScope ps("k_lorenzo", s);
    (void)ng;
    const int nxs = (n0 + MC_LZ_W - 1) / MC_LZ_W;
    if (dim == 3) {
        const int nyb = (n1 + MC_LZ_RY - 1) / MC_LZ_RY;
        const unsigned nunits = (unsigned)((long long)nxs * nyb * ((n2 + MC_LZ3_CH - 1) / MC_LZ3_CH));
        hipLaunchKernelGGL(k_lorenzo3, dim3((nunits + 3) / 4), dim3(256), 0, s, p, n0, n1, n2, nxs, nyb, nunits, codes,
                           count, gsum, remap);
        return hipGetLastError();
    }
    const unsigned nunits = (unsigned)((long long)nxs * ((n1 + MC_LZ_CHUNK - 1) / MC_LZ_CHUNK));
    hipLaunchKernelGGL(k_lorenzo<2>, dim3((nunits + 3) / 4), dim3(256), 0, s, p, n0, n1, n2, nxs, nunits, codes,
                       count, gsum, remap);
    return hipGetLastError();
}

hipError_t codes(const int32_t* p, int dim, int n0, int n1, int n2, uint16_t* gcodes, unsigned int* gcount,
                 unsigned int* gsum, const float* coords, long long nv, GridGeom gg, const float* xh,
                 const int32_t* pq, const void* x, int dtype, const DevBound* bnd, uint16_t* vcodes, float* dbg_g,
                 unsigned int* vcount, unsigned int* vsum, unsigned remap, hipStream_t s)
{
    const bool nt = (remap & MC_KNOB_NT_VERT) != 0;
    const unsigned rl = remap & MC_KNOB_LORENZO, rr = remap & MC_KNOB_RESIDUAL;
    ProfScope ps("k_codes", s);
    const int nxs = (n0 + MC_LZ_W - 1) / MC_LZ_W;
    int nyb = 0;
    unsigned nunits;
    if (dim == 3) {
        nyb = (n1 + MC_LZ_RY - 1) / MC_LZ_RY;
        nunits = (unsigned)((long long)nxs * nyb * ((n2 + MC_LZ3_CH - 1) / MC_LZ3_CH));
    } else {
        nunits = (unsigned)((long long)nxs * ((n1 + MC_LZ_CHUNK - 1) / MC_LZ_CHUNK));
    }
    const unsigned nbl = ((nunits + 3) / 4 + 7) / 8 * 8;
    const unsigned nbr = (unsigned)((nv + MC_TILE - 1) / MC_TILE);
    const dim3 grid(nbl + nbr);
#define MC_CD(T, D, FP, NT) hipLaunchKernelGGL((k_codes<T, D, FP, NT>), grid, dim3(256), 0, s, p, n0, n1, n2, nxs, nyb, \
                                               nunits, gcodes, gcount, gsum, nbl, coords, nv, gg, \
                                               FP ? (const void*)pq : (const void*)xh, (const T*)x, bnd, vcodes, dbg_g, \
                                               vcount, vsum, rl, rr)
#define MC_CDD(T, D) do { if (pq) { if (nt) MC_CD(T, D, true, true); else MC_CD(T, D, true, false); } \
                          else { if (nt) MC_CD(T, D, false, true); else MC_CD(T, D, false, false); } } while (0)
    if (dtype == MC_F64) { if (dim == 2) MC_CDD(double, 2); else MC_CDD(double, 3); }
    else { if (dim == 2) MC_CDD(float, 2); else MC_CDD(float, 3); }
#undef MC_CDD
#undef MC_CD
    return hipGetLastError();
}

hipError_t residual(const float* coords, long long nv, GridGeom gg, const float* xh, const int32_t* pq,
                    const void* x, int dtype, const DevBound* bnd, uint16_t* codes, float* dbg_g,
                    unsigned int* count, unsigned int* vsum, unsigned remap, hipStream_t s)
{
    const bool nt = (remap & MC_KNOB_NT_VERT) != 0;
    remap &= MC_KNOB_RESIDUAL;
    const long long ntv = (nv + MC_TILE - 1) / MC_TILE;
    ProfScope ps("k_residual", s);
    const dim3 grid((unsigned)ntv);
#define MC_RQ(T, D, FP, NT) hipLaunchKernelGGL((k_residual<T, D, FP, NT>), grid, dim3(256), 0, s, coords, nv, gg, \
                                               FP ? (const void*)pq : (const void*)xh, (const T*)x, bnd, codes, \
                                               dbg_g, count, vsum, remap)
#define MC_RQD(T, D) do { if (pq) { if (nt) MC_RQ(T, D, true, true); else MC_RQ(T, D, true, false); } \
                          else { if (nt) MC_RQ(T, D, false, true); else MC_RQ(T, D, false, false); } } while (0)
    if (dtype == MC_F64) { if (gg.dim == 2) MC_RQD(double, 2); else MC_RQD(double, 3); }
    else { if (gg.dim == 2) MC_RQD(float, 2); else MC_RQD(float, 3); }
#undef MC_RQD
#undef MC_RQ
    return hipGetLastError();
}

void lorenzo_units(int dim, int n0, int n1, int n2, int* nxs, int* nyb, unsigned* nunits)
{
    *nxs = (n0 + MC_LZ_W - 1) / MC_LZ_W;
    if (dim == 3) {
        *nyb = (n1 + MC_LZ_RY - 1) / MC_LZ_RY;
        *nunits = (unsigned)((long long)*nxs * *nyb * ((n2 + MC_LZ3_CH - 1) / MC_LZ3_CH));
    } else {
        *nyb = 0;
        *nunits = (unsigned)((long long)*nxs * ((n1 + MC_LZ_CHUNK - 1) / MC_LZ_CHUNK));
    }
}

hipError_t batch_range(const BItemC* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s)
{
    ProfScope ps("k_b_range", s);
    hipLaunchKernelGGL(k_b_range, dim3(nblocks), dim3(256), 0, s, items, base, n);
    return hipGetLastError();
}

hipError_t batch_range_final(const BItemC* items, int n, hipStream_t s)
{
    ProfScope ps("k_b_range_final", s);
    hipLaunchKernelGGL(k_b_range_final, dim3((unsigned)n), dim3(256), 0, s, items);
    return hipGetLastError();
}

hipError_t batch_resample(const BItemC* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s)
{
    ProfScope ps("k_b_resample", s);
    hipLaunchKernelGGL(k_b_resample, dim3(nblocks), dim3(256), 0, s, items, base, n);
    return hipGetLastError();
}

hipError_t batch_codes(const BItemC* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s)
{
    ProfScope ps("k_b_codes", s);
    hipLaunchKernelGGL(k_b_codes, dim3(nblocks), dim3(256), 0, s, items, base, n);
    return hipGetLastError();
}

hipError_t batch_scatter(const BItemC* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s)
{
    ProfScope ps("k_b_scatter", s);
    hipLaunchKernelGGL(k_b_scatter, dim3(nblocks), dim3(256), 0, s, items, base, n);
    return hipGetLastError();
}

hipError_t xhat_from_p(const int32_t* p, long long ng, const DevBound* bnd, float* xh, hipStream_t s)
{
    ProfScope ps("k_xhat_from_p", s);
    hipLaunchKernelGGL(k_xhat_from_p, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, p, ng, bnd, xh);
    return hipGetLastError();
}

hipError_t compact(const int32_t* p, int dim, int n0, int n1, long long ng, int gpred, const float* gref,
                   const uint16_t* gcodes,
                   unsigned int* gcount, unsigned int* gsum, int32_t* gidx, int32_t* gdelta, long long gcap,
                   const void* x, int dtype,
                   long long nv, const uint16_t* vcodes, unsigned int* vcount, unsigned int* vsum, int32_t* vidx,
                   void* vval, long long vcap, unsigned int* err, mc_result* res, hipStream_t s)
{
    const long long ntg = (ng + MC_TILE - 1) / MC_TILE, ntv = (nv + MC_TILE - 1) / MC_TILE;
    ProfScope ps("k_scatter", s);
    dim3 grid((unsigned)((ntg + MC_SC_TILES - 1) / MC_SC_TILES + (ntv + MC_SC_TILES - 1) / MC_SC_TILES));
#define MC_SC(T, D) hipLaunchKernelGGL((k_scatter<T, D>), grid, dim3(256), 0, s, p, n0, n1, ng, gpred, gref, gcodes, gcount, \
                                       gsum, gidx, gdelta, gcap, ntg, (const T*)x, nv, vcodes, vcount, vsum, vidx, \
                                       (T*)vval, vcap, err, res)
    if (dtype == MC_F64) { if (dim == 2) MC_SC(double, 2); else MC_SC(double, 3); }
    else { if (dim == 2) MC_SC(float, 2); else MC_SC(float, 3); }
#undef MC_SC
    return hipGetLastError();
}

}  // namespace mck
