// k_serial.hip -- the 1-D serialisation baseline on gfx950: the vertex array
// compressed as a plain 1-D signal by the same kind of predictor-quantiser
// (the "default" compression the multi-component scheme is compared with,
// paper Sec. V-C).  With the whole bound tau on the one component:
//   p_i = rint((x_i - c) / (2 tau)), d_i = p_i - p_{i-1} (p_{-1} = 0),
//   x'_i = (T)(c + p_i * 2 tau); code d_i + R if |d_i| <= R - 1 and
//   |x_i - x'_i| <= tau, else 0 with the raw value stored.
// The decoder's p is a running sum of the codes that restarts at every raw
// value from rint((raw - c) / (2 tau)): a segmented prefix sum, done as
// tile aggregates -> one-workgroup scan of the aggregates -> apply.
//   k_ser_codes   codes and per-tile raw counts (compaction: k_scatter)
//   k_ser_tot     per-tile aggregate (restart flag, value)
//   k_ser_carry   exclusive segmented scan of the tile aggregates
//   k_ser_apply   p and x' of every value
#include "mc_dev.h"
#include "mc_kernels.h"
#include "mc_seg.h"

// Thread t of a tile codes its 4 consecutive values; p_{i-1} of its first
// comes from the lane before (the wave's first lane loads it).  V: x is
// 16-byte and codes 8-byte aligned (vector loads and stores).
template <typename T, bool V>
__global__ __launch_bounds__(256) void k_ser_codes(const T* __restrict__ x, long long n,
                                                   const DevBound* __restrict__ bnd, uint16_t* __restrict__ codes,
                                                   unsigned int* __restrict__ count, unsigned int* __restrict__ vsum,
                                                   unsigned int* __restrict__ err, mc_result* __restrict__ res,
                                                   int dtype)
{
    __shared__ int s_cnt[4];
    const DevBound b = *bnd;
    const long long tile = blockIdx.x;
    if (tile == 0 && threadIdx.x == 0) {
        res->status = b.ok ? 0 : 1;
        res->dtype = dtype;
        res->tau = b.tau;
        res->tau1 = b.tau;
        res->tau2 = 0.0;
        res->c = b.c;
        res->xmin = b.xmin;
        res->xmax = b.xmax;
        if (!b.ok) atomicOr(err, (b.flags & MC_EBIT_NONFINITE) ? MC_EBIT_NONFINITE : MC_EBIT_TAU);
    }
    const double step = 2.0 * b.tau, inv = 1.0 / (2.0 * b.tau);
    const long long e0 = tile * MC_TILE + 4 * (long long)threadIdx.x;
    const long long wfirst = tile * MC_TILE + 4 * (long long)(threadIdx.x & ~63u);
    T xi[4];
    if (V && e0 + 3 < n) {
        if constexpr (sizeof(T) == 4) {
            const float4 q = *(const float4*)(x + e0);
            xi[0] = q.x; xi[1] = q.y; xi[2] = q.z; xi[3] = q.w;
        } else {
            const double2 q0 = *(const double2*)(x + e0), q1 = *(const double2*)(x + e0 + 2);
            xi[0] = q0.x; xi[1] = q0.y; xi[2] = q1.x; xi[3] = q1.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) xi[k] = x[e0 + k < n ? e0 + k : 0];
    }
    const T xw = x[wfirst > 0 && wfirst - 1 < n ? wfirst - 1 : 0];   // one address per wave
    int p[4];
    bool inr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double sc = ((double)xi[k] - b.c) * inv;
        inr[k] = fabs(sc) < 134217728.0;
        p[k] = inr[k] ? (int)rint(sc) : 0;
    }
    const double sw = ((double)xw - b.c) * inv;
    const int pw = wfirst > 0 && fabs(sw) < 134217728.0 ? (int)rint(sw) : 0;
    int pprev = __shfl_up(p[3], 1, 64);
    if (lane_id() == 0) pprev = pw;
    int nout = 0;
    bool range_bad = false;
    uint16_t cd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool valid = e0 + k < n && b.ok;
        const int d = p[k] - (k ? p[k - 1] : pprev);
        const T xr = (T)(b.c + (double)p[k] * step);
        const bool ok = inr[k] && d >= -(MC_R - 1) && d <= MC_R - 1 && fabs((double)xi[k] - (double)xr) <= b.tau;
        cd[k] = ok ? (uint16_t)(d + MC_R) : (uint16_t)0;
        range_bad |= valid && !inr[k];
        nout += valid && !ok ? 1 : 0;
    }
    if (b.ok) {
        if (V && e0 + 3 < n) {
            *(uint2*)(codes + e0) = make_uint2((unsigned)cd[0] | ((unsigned)cd[1] << 16),
                                               (unsigned)cd[2] | ((unsigned)cd[3] << 16));
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (e0 + k < n) codes[e0 + k] = cd[k];
        }
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

// Index of outlier i in the ascending list (nout entries), or -1.
__device__ __forceinline__ long long ser_find(const int32_t* __restrict__ oidx, long long nout, long long i)
{
    long long lo = 0, hi = nout;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if ((long long)oidx[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    return (lo < nout && (long long)oidx[lo] == i) ? lo : -1;
}

// Element of the running sum: the code's difference, or a restart at the
// raw value's p (a code-0 entry with no stored value restarts at 0).
template <typename T>
__device__ __forceinline__ Seg ser_elem(int code, const int32_t* __restrict__ oidx, const T* __restrict__ oval,
                                        long long nout, long long i, double c, double inv)
{
    if (code != 0) return Seg{0, code - MC_R};
    const long long k = ser_find(oidx, nout, i);
    const double raw = k >= 0 ? (double)oval[k] : 0.0;
    return Seg{1, (int)rint((raw - c) * inv)};
}

// The decoder's tiles: MC_SER_SUB sub-tiles of 1024 values; in each, thread
// t holds values 4t..4t+3 (8-byte code loads, 16-byte stores, coalesced).
// Running-sum order: sub-tile, then thread, then value.
#define MC_SER_SUB 4
#define MC_SER_DTILE (MC_SER_SUB * 1024)
#define MC_SER_CARRY_WG 1024

// The 4 consecutive codes from i (MC_R, a zero difference, past n; one
// aligned 8-byte load when all are in range).
__device__ __forceinline__ void ser_codes(const uint16_t* __restrict__ codes, long long n, long long i, int (&c)[4])
{
    if (i + 3 < n && (((uintptr_t)(codes + i)) & 7u) == 0) {
        const uint2 q = *(const uint2*)(codes + i);
        c[0] = (int)(q.x & 0xffffu); c[1] = (int)(q.x >> 16);
        c[2] = (int)(q.y & 0xffffu); c[3] = (int)(q.y >> 16);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = i + k < n ? (int)codes[i + k < n ? i + k : 0] : MC_R;
    }
}

// Codes of the thread's values in a tile and its fold per sub-tile.
template <typename T>
__device__ __forceinline__ void ser_tile_fold(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                              const T* __restrict__ oval, long long nout, long long n,
                                              long long tbase, double c, double inv, int (&cd)[MC_SER_SUB][4],
                                              Seg (&sj)[MC_SER_SUB])
{
#pragma unroll
    for (int j = 0; j < MC_SER_SUB; ++j) ser_codes(codes, n, tbase + j * 1024 + 4 * threadIdx.x, cd[j]);
#pragma unroll
    for (int j = 0; j < MC_SER_SUB; ++j) {
        const long long b = tbase + j * 1024 + 4 * threadIdx.x;
        Seg s{0, 0};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (cd[j][k] != 0) s.v += cd[j][k] - MC_R;
            else s = seg_op(s, ser_elem<T>(0, oidx, oval, nout, b + k, c, inv));
        }
        sj[j] = s;
    }
}

// Exclusive segmented scan over the tile (sub-tile, wave, lane order) from
// `init`: ex[j] is everything before the thread's run in sub-tile j;
// *total is init combined with the whole tile.  s_w: [MC_SER_SUB][4].
__device__ __forceinline__ void tile_seg_excl(const Seg (&sj)[MC_SER_SUB], Seg init, Seg (*s_w)[4],
                                              Seg (&ex)[MC_SER_SUB], Seg* total)
{
    const int l = lane_id(), w = threadIdx.x >> 6;
    Seg inc[MC_SER_SUB];
#pragma unroll
    for (int j = 0; j < MC_SER_SUB; ++j) inc[j] = wave_seg_incl(sj[j]);
    if (l == 63) {
#pragma unroll
        for (int j = 0; j < MC_SER_SUB; ++j) s_w[j][w] = inc[j];
    }
    __syncthreads();
    Seg run = init;
#pragma unroll
    for (int j = 0; j < MC_SER_SUB; ++j) {
        Seg pre = run;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const Seg a = s_w[j][k];
            if (k < w) pre = seg_op(pre, a);
            run = seg_op(run, a);
        }
        Seg e;
        e.f = __shfl_up(inc[j].f, 1, 64);
        e.v = __shfl_up(inc[j].v, 1, 64);
        if (l == 0) e = Seg{0, 0};
        ex[j] = seg_op(pre, e);
    }
    *total = run;
}

// Per-tile aggregate (restart seen, running value) of the codes.
template <typename T>
__global__ __launch_bounds__(256) void k_ser_tot(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                 const T* __restrict__ oval, const mc_result* __restrict__ res,
                                                 long long vcap, long long n, int2* __restrict__ agg)
{
    __shared__ Seg s_w[MC_SER_SUB][4];
    const double c = res->c, inv = 1.0 / (2.0 * res->tau);
    const long long nout = res->n_vertex_outliers < vcap ? res->n_vertex_outliers : vcap;
    int cd[MC_SER_SUB][4];
    Seg sj[MC_SER_SUB], ex[MC_SER_SUB], total;
    ser_tile_fold<T>(codes, oidx, oval, nout, n, (long long)blockIdx.x * MC_SER_DTILE, c, inv, cd, sj);
    tile_seg_excl(sj, Seg{0, 0}, s_w, ex, &total);
    if (threadIdx.x == 0) agg[blockIdx.x] = make_int2(total.f, total.v);
}

// One workgroup: carry[t] = p before tile t; the scan starts from a restart
// at 0 since p_{-1} = 0.  Thread k folds a run of consecutive tiles, 8
// loads in flight.
__global__ __launch_bounds__(MC_SER_CARRY_WG) void k_ser_carry(const int2* __restrict__ agg, long long ntiles,
                                                               int* __restrict__ carry)
{
    __shared__ Seg s_w[MC_SER_CARRY_WG / 64];
    const long long per = (ntiles + MC_SER_CARRY_WG - 1) / MC_SER_CARRY_WG;
    const long long t0 = per * threadIdx.x, t1 = t0 + per < ntiles ? t0 + per : ntiles;
    Seg s{0, 0};
    for (long long tb = t0; tb < t1; tb += 8) {
        int2 a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = agg[tb + u < t1 ? tb + u : t0];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (tb + u < t1) s = seg_op(s, Seg{a[u].x, a[u].y});
    }
    Seg total;
    Seg run = block_seg_excl<MC_SER_CARRY_WG / 64>(s, Seg{1, 0}, s_w, &total);
    for (long long tb = t0; tb < t1; tb += 8) {
        int2 a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = agg[tb + u < t1 ? tb + u : t0];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (tb + u < t1) {
                carry[tb + u] = run.v;
                run = seg_op(run, Seg{a[u].x, a[u].y});
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_ser_apply(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                   const T* __restrict__ oval, const mc_result* __restrict__ res,
                                                   long long vcap, long long n, const int* __restrict__ carry,
                                                   T* __restrict__ out)
{
    __shared__ Seg s_w[MC_SER_SUB][4];
    const double c = res->c, step = 2.0 * res->tau, inv = 1.0 / (2.0 * res->tau);
    const long long nout = res->n_vertex_outliers < vcap ? res->n_vertex_outliers : vcap;
    const long long tbase = (long long)blockIdx.x * MC_SER_DTILE;
    int cd[MC_SER_SUB][4];
    Seg sj[MC_SER_SUB], ex[MC_SER_SUB], total;
    ser_tile_fold<T>(codes, oidx, oval, nout, n, tbase, c, inv, cd, sj);
    tile_seg_excl(sj, Seg{1, carry[blockIdx.x]}, s_w, ex, &total);
#pragma unroll
    for (int j = 0; j < MC_SER_SUB; ++j) {
        const long long b = tbase + j * 1024 + 4 * threadIdx.x;
        int p = ex[j].v;                   // ex.f is set: the scan starts from a restart
        T v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (cd[j][k] != 0) {
                p += cd[j][k] - MC_R;
                v[k] = (T)(c + (double)p * step);
            } else {
                const long long o = ser_find(oidx, nout, b + k);
                const double raw = o >= 0 ? (double)oval[o] : 0.0;
                p = (int)rint((raw - c) * inv);
                v[k] = (T)raw;
            }
        }
        if (b + 3 < n && (((uintptr_t)(out + b)) & 15u) == 0) {
            if constexpr (sizeof(T) == 4) {
                *(float4*)(out + b) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                *(double2*)(out + b) = make_double2(v[0], v[1]);
                *(double2*)(out + b + 2) = make_double2(v[2], v[3]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (b + k < n) out[b + k] = v[k];
        }
    }
}

namespace mck {

hipError_t serial_codes(const void* x, int dtype, long long n, const DevBound* bnd, uint16_t* codes, unsigned* count,
                        unsigned* vsum, unsigned* err, mc_result* res, hipStream_t s)
{
    ProfScope ps("k_ser_codes", s);
    dim3 grid((unsigned)((n + MC_TILE - 1) / MC_TILE));
    const bool V = ((uintptr_t)x & 15u) == 0 && ((uintptr_t)codes & 7u) == 0;
#define MC_SCK(T, VV) hipLaunchKernelGGL((k_ser_codes<T, VV>), grid, dim3(256), 0, s, (const T*)x, n, bnd, codes, \
                                         count, vsum, err, res, dtype)
    if (dtype == MC_F64) { if (V) MC_SCK(double, true); else MC_SCK(double, false); }
    else { if (V) MC_SCK(float, true); else MC_SCK(float, false); }
#undef MC_SCK
    return hipGetLastError();
}

hipError_t seg_carry(const int2* agg, long long ntiles, int* carry, hipStream_t s)
{
    hipLaunchKernelGGL(k_ser_carry, dim3(1), dim3(MC_SER_CARRY_WG), 0, s, agg, ntiles, carry);
    return hipGetLastError();
}

hipError_t serial_decode(const uint16_t* codes, const int32_t* oidx, const void* oval, long long vcap,
                         const mc_result* res, long long n, int dtype, int2* agg, int* carry, void* out, hipStream_t s)
{
    hipError_t e;
    const long long ntiles = (n + MC_SER_DTILE - 1) / MC_SER_DTILE;
    dim3 grid((unsigned)ntiles);
    {
        ProfScope ps("k_ser_tot", s);
        if (dtype == MC_F64)
            hipLaunchKernelGGL(k_ser_tot<double>, grid, dim3(256), 0, s, codes, oidx, (const double*)oval, res, vcap, n,
                               agg);
        else
            hipLaunchKernelGGL(k_ser_tot<float>, grid, dim3(256), 0, s, codes, oidx, (const float*)oval, res, vcap, n,
                               agg);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        ProfScope ps("k_ser_carry", s);
        hipLaunchKernelGGL(k_ser_carry, dim3(1), dim3(MC_SER_CARRY_WG), 0, s, agg, ntiles, carry);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    ProfScope ps("k_ser_apply", s);
    if (dtype == MC_F64)
        hipLaunchKernelGGL(k_ser_apply<double>, grid, dim3(256), 0, s, codes, oidx, (const double*)oval, res, vcap, n,
                           carry, (double*)out);
    else
        hipLaunchKernelGGL(k_ser_apply<float>, grid, dim3(256), 0, s, codes, oidx, (const float*)oval, res, vcap, n,
                           carry, (float*)out);
    return hipGetLastError();
}

}  // namespace mck
