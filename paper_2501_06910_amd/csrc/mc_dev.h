// mc_dev.h -- device helpers shared by the gfx950 kernels: grid geometry,
// error-bound split, ordered block compaction (wave ballots + a workgroup
// scan) and decoupled look-back over tiles taken in ticket order.
//
// Every bit-exact formula is written as parenthesised and compiled with
// -ffp-contract=off (and the pragma below), so each + - * / is one IEEE
// round-to-nearest-even operation; rint() rounds half to even.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mc.h"

#define MC_R 32768
#define MC_TILE 1024          // items per workgroup tile (256 threads x 4)
#define MC_LZ_CHUNK 16        // rows per 2-D Lorenzo sweep
#define MC_SC_TILES 16        // outlier scatter: tiles per workgroup
#define MC_RANGE_BLOCKS 2048  // field range: per-block partials (3 words each)
#define MC_DZ_PLANES 8        // 3-D decode: planes per z chunk
#define MC_DY_ROWS 8          // 3-D decode: rows per xy chunk (4 waves x 2 rows)
#define MC_WG 256
#define MC_IPT 4              // items per thread in a tile
#define MC_LBLOCK 4096        // vertices per learned/plain decision block

// error bits accumulated in the workspace while a compress call runs
#define MC_EBIT_NONFINITE 1u
#define MC_EBIT_RANGE 2u
#define MC_EBIT_GCAP 4u
#define MC_EBIT_VCAP 8u
#define MC_EBIT_TAU 16u

struct GridGeom {
    int dim;
    int n0, n1, n2;           // n2 = 1 in 2-D
    float of[3], hf[3], ihf[3];   // (float)origin, (float)spacing, (float)(1/spacing)
};

// Field range in ordered-integer keys (min/max are exact and order-free).
struct RangeOut {
    unsigned long long kmin, kmax;
    unsigned int flags;
    unsigned int pad;
};

struct BoundParams {
    double eb;
    double split;
    int relative;
    int mode;                    // MC_SPLIT_SUM: tau2 = tau - tau1; MC_SPLIT_FULL: tau2 = tau
};

// The error split of one call, computed once per call by k_range_final and
// read by the kernels that quantise.
struct DevBound {
    double tau, tau1, tau2, c, xmin, xmax, inv1, step1, inv2, step2;
    int ok;
    unsigned flags;              // range flags (MC_EBIT_NONFINITE)
};

__device__ __forceinline__ unsigned long long dkey(double d)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(d);
    if (d == 0.0) b = 0ull;                       // -0 and +0 are one key
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double dkey_inv(unsigned long long k)
{
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// tau = eb * (xmax - xmin) or eb; tau1 = split * tau; tau2 = tau - tau1;
// c = 0.5 * (xmin + xmax); step_k = 2 tau_k, inv_k = 1 / (2 tau_k).
__device__ __forceinline__ DevBound make_bound(const RangeOut* r, BoundParams bp)
{
    DevBound b;
    double mn = dkey_inv(r->kmin), mx = dkey_inv(r->kmax);
    b.xmin = mn;
    b.xmax = mx;
    b.tau = bp.relative ? bp.eb * (mx - mn) : bp.eb;
    b.tau1 = bp.split * b.tau;
    b.tau2 = bp.mode == MC_SPLIT_FULL ? b.tau : b.tau - b.tau1;
    b.c = 0.5 * (mn + mx);
    b.step1 = 2.0 * b.tau1;
    b.inv1 = 1.0 / (2.0 * b.tau1);
    b.step2 = 2.0 * b.tau2;
    b.inv2 = 1.0 / (2.0 * b.tau2);
    b.ok = !(r->flags & MC_EBIT_NONFINITE) && (b.tau1 > 0.0) && (b.tau2 > 0.0);
    b.flags = (unsigned)r->flags;
    return b;
}

template <typename T> __device__ __forceinline__ double as_double(T v) { return (double)v; }
template <typename T> __device__ __forceinline__ float as_float(T v) { return (float)v; }

// Reconstructed grid value x1' = (float)(c + (double)p * step1).
__device__ __forceinline__ float xhat_of(int32_t p, double c, double step1)
{
    return (float)(c + (double)p * step1);
}

// Position of grid node j in the ascending outlier list, or -1.
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

// Bits of the zigzag code of k (the cost of a code in the learned block
// choice).
__device__ __forceinline__ int zz_bits(int k)
{
    const unsigned z = ((unsigned)k << 1) ^ (unsigned)(k >> 31);
    return 32 - __clz(z);
}

// Residual quantisation of one vertex: r = x - g, q = rint(r / (2 tau2)),
// x' = (T)(g + q * 2 tau2); accepted iff |q| <= R-1 and |x - x'| <= tau2.
template <typename T>
__device__ __forceinline__ bool quantize_residual(T xv, float g, const DevBound& b, int& qi)
{
    const double r = (double)xv - (double)g;
    const double q = rint(r * b.inv2);
    const T xr = (T)((double)g + q * b.step2);
    const bool ok = fabs(q) <= (double)(MC_R - 1) && fabs((double)xv - (double)xr) <= b.tau2;
    qi = ok ? (int)q : 0;
    return ok;
}

// Prediction error of grid node j: its code, or its outlier entry.
__device__ __forceinline__ int delta_at(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                        const int32_t* __restrict__ odelta, long long nout, long long j)
{
    const int c = codes[j];
    if (c != 0) return c - MC_R;
    const long long k = find_outlier(oidx, nout, j);
    return k >= 0 ? odelta[k] : 0;
}

__device__ __forceinline__ float lerpf_(float a, float b, float t)
{
    return (1.0f - t) * a + t * b;
}

// Grid cell and in-cell offset of a vertex coordinate along one axis:
// u = (P - of) * ihf, i = clamp(floor(u), 0, n-2), t = clamp(u - i, 0, 1).
__device__ __forceinline__ void axis_cell(float P, float of, float ihf, int n, int& i, float& t)
{
    const float u = (P - of) * ihf;
    const float fl = floorf(u);
    const int ic = (int)fl;
    i = fl < 0.0f ? 0 : (fl > (float)(n - 2) ? n - 2 : ic);
    const float tt = u - (float)i;
    t = tt < 0.0f ? 0.0f : (tt > 1.0f ? 1.0f : tt);
}

// XCD-aware tile order.  Workgroups are handed to the 8 XCDs round-robin
// (block b runs on XCD b % 8); renumbering them so that XCD x processes a
// contiguous range of tiles keeps neighbouring tiles -- and the grid planes,
// rows and field values they share -- in one XCD's L2.  A bijection on
// [0, n).
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned n)
{
    const unsigned per = n >> 3, rem = n & 7u, x = b & 7u, r = b >> 3;
    return (x < rem ? x * (per + 1u) : rem * (per + 1u) + (x - rem) * per) + r;
}

// Loads and stores of data streamed once through a kernel.  NT: the
// non-temporal (streaming) cache policy, so that the stream does not evict
// lines other threads will read again (cell corners, gathered field values).
template <bool NT, typename T>
__device__ __forceinline__ T ld_s(const T* __restrict__ p)
{
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_s(T* __restrict__ p, T v)
{
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Two consecutive floats at a 4-byte aligned address.
typedef float f2a4 __attribute__((ext_vector_type(2), aligned(4)));

// ---------------------------------------------------------------------------
// g(x1') for N vertices of one thread from their coordinates P: cells, then
// every corner of every cell, then the nested lerps (x, then y, then z) in
// the order of the definition, so that all gathers issue together.
// FROM_P: src is the prequantised grid (int32) and each corner is converted
// to x1' = (float)(c + p * step1) exactly as the grid decoder produces it;
// otherwise src is x1' itself (float).
typedef int i2a4 __attribute__((ext_vector_type(2), aligned(4)));

template <bool FROM_P>
__device__ __forceinline__ void corner_pair(const void* __restrict__ src, unsigned j, double c, double step1,
                                            float& a, float& b)
{
    if (FROM_P) {
        const i2a4 q = *reinterpret_cast<const i2a4*>((const int32_t*)src + j);
        a = xhat_of(q.x, c, step1);
        b = xhat_of(q.y, c, step1);
    } else {
        const f2a4 e = *reinterpret_cast<const f2a4*>((const float*)src + j);
        a = e.x;
        b = e.y;
    }
}

template <int D, int N, bool FROM_P>
__device__ __forceinline__ void back_interp_p(const float (&P)[N][3], const GridGeom& gg,
                                              const void* __restrict__ src, double cc, double step1, float (&g)[N])
{
    const unsigned n0 = (unsigned)gg.n0, n01 = (unsigned)gg.n0 * (unsigned)gg.n1;
    unsigned j[N];
    float t[N][3];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        int i0, i1, i2 = 0;
        axis_cell(P[i][0], gg.of[0], gg.ihf[0], gg.n0, i0, t[i][0]);
        axis_cell(P[i][1], gg.of[1], gg.ihf[1], gg.n1, i1, t[i][1]);
        if (D == 3) axis_cell(P[i][2], gg.of[2], gg.ihf[2], gg.n2, i2, t[i][2]);
        j[i] = (unsigned)i0 + n0 * (unsigned)i1 + n01 * (unsigned)i2;
    }
    // the two corners of a cell edge along x are adjacent: one 8-byte load
    // each (4-byte aligned, which global loads of two dwords accept), half
    // the gather instructions of single-value loads
    float c[N][8];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        corner_pair<FROM_P>(src, j[i], cc, step1, c[i][0], c[i][1]);
        corner_pair<FROM_P>(src, j[i] + n0, cc, step1, c[i][2], c[i][3]);
        if (D == 3) {
            corner_pair<FROM_P>(src, j[i] + n01, cc, step1, c[i][4], c[i][5]);
            corner_pair<FROM_P>(src, j[i] + n01 + n0, cc, step1, c[i][6], c[i][7]);
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const float c00 = lerpf_(c[i][0], c[i][1], t[i][0]);
        const float c10 = lerpf_(c[i][2], c[i][3], t[i][0]);
        const float c0 = lerpf_(c00, c10, t[i][1]);
        if (D == 2) {
            g[i] = c0;
        } else {
            const float c01 = lerpf_(c[i][4], c[i][5], t[i][0]);
            const float c11 = lerpf_(c[i][6], c[i][7], t[i][0]);
            g[i] = lerpf_(c0, lerpf_(c01, c11, t[i][1]), t[i][2]);
        }
    }
}

template <int D, int N>
__device__ __forceinline__ void back_interp_p(const float (&P)[N][3], const GridGeom& gg,
                                              const float* __restrict__ xh, float (&g)[N])
{
    back_interp_p<D, N, false>(P, gg, xh, 0.0, 0.0, g);
}

// The same for N vertices v[i] (strided ownership): coordinates loaded
// first.  act[i] false: vertex 0 stands in (its result is ignored), so no
// load depends on a branch.
template <int D, int N, bool FROM_P, bool NT = false>
__device__ __forceinline__ void back_interp_n(const float* __restrict__ coords, long long nv, const GridGeom& gg,
                                              const void* __restrict__ src, double cc, double step1,
                                              const long long (&v)[N], const bool (&act)[N], float (&g)[N])
{
    float P[N][3];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const long long vc = act[i] ? v[i] : 0;
#pragma unroll
        for (int d = 0; d < D; ++d) P[i][d] = ld_s<NT>(coords + d * nv + vc);
        if (D == 2) P[i][2] = 0.0f;
    }
    back_interp_p<D, N, FROM_P>(P, gg, src, cc, step1, g);
}

template <int D, int N>
__device__ __forceinline__ void back_interp_n(const float* __restrict__ coords, long long nv, const GridGeom& gg,
                                              const float* __restrict__ xh, const long long (&v)[N],
                                              const bool (&act)[N], float (&g)[N])
{
    back_interp_n<D, N, false>(coords, nv, gg, xh, 0.0, 0.0, v, act, g);
}

// Four consecutive values of T from a 16-byte aligned address.
template <typename T> struct Quad { T v[4]; };
__device__ __forceinline__ Quad<float> load_quad(const float* __restrict__ p)
{
    const float4 a = *reinterpret_cast<const float4*>(p);
    return Quad<float>{{a.x, a.y, a.z, a.w}};
}
__device__ __forceinline__ Quad<double> load_quad(const double* __restrict__ p)
{
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    return Quad<double>{{a.x, a.y, b.x, b.y}};
}
// Field of block b in a batched stage launch: the i with
// base[i] <= b < base[i + 1] (base ascending, n fields).
__device__ __forceinline__ int item_of(const unsigned* __restrict__ base, int n, unsigned b)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Tile of this workgroup: XCD-contiguous order when `remap` is set.
__device__ __forceinline__ unsigned tile_of(unsigned remap)
{
    return remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
}

// ---------------------------------------------------------------------------
// wave / workgroup primitives (wave64)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int mbcnt64(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

template <typename T> __device__ __forceinline__ T wave_incl_scan(T v)
{
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(v, d, 64);
        if (l >= d) v += o;
    }
    return v;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Ordered compaction of a tile: item (i, t) of thread t is at tile offset
// i*256 + t.  Returns each flagged item's exclusive rank in index order and
// the tile total.  s_cnt needs MC_IPT*4 + 1 ints of LDS.
__device__ __forceinline__ int tile_ranks(const bool (&flag)[MC_IPT], int (&rank)[MC_IPT], int* s_cnt)
{
    const int l = lane_id(), w = threadIdx.x >> 6;
    unsigned long long ball[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        ball[i] = __ballot(flag[i]);
        if (l == 0) s_cnt[i * 4 + w] = __popcll(ball[i]);
    }
    __syncthreads();
    if (w == 0) {
        const int v = l < MC_IPT * 4 ? s_cnt[l] : 0;
        const int inc = wave_incl_scan(v);
        if (l < MC_IPT * 4) s_cnt[l] = inc - v;
        if (l == 63) s_cnt[MC_IPT * 4] = inc;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) rank[i] = s_cnt[i * 4 + w] + mbcnt64(ball[i]);
    return s_cnt[MC_IPT * 4];
}

// Block-wide sum of a uint64 (256 threads); s needs 4 slots.
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* s)
{
    v = wave_sum(v);
    if (lane_id() == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    const unsigned long long t = s[0] + s[1] + s[2] + s[3];
    __syncthreads();
    return t;
}

// Block-wide sum of an int64 (256 threads); s needs 4 slots.
__device__ __forceinline__ long long block_sum_i64(long long v, long long* s)
{
    v = wave_sum(v);
    if (lane_id() == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = s[0] + s[1] + s[2] + s[3];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// decoupled look-back over tiles (scalar payload in the status word)
// status word: bits 62..63 flag (1 = tile aggregate, 2 = inclusive prefix),
// bits 0..61 value.  Tiles are numbered by an atomic ticket, so a tile only
// waits on tiles that started earlier: every wait ends.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void lb_store(unsigned long long* st, long long tile, unsigned long long flag,
                                         unsigned long long val)
{
    __hip_atomic_store(&st[tile], (flag << 62) | val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long lb_exclusive(unsigned long long* st, long long tile)
{
    unsigned long long excl = 0;
    long long k = tile - 1;
    while (k >= 0) {
        unsigned long long s = __hip_atomic_load(&st[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long f = s >> 62;
        if (f == 0) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += s & 0x3fffffffffffffffull;
        if (f == 2) break;
        --k;
    }
    return excl;
}

// Takes the next tile ticket; every thread of the block gets it.
__device__ __forceinline__ long long take_ticket(unsigned int* counter, long long* s_slot)
{
    if (threadIdx.x == 0) *s_slot = (long long)atomicAdd(counter, 1u);
    __syncthreads();
    long long t = *s_slot;
    __syncthreads();
    return t;
}

// Publishes this tile's value (a count, or several counts packed in one
// word) and returns the exclusive prefix over all earlier tiles (thread 0
// does the look-back; the result is broadcast through LDS).
__device__ __forceinline__ unsigned long long tile_prefix(unsigned long long* st, long long tile,
                                                          unsigned long long val, long long* s_slot)
{
    if (threadIdx.x == 0) {
        unsigned long long excl = 0;
        if (tile == 0) {
            lb_store(st, 0, 2ull, val);
        } else {
            lb_store(st, tile, 1ull, val);
            excl = lb_exclusive(st, tile);
            lb_store(st, tile, 2ull, excl + val);
        }
        *s_slot = (long long)excl;
    }
    __syncthreads();
    unsigned long long e = (unsigned long long)*s_slot;
    __syncthreads();
    return e;
}

// Final status of a compress call from the accumulated error bits.
__device__ __forceinline__ int status_from_bits(unsigned int e)
{
    if (e & (MC_EBIT_NONFINITE | MC_EBIT_TAU)) return 1;
    if (e & MC_EBIT_RANGE) return 2;
    if (e & (MC_EBIT_GCAP | MC_EBIT_VCAP)) return 3;
    return 0;
}

// ---------------------------------------------------------------------------
// epoch-tagged status words for look-back with one word per element: bits
// 62..63 flag (1 aggregate, 2 inclusive), bits 32..61 the call's epoch,
// bits 0..31 the value.  A word from an earlier call carries another epoch
// and reads as "not ready", so the arrays never need clearing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long ep_word(unsigned flag, unsigned epoch, int v)
{
    return ((unsigned long long)flag << 62) | ((unsigned long long)(epoch & 0x3fffffffu) << 32) |
           (unsigned long long)(unsigned)v;
}

__device__ __forceinline__ void ep_store(unsigned long long* a, unsigned long long w)
{
    __hip_atomic_store(a, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spins until the word carries this epoch; returns it.
__device__ __forceinline__ unsigned long long ep_wait(unsigned long long* a, unsigned epoch)
{
    unsigned long long w;
    for (;;) {
        w = __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((w >> 62) != 0 && (unsigned)((w >> 32) & 0x3fffffffu) == (epoch & 0x3fffffffu)) return w;
        __builtin_amdgcn_s_sleep(1);
    }
}

// Per-wave ticket from a monotonic 64-bit counter: tile = ticket - base.
__device__ __forceinline__ long long wave_ticket(unsigned long long* counter, unsigned long long base)
{
    unsigned long long t = 0;
    if (lane_id() == 0) t = atomicAdd(counter, 1ull);
    t = __shfl(t, 0, 64);
    return (long long)(t - base);
}
