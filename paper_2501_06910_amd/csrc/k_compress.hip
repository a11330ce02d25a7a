// k_compress.hip -- the compression hot path on gfx950 (paper Alg. 3 with
// the residual taken against the reconstructed grid):
//   k_range(_final)  field min/max (ordered integer keys: per-block partials,
//                    then one workgroup) and non-finite check; clears the
//                    per-call state of the kernels after it
//   k_resample       f: v_j = sum_k w_kj * x[vid_kj] (FP32, fixed order), the
//                    prequantised grid p_j = rint((v_j - c) / (2 tau1)) and the
//                    reconstructed grid x1'_j = (float)(c + p_j * 2 tau1)
//   k_lorenzo        Lorenzo prediction error of p, uint16 codes, per-tile
//                    outlier counts
//   k_learned_cost   learned mode: both code costs per 4096-vertex block
//   k_residual       g: multilinear x1' at each vertex, residual quantisation
//                    with the per-vertex bound check, learned shift in the
//                    blocks where it is cheaper, per-tile outlier counts
//   k_scan_counts    exclusive scan of the per-tile counts
//   k_scatter        outlier lists in index order (wave ballots)
#include "mc_dev.h"
#include "mc_kernels.h"

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_range(const T* __restrict__ x, long long n,
                                               unsigned long long* __restrict__ partial,
                                               unsigned int* __restrict__ zero, long long nzero)
{
    __shared__ unsigned long long s_mn[4], s_mx[4];
    __shared__ unsigned int s_fl[4];
    const long long stride = (long long)gridDim.x * 256;
    const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
    for (long long i = gid; i < nzero; i += stride) zero[i] = 0u;
    double mn = __builtin_inf(), mx = -__builtin_inf();
    bool bad = false;
    constexpr int U = 8;
    long long i = gid;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = x[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double d = (double)v[u];
            bad |= !isfinite(d);
            mn = fmin(mn, d);
            mx = fmax(mx, d);
        }
    }
    for (; i < n; i += stride) {
        const double d = (double)x[i];
        bad |= !isfinite(d);
        mn = fmin(mn, d);
        mx = fmax(mx, d);
    }
    // keys of the per-thread extremes (-0 and +0 share a key; an empty
    // thread contributes the neutral keys)
    unsigned long long kmn = mn <= mx ? dkey(mn) : ~0ull;
    unsigned long long kmx = mn <= mx ? dkey(mx) : 0ull;
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
        partial[3 * blockIdx.x] = kmn;
        partial[3 * blockIdx.x + 1] = kmx;
        partial[3 * blockIdx.x + 2] = fl;
    }
}

// One workgroup folds the per-block partials into the range slot.
__global__ __launch_bounds__(256) void k_range_final(const unsigned long long* __restrict__ partial, int nparts,
                                                     RangeOut* __restrict__ out)
{
    __shared__ unsigned long long s_mn[4], s_mx[4];
    __shared__ unsigned int s_fl[4];
    unsigned long long kmn = ~0ull, kmx = 0ull;
    unsigned int fl = 0;
    for (int i = threadIdx.x; i < nparts; i += 256) {
        const unsigned long long a = partial[3 * i], b = partial[3 * i + 1];
        kmn = a < kmn ? a : kmn;
        kmx = b > kmx ? b : kmx;
        fl |= (unsigned)partial[3 * i + 2];
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
        out->kmin = kmn;
        out->kmax = kmx;
        out->flags = fl;
    }
}

// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(256) void k_resample(const int32_t* __restrict__ vid, const float* __restrict__ w,
                                                  long long ng, const T* __restrict__ x,
                                                  const RangeOut* __restrict__ range, BoundParams bp,
                                                  int32_t* __restrict__ p, float* __restrict__ xh,
                                                  float* __restrict__ dbg_v, uint32_t* __restrict__ bflags,
                                                  long long nbflags, unsigned int* __restrict__ err,
                                                  mc_result* __restrict__ res, int dtype,
                                                  unsigned int* __restrict__ gcount, long long ntg)
{
    const DevBound b = make_bound(range, bp);
    const long long j = (long long)xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
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
        if (!b.ok) atomicOr(err, (range->flags & MC_EBIT_NONFINITE) ? MC_EBIT_NONFINITE : MC_EBIT_TAU);
    }
    if (!b.ok || j >= ng) return;
    // all mapping loads, then all field gathers (a node with vid < 0 is a
    // mid-range fill and gathers vertex 0 for nothing)
    int id[D + 1];
    float wk[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        id[k] = vid[k * ng + j];
        wk[k] = w[k * ng + j];
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
    xh[j] = xhat_of(q, b.c, b.step1);      // reconstructed grid x1', as the decoder rebuilds it
    if (dbg_v) dbg_v[j] = v;
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
// 64 consecutive x of one row (3-D) or of a run of rows (2-D) and sweeps
// MC_LZ_CHUNK planes (rows), carrying the previous plane's (row's) error in a
// register, so each node costs four (two) coalesced loads.  Outliers are
// counted per 1024-node tile with at most two atomics per wave and row (a
// 64-run meets at most two tiles); the counts were zeroed by k_resample.
// Loads are unconditional (inactive lanes read node 0, neighbours outside
// the grid are masked with bitwise ands, not selects) so that the compiler
// keeps a sweep's loads together instead of sinking them into branches.
// The result of an inactive lane is never used.
template <int D>
__device__ __forceinline__ int lz_line(const int32_t* __restrict__ p, unsigned j, bool act, bool hx, bool hy,
                                       unsigned n0)
{
    const unsigned jj = act ? j : 0u;
    const unsigned ox = (hx && act) ? 1u : 0u, oy = (hy && act) ? n0 : 0u;
    const int mx = -(int)hx, my = -(int)hy;
    const int a = p[jj];
    const int b = p[jj - ox];
    if (D == 2) return a - (b & mx);
    const int c = p[jj - oy];
    const int e = p[jj - oy - ox];
    return ((a - (b & mx)) - (c & my)) + (e & (mx & my));
}

__device__ __forceinline__ void lz_count(unsigned j, bool out, bool act, unsigned int* __restrict__ count)
{
    const unsigned long long m = __ballot(out);
    if (m == 0ull) return;
    const unsigned long long live = __ballot(act);
    const int first = __builtin_ctzll(live), last = 63 - __builtin_clzll(live);
    const unsigned jf = __shfl(j, first, 64), jl = __shfl(j, last, 64);
    const unsigned tf = jf / MC_TILE, tl = jl / MC_TILE;
    const unsigned long long lo = __ballot(out && j / MC_TILE == tf), hi = m & ~lo;
    if (lane_id() == first) {
        if (lo) atomicAdd(&count[tf], (unsigned)__popcll(lo));
        if (hi) atomicAdd(&count[tl], (unsigned)__popcll(hi));
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_lorenzo(const int32_t* __restrict__ p, int n0, int n1, int n2, int nxs,
                                                 unsigned nunits, uint16_t* __restrict__ codes,
                                                 unsigned int* __restrict__ count)
{
    const unsigned u = xcd_tile(blockIdx.x, gridDim.x) * 4u + (threadIdx.x >> 6);
    if (u >= nunits) return;
    const unsigned xs = u % (unsigned)nxs, r = u / (unsigned)nxs;
    const unsigned x = xs * 64u + (unsigned)lane_id();
    const bool act = x < (unsigned)n0, hx = x > 0;
    // the whole sweep's loads are issued before any is used
    constexpr int CH = MC_LZ_CHUNK;
    unsigned base, step;
    int l0, l1;
    bool hy = false;
    if (D == 3) {
        const unsigned y = r % (unsigned)n1, zc = r / (unsigned)n1;
        base = x + (unsigned)n0 * y;
        step = (unsigned)n0 * (unsigned)n1;
        l0 = (int)zc * CH;
        l1 = min(l0 + CH, n2);
        hy = y > 0;
    } else {
        base = x;
        step = (unsigned)n0;
        l0 = (int)r * CH;
        l1 = min(l0 + CH, n1);
    }
    // plane (row) l0 - 1 for the first difference; past the end, the last
    // plane (row) is read again and ignored
    const int pz = lz_line<D>(p, base + step * (unsigned)(l0 > 0 ? l0 - 1 : 0), act, hx, hy, (unsigned)n0);
    int prev = l0 > 0 ? pz : 0;
    int cur[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) cur[k] = lz_line<D>(p, base + step * (unsigned)min(l0 + k, l1 - 1), act, hx, hy, (unsigned)n0);
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        if (l0 + k >= l1) break;
        const int d = cur[k] - prev;
        prev = cur[k];
        const unsigned j = base + step * (unsigned)(l0 + k);
        const bool in = d >= -(MC_R - 1) && d <= MC_R - 1;
        if (act) codes[j] = in ? (uint16_t)(d + MC_R) : (uint16_t)0;
        lz_count(j, act && !in, act, count);
    }
}

// ---------------------------------------------------------------------------
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

// Learned mode, first pass: per 4096-vertex block, the cost of the plain and
// of the shifted codes: sum of bitlen(zigzag(code)) over coded vertices plus
// (32 + 8 sizeof(T)) per outlier.  Integer atomics: order-independent.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_learned_cost(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                      const float* __restrict__ xh, const T* __restrict__ x,
                                                      const RangeOut* __restrict__ range, BoundParams bp,
                                                      const int32_t* __restrict__ rho_q,
                                                      unsigned int* __restrict__ bcost)
{
    __shared__ long long s_red[4];
    const DevBound b = make_bound(range, bp);
    const long long tile = xcd_tile(blockIdx.x, gridDim.x);
    const int ocost = 32 + 8 * (int)sizeof(T);
    long long v[MC_IPT];
    bool act[MC_IPT];
    T xv[MC_IPT];
    int rq[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        v[i] = tile * MC_TILE + i * MC_WG + threadIdx.x;
        act[i] = v[i] < nv && b.ok;
        const long long vc = act[i] ? v[i] : 0;
        xv[i] = x[vc];
        rq[i] = rho_q[vc];
    }
    float g[MC_IPT];
    back_interp_n<D, MC_IPT>(coords, nv, gg, xh, v, act, g);
    int cp = 0, cl = 0;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (!act[i]) continue;
        int qi;
        if (quantize_residual<T>(xv[i], g[i], b, qi)) {
            const int l = qi - rq[i];
            cp += zz_bits(qi);
            cl += (l >= -(MC_R - 1) && l <= MC_R - 1) ? zz_bits(l) : ocost;
        } else {
            cp += ocost;
            cl += ocost;
        }
    }
    const long long sp = block_sum_i64(cp, s_red);
    const long long sl = block_sum_i64(cl, s_red);
    if (threadIdx.x == 0) {
        const long long blk = (tile * MC_TILE) / MC_LBLOCK;   // a tile lies inside one block
        atomicAdd(&bcost[2 * blk], (unsigned)sp);
        atomicAdd(&bcost[2 * blk + 1], (unsigned)sl);
    }
}

// Residual codes of one tile (1024 vertices) and its outlier count; bit 31
// of the count marks the first tile of a learned block.
template <typename T, int D, bool LEARNED>
__global__ __launch_bounds__(256) void k_residual(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                  const float* __restrict__ xh, const T* __restrict__ x,
                                                  const RangeOut* __restrict__ range, BoundParams bp,
                                                  const int32_t* __restrict__ rho_q,
                                                  const unsigned int* __restrict__ bcost,
                                                  uint16_t* __restrict__ codes, uint32_t* __restrict__ bflags,
                                                  float* __restrict__ dbg_g, unsigned int* __restrict__ count)
{
    __shared__ int s_cnt[4];
    const DevBound b = make_bound(range, bp);
    const long long tile = xcd_tile(blockIdx.x, gridDim.x);
    // every tile lies inside one decision block (MC_LBLOCK % MC_TILE == 0)
    const long long blk = (tile * MC_TILE) / MC_LBLOCK;
    bool learned = false;
    if (LEARNED) learned = bcost[2 * blk + 1] < bcost[2 * blk];
    long long v[MC_IPT];
    bool act[MC_IPT];
    T xv[MC_IPT];
    int rq[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        v[i] = tile * MC_TILE + i * MC_WG + threadIdx.x;
        act[i] = v[i] < nv && b.ok;
        const long long vc = act[i] ? v[i] : 0;
        xv[i] = x[vc];
        rq[i] = (LEARNED && learned) ? rho_q[vc] : 0;
    }
    float g[MC_IPT];
    back_interp_n<D, MC_IPT>(coords, nv, gg, xh, v, act, g);
    int nout = 0;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (!act[i]) continue;
        if (dbg_g) dbg_g[v[i]] = g[i];
        int qi;
        bool ok = quantize_residual<T>(xv[i], g[i], b, qi);
        if (LEARNED && ok && learned) {
            qi -= rq[i];
            ok = qi >= -(MC_R - 1) && qi <= MC_R - 1;
        }
        codes[v[i]] = ok ? (uint16_t)(qi + MC_R) : (uint16_t)0;
        nout += ok ? 0 : 1;
    }
    const bool first_of_block = (tile * MC_TILE) % MC_LBLOCK == 0;
    nout = wave_sum(nout);
    if (lane_id() == 0) s_cnt[threadIdx.x >> 6] = nout;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned c = (unsigned)(s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3]);
        if (LEARNED && learned && first_of_block) {
            c |= 0x80000000u;
            atomicOr(&bflags[blk >> 5], 1u << (blk & 31));
        }
        count[tile] = c;
    }
}

// Exclusive scan of the per-tile outlier counts (bit 31 excluded), one
// workgroup per list: block 0 the grid tiles, block 1 the vertex tiles.
// Writes the totals to the result header and flags a capacity overflow.
__global__ __launch_bounds__(1024) void k_scan_counts(const unsigned int* __restrict__ gcount, long long ntg,
                                                      unsigned int* __restrict__ goff, long long gcap,
                                                      const unsigned int* __restrict__ vcount, long long ntv,
                                                      unsigned int* __restrict__ voff, long long vcap,
                                                      unsigned int* __restrict__ err, mc_result* __restrict__ res)
{
    const int PT = 8;
    __shared__ unsigned s_v[1024 * PT];
    __shared__ unsigned s_w[16];
    __shared__ unsigned s_carry, s_learn;
    const bool vert = blockIdx.x == 1;
    const unsigned int* cnt = vert ? vcount : gcount;
    unsigned int* off = vert ? voff : goff;
    const long long n = vert ? ntv : ntg;
    if (threadIdx.x == 0) { s_carry = 0; s_learn = 0; }
    unsigned learned = 0;
    for (long long base = 0; base < n; base += 1024 * PT) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PT; ++k) {            // coalesced load into LDS
            const long long i = base + k * 1024 + threadIdx.x;
            const unsigned c = i < n ? cnt[i] : 0u;
            learned += c >> 31;
            s_v[k * 1024 + threadIdx.x] = c & 0x7fffffffu;
        }
        __syncthreads();
        unsigned v[PT], run = 0;
#pragma unroll
        for (int k = 0; k < PT; ++k) { v[k] = s_v[threadIdx.x * PT + k]; run += v[k]; }
        const unsigned inc = wave_incl_scan(run);
        const int w = threadIdx.x >> 6;
        if (lane_id() == 63) s_w[w] = inc;
        __syncthreads();
        unsigned pre = s_carry, tot = 0;
        for (int k = 0; k < 16; ++k) { if (k < w) pre += s_w[k]; tot += s_w[k]; }
        unsigned acc = pre + inc - run;
#pragma unroll
        for (int k = 0; k < PT; ++k) { s_v[threadIdx.x * PT + k] = acc; acc += v[k]; }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const long long i = base + k * 1024 + threadIdx.x;
            if (i < n) off[i] = s_v[k * 1024 + threadIdx.x];
        }
        if (threadIdx.x == 0) s_carry += tot;
    }
    learned = wave_sum(learned);
    if (lane_id() == 0) atomicAdd(&s_learn, learned);
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long total = s_carry;
        if (vert) {
            res->n_vertex_outliers = total;
            res->n_learned_blocks = s_learn;
            if (total > vcap) atomicOr(err, MC_EBIT_VCAP);
        } else {
            res->n_grid_outliers = total;
            if (total > gcap) atomicOr(err, MC_EBIT_GCAP);
        }
    }
}

// Gathers the outliers of each tile that has any, in index order: grid
// tiles (blocks < ntg) recompute the Lorenzo error of their code-0 nodes,
// vertex tiles copy the raw value.  Block 0 also writes the final status.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ p, int n0, int n1, long long ng,
                                                 const uint16_t* __restrict__ gcodes,
                                                 const unsigned int* __restrict__ gcount,
                                                 const unsigned int* __restrict__ goff, int32_t* __restrict__ gidx,
                                                 int32_t* __restrict__ gdelta, long long gcap, long long ntg,
                                                 const T* __restrict__ x, long long nv,
                                                 const uint16_t* __restrict__ vcodes,
                                                 const unsigned int* __restrict__ vcount,
                                                 const unsigned int* __restrict__ voff, int32_t* __restrict__ vidx,
                                                 T* __restrict__ vval, long long vcap,
                                                 const unsigned int* __restrict__ err, mc_result* __restrict__ res)
{
    __shared__ int s_cnt[MC_IPT * 4 + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        unsigned e = *err;
        if (res->n_grid_outliers > gcap) e |= MC_EBIT_GCAP;
        if (res->n_vertex_outliers > vcap) e |= MC_EBIT_VCAP;
        res->status = status_from_bits(e);
    }
    const bool vert = blockIdx.x >= ntg;
    const long long tile = vert ? blockIdx.x - ntg : blockIdx.x;
    const unsigned c = (vert ? vcount[tile] : gcount[tile]) & 0x7fffffffu;
    if (c == 0) return;
    const long long n = vert ? nv : ng;
    const uint16_t* codes = vert ? vcodes : gcodes;
    bool flag[MC_IPT];
    int rank[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        const long long j = tile * MC_TILE + i * MC_WG + threadIdx.x;
        flag[i] = j < n && codes[j] == 0;
    }
    tile_ranks(flag, rank, s_cnt);
    const long long base = vert ? voff[tile] : goff[tile];
    const long long n01 = (long long)n0 * n1;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (!flag[i]) continue;
        const long long j = tile * MC_TILE + i * MC_WG + threadIdx.x;
        const long long pos = base + rank[i];
        if (vert) {
            if (pos < vcap) { vidx[pos] = (int32_t)j; vval[pos] = x[j]; }
        } else if (pos < gcap) {
            const int i0 = (int)(j % n0);
            const long long r = j / n0;
            gidx[pos] = (int32_t)j;
            gdelta[pos] = (int32_t)lorenzo_delta<D>(p, j, i0, (int)(r % n1), (int)(r / n1), n0, n01);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace mck {

hipError_t range(const void* x, int dtype, long long n, unsigned long long* partial, RangeOut* cur,
                 unsigned int* zero, long long nzero, hipStream_t s)
{
    const int nblocks = 1024;
    {
        ProfScope ps("k_range", s);
        if (dtype == MC_F64)
            hipLaunchKernelGGL(k_range<double>, dim3(nblocks), dim3(256), 0, s, (const double*)x, n, partial, zero, nzero);
        else
            hipLaunchKernelGGL(k_range<float>, dim3(nblocks), dim3(256), 0, s, (const float*)x, n, partial, zero, nzero);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ProfScope ps("k_range_final", s);
    hipLaunchKernelGGL(k_range_final, dim3(1), dim3(256), 0, s, partial, nblocks, cur);
    return hipGetLastError();
}

hipError_t resample(const int32_t* vid, const float* w, int dim, long long ng, const void* x, int dtype,
                    const RangeOut* range, BoundParams bp, int32_t* p, float* xh, float* dbg_v, uint32_t* bflags,
                    long long nbflags, unsigned int* err, mc_result* res, unsigned int* gcount, long long ntg,
                    hipStream_t s)
{
    ProfScope ps("k_resample", s);
    const long long need = ng > nbflags ? ng : nbflags;
    dim3 grid((unsigned)((need + 255) / 256));
#define MC_RS(T, D) hipLaunchKernelGGL((k_resample<T, D>), grid, dim3(256), 0, s, vid, w, ng, (const T*)x, range, bp, \
                                       p, xh, dbg_v, bflags, nbflags, err, res, dtype, gcount, ntg)
    if (dtype == MC_F64) { if (dim == 2) MC_RS(double, 2); else MC_RS(double, 3); }
    else { if (dim == 2) MC_RS(float, 2); else MC_RS(float, 3); }
#undef MC_RS
    return hipGetLastError();
}

hipError_t lorenzo(const int32_t* p, int dim, int n0, int n1, int n2, long long ng, uint16_t* codes,
                   unsigned int* count, hipStream_t s)
{
    ProfScope ps("k_lorenzo", s);
    (void)ng;
    const int nxs = (n0 + 63) / 64;
    const long long lines = (long long)nxs * (dim == 3 ? (long long)n1 : 1);
    const int len = dim == 3 ? n2 : n1;
    const unsigned nunits = (unsigned)(lines * ((len + MC_LZ_CHUNK - 1) / MC_LZ_CHUNK));
    dim3 grid((nunits + 3) / 4);
    if (dim == 2)
        hipLaunchKernelGGL(k_lorenzo<2>, grid, dim3(256), 0, s, p, n0, n1, n2, nxs, nunits, codes, count);
    else
        hipLaunchKernelGGL(k_lorenzo<3>, grid, dim3(256), 0, s, p, n0, n1, n2, nxs, nunits, codes, count);
    return hipGetLastError();
}

hipError_t residual(const float* coords, long long nv, GridGeom gg, const float* xh, const void* x, int dtype,
                    const RangeOut* range, BoundParams bp, const int32_t* rho_q, unsigned int* bcost, uint16_t* codes,
                    uint32_t* bflags, float* dbg_g, unsigned int* count, hipStream_t s)
{
    const bool L = rho_q != nullptr;
    if (L) {
        ProfScope ps("k_learned_cost", s);
        dim3 grid((unsigned)((nv + MC_TILE - 1) / MC_TILE));
#define MC_LC(T, D) hipLaunchKernelGGL((k_learned_cost<T, D>), grid, dim3(256), 0, s, coords, nv, gg, xh, (const T*)x, \
                                       range, bp, rho_q, bcost)
        if (dtype == MC_F64) { if (gg.dim == 2) MC_LC(double, 2); else MC_LC(double, 3); }
        else { if (gg.dim == 2) MC_LC(float, 2); else MC_LC(float, 3); }
#undef MC_LC
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ProfScope ps(L ? "k_residual_learned" : "k_residual", s);
    const long long ntiles = (nv + MC_TILE - 1) / MC_TILE;
    dim3 grid((unsigned)ntiles);
#define MC_RQ(T, D, LL) hipLaunchKernelGGL((k_residual<T, D, LL>), grid, dim3(256), 0, s, coords, nv, gg, xh, (const T*)x, \
                                           range, bp, rho_q, bcost, codes, bflags, dbg_g, count)
    if (dtype == MC_F64) {
        if (gg.dim == 2) { if (L) MC_RQ(double, 2, true); else MC_RQ(double, 2, false); }
        else { if (L) MC_RQ(double, 3, true); else MC_RQ(double, 3, false); }
    } else {
        if (gg.dim == 2) { if (L) MC_RQ(float, 2, true); else MC_RQ(float, 2, false); }
        else { if (L) MC_RQ(float, 3, true); else MC_RQ(float, 3, false); }
    }
#undef MC_RQ
    return hipGetLastError();
}

hipError_t compact(const int32_t* p, int dim, int n0, int n1, long long ng, const uint16_t* gcodes, unsigned int* gcount,
                   unsigned int* goff, int32_t* gidx, int32_t* gdelta, long long gcap, const void* x, int dtype,
                   long long nv, const uint16_t* vcodes, unsigned int* vcount, unsigned int* voff, int32_t* vidx,
                   void* vval, long long vcap, unsigned int* err, mc_result* res, hipStream_t s)
{
    const long long ntg = (ng + MC_TILE - 1) / MC_TILE, ntv = (nv + MC_TILE - 1) / MC_TILE;
    {
        ProfScope ps("k_scan_counts", s);
        hipLaunchKernelGGL(k_scan_counts, dim3(2), dim3(1024), 0, s, gcount, ntg, goff, gcap, vcount, ntv, voff, vcap,
                           err, res);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ProfScope ps("k_scatter", s);
    dim3 grid((unsigned)(ntg + ntv));
#define MC_SC(T, D) hipLaunchKernelGGL((k_scatter<T, D>), grid, dim3(256), 0, s, p, n0, n1, ng, gcodes, gcount, goff, \
                                       gidx, gdelta, gcap, ntg, (const T*)x, nv, vcodes, vcount, voff, vidx, (T*)vval, \
                                       vcap, err, res)
    if (dtype == MC_F64) { if (dim == 2) MC_SC(double, 2); else MC_SC(double, 3); }
    else { if (dim == 2) MC_SC(float, 2); else MC_SC(float, 3); }
#undef MC_SC
    return hipGetLastError();
}

}  // namespace mck
