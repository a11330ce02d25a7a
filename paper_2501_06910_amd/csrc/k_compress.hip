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
                                                  mc_result* __restrict__ res, int dtype)
{
    const DevBound b = make_bound(range, bp);
    const long long j = (long long)xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (bflags && j < nbflags) bflags[j] = 0u;      // learned-block bits start clear
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
    const int v0 = vid[j];
    float v;
    if (v0 < 0) {
        v = (float)b.c;
    } else {
        float acc = w[j] * as_float(x[v0]);
#pragma unroll
        for (int k = 1; k <= D; ++k) acc = acc + w[k * ng + j] * as_float(x[vid[k * ng + j]]);
        v = acc;
    }
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

// Codes of one tile (1024 nodes, 4 per thread, strided by 256) and its
// outlier count; the outliers themselves are gathered by k_scatter.
template <int D>
__global__ __launch_bounds__(256) void k_lorenzo(const int32_t* __restrict__ p, int n0, int n1, int n2,
                                                 long long ng, uint16_t* __restrict__ codes,
                                                 unsigned int* __restrict__ count)
{
    __shared__ int s_cnt[4];
    const long long tile = xcd_tile(blockIdx.x, gridDim.x);
    const long long n01 = (long long)n0 * n1;
    long long j = tile * MC_TILE + threadIdx.x;
    const unsigned j32 = (unsigned)j, r32 = j32 / (unsigned)n0;     // ng < 2^31
    int i0 = (int)(j32 - r32 * (unsigned)n0);
    int i1 = (int)(r32 % (unsigned)n1);
    int i2 = (int)(r32 / (unsigned)n1);
    int nout = 0;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (j < ng) {
            const long long d = lorenzo_delta<D>(p, j, i0, i1, i2, n0, n01);
            const bool in = d >= -(MC_R - 1) && d <= MC_R - 1;
            codes[j] = in ? (uint16_t)(d + MC_R) : (uint16_t)0;
            nout += in ? 0 : 1;
        }
        j += MC_WG;
        i0 += MC_WG;
        while (i0 >= n0) {
            i0 -= n0;
            if (++i1 == n1) { i1 = 0; ++i2; }
        }
    }
    nout = wave_sum(nout);
    if (lane_id() == 0) s_cnt[threadIdx.x >> 6] = nout;
    __syncthreads();
    if (threadIdx.x == 0) count[tile] = (unsigned)(s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3]);
}

// ---------------------------------------------------------------------------
// g(x1') at a vertex: multilinear interpolation of the reconstructed grid.
template <int D>
__device__ __forceinline__ float back_interp(const float* __restrict__ coords, long long nv, long long v,
                                             const GridGeom& gg, const float* __restrict__ xh)
{
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
    const float c0 = lerpf_(c00, c10, t1);
    if (D == 2) return c0;
    const float c01 = lerpf_(xh[j + n01], xh[j + n01 + 1], t0);
    const float c11 = lerpf_(xh[j + n01 + n0], xh[j + n01 + n0 + 1], t0);
    const float c1 = lerpf_(c01, c11, t1);
    return lerpf_(c0, c1, t2);
}

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
    const long long lb = xcd_tile(blockIdx.x, gridDim.x);
    const long long v = lb * 256 + threadIdx.x;
    const int ocost = 32 + 8 * (int)sizeof(T);
    int cp = 0, cl = 0;
    if (v < nv && b.ok) {
        const float g = back_interp<D>(coords, nv, v, gg, xh);
        int qi;
        if (quantize_residual<T>(x[v], g, b, qi)) {
            const int l = qi - rho_q[v];
            cp = zz_bits(qi);
            cl = (l >= -(MC_R - 1) && l <= MC_R - 1) ? zz_bits(l) : ocost;
        } else {
            cp = ocost;
            cl = ocost;
        }
    }
    const long long sp = block_sum_i64(cp, s_red);
    const long long sl = block_sum_i64(cl, s_red);
    if (threadIdx.x == 0) {
        const long long blk = (lb * 256) / MC_LBLOCK;
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
    int nout = 0;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        const long long v = tile * MC_TILE + i * MC_WG + threadIdx.x;
        if (v < nv && b.ok) {
            const float g = back_interp<D>(coords, nv, v, gg, xh);
            if (dbg_g) dbg_g[v] = g;
            int qi;
            bool ok = quantize_residual<T>(x[v], g, b, qi);
            if (LEARNED && ok && learned) {
                qi -= rho_q[v];
                ok = qi >= -(MC_R - 1) && qi <= MC_R - 1;
            }
            codes[v] = ok ? (uint16_t)(qi + MC_R) : (uint16_t)0;
            nout += ok ? 0 : 1;
        }
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
                    long long nbflags, unsigned int* err, mc_result* res, hipStream_t s)
{
    ProfScope ps("k_resample", s);
    const long long need = ng > nbflags ? ng : nbflags;
    dim3 grid((unsigned)((need + 255) / 256));
#define MC_RS(T, D) hipLaunchKernelGGL((k_resample<T, D>), grid, dim3(256), 0, s, vid, w, ng, (const T*)x, range, bp, \
                                       p, xh, dbg_v, bflags, nbflags, err, res, dtype)
    if (dtype == MC_F64) { if (dim == 2) MC_RS(double, 2); else MC_RS(double, 3); }
    else { if (dim == 2) MC_RS(float, 2); else MC_RS(float, 3); }
#undef MC_RS
    return hipGetLastError();
}

hipError_t lorenzo(const int32_t* p, int dim, int n0, int n1, int n2, long long ng, uint16_t* codes,
                   unsigned int* count, hipStream_t s)
{
    ProfScope ps("k_lorenzo", s);
    const long long ntiles = (ng + MC_TILE - 1) / MC_TILE;
    if (dim == 2)
        hipLaunchKernelGGL(k_lorenzo<2>, dim3((unsigned)ntiles), dim3(256), 0, s, p, n0, n1, n2, ng, codes, count);
    else
        hipLaunchKernelGGL(k_lorenzo<3>, dim3((unsigned)ntiles), dim3(256), 0, s, p, n0, n1, n2, ng, codes, count);
    return hipGetLastError();
}

hipError_t residual(const float* coords, long long nv, GridGeom gg, const float* xh, const void* x, int dtype,
                    const RangeOut* range, BoundParams bp, const int32_t* rho_q, unsigned int* bcost, uint16_t* codes,
                    uint32_t* bflags, float* dbg_g, unsigned int* count, hipStream_t s)
{
    const bool L = rho_q != nullptr;
    if (L) {
        ProfScope ps("k_learned_cost", s);
        dim3 grid((unsigned)((nv + 255) / 256));
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
