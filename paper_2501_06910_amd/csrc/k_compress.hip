// k_compress.hip -- the compression hot path on gfx950 (paper Alg. 3 with
// the residual taken against the reconstructed grid):
//   k_range      field min/max (ordered integer keys) and non-finite check;
//                also clears the look-back state of the kernels after it
//   k_resample   f: v_j = sum_k w_kj * x[vid_kj] (FP32, fixed order), then
//                the prequantised grid p_j = rint((v_j - c) / (2 tau1))
//   k_lorenzo    Lorenzo prediction error of p, uint16 codes, outliers
//                compacted in index order (ballots + decoupled look-back)
//   k_residual   g: multilinear x1' at each vertex, residual quantisation
//                with the per-vertex bound check, optional learned shift
//                with the per-block choice, outliers in index order
#include "mc_dev.h"
#include "mc_kernels.h"

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_range(const T* __restrict__ x, long long n,
                                               unsigned long long* __restrict__ partial,
                                               unsigned int* __restrict__ done, RangeOut* __restrict__ out,
                                               unsigned long long* __restrict__ zero_a, long long nzero_a,
                                               unsigned int* __restrict__ zero_b, long long nzero_b,
                                               unsigned int* __restrict__ err)
{
    __shared__ unsigned long long s_mn[4], s_mx[4];
    __shared__ unsigned int s_fl[4];
    __shared__ int s_last;
    const long long stride = (long long)gridDim.x * 256;
    const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
    for (long long i = gid; i < nzero_a; i += stride) zero_a[i] = 0ull;
    for (long long i = gid; i < nzero_b; i += stride) zero_b[i] = 0u;
    if (gid == 0) *err = 0u;

    unsigned long long kmn = ~0ull, kmx = 0ull;
    unsigned int fl = 0;
    for (long long i = gid; i < n; i += stride) {
        double d = (double)x[i];
        if (!isfinite(d)) {
            fl = MC_EBIT_NONFINITE;
        } else {
            unsigned long long k = dkey(d);
            kmn = k < kmn ? k : kmn;
            kmx = k > kmx ? k : kmx;
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        unsigned long long a = __shfl_xor(kmn, d, 64), b = __shfl_xor(kmx, d, 64);
        unsigned int f = __shfl_xor(fl, d, 64);
        kmn = a < kmn ? a : kmn;
        kmx = b > kmx ? b : kmx;
        fl |= f;
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) { s_mn[w] = kmn; s_mx[w] = kmx; s_fl[w] = fl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            s_mn[0] = s_mn[k] < s_mn[0] ? s_mn[k] : s_mn[0];
            s_mx[0] = s_mx[k] > s_mx[0] ? s_mx[k] : s_mx[0];
            s_fl[0] |= s_fl[k];
        }
        partial[3 * blockIdx.x + 0] = s_mn[0];
        partial[3 * blockIdx.x + 1] = s_mx[0];
        partial[3 * blockIdx.x + 2] = s_fl[0];
        __threadfence();
        unsigned int prev = atomicAdd(done, 1u);
        s_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        unsigned long long a = ~0ull, b = 0ull, f = 0ull;
        for (unsigned int k = 0; k < gridDim.x; ++k) {
            unsigned long long pa = __hip_atomic_load(&partial[3 * k + 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned long long pb = __hip_atomic_load(&partial[3 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned long long pf = __hip_atomic_load(&partial[3 * k + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            a = pa < a ? pa : a;
            b = pb > b ? pb : b;
            f |= pf;
        }
        out->kmin = a;
        out->kmax = b;
        out->flags = (unsigned int)f;
        *done = 0u;                      // ready for the next call
    }
}

// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(256) void k_resample(const int32_t* __restrict__ vid, const float* __restrict__ w,
                                                  long long ng, const T* __restrict__ x,
                                                  const RangeOut* __restrict__ range, BoundParams bp,
                                                  int32_t* __restrict__ p, float* __restrict__ dbg_v,
                                                  uint32_t* __restrict__ bflags, long long nbflags,
                                                  unsigned int* __restrict__ err, mc_result* __restrict__ res,
                                                  int dtype)
{
    const DevBound b = make_bound(range, bp);
    {
        const long long jz = (long long)blockIdx.x * 256 + threadIdx.x;
        if (bflags && jz < nbflags) bflags[jz] = 0u;      // learned-block bits start clear
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        res->status = b.ok ? 0 : 1;
        res->dtype = dtype;
        res->tau = b.tau;
        res->tau1 = b.tau1;
        res->tau2 = b.tau2;
        res->c = b.c;
        res->xmin = b.xmin;
        res->xmax = b.xmax;
        if (!b.ok) atomicOr(err, range->flags & MC_EBIT_NONFINITE ? MC_EBIT_NONFINITE : MC_EBIT_TAU);
    }
    if (!b.ok) return;
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (j >= ng) return;
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
    if (dbg_v) dbg_v[j] = v;
}

// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_lorenzo(const int32_t* __restrict__ p, int n0, int n1, int n2,
                                                 long long ng, uint16_t* __restrict__ codes,
                                                 int32_t* __restrict__ oidx, int32_t* __restrict__ odelta,
                                                 long long cap, unsigned long long* __restrict__ st,
                                                 unsigned int* __restrict__ ticket, long long ntiles,
                                                 unsigned int* __restrict__ err, mc_result* __restrict__ res)
{
    __shared__ int s_cnt[65];
    __shared__ long long s_slot;
    const long long tile = take_ticket(ticket, &s_slot);
    const unsigned n01 = (unsigned)n0 * (unsigned)n1;
    bool flag[MC_IPT];
    int rank[MC_IPT];
    int dv[MC_IPT];
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        const long long jj = tile * MC_TILE + i * MC_WG + threadIdx.x;
        flag[i] = false;
        dv[i] = 0;
        if (jj < ng) {
            const unsigned j = (unsigned)jj;
            const unsigned i0 = j % (unsigned)n0;
            const unsigned r = j / (unsigned)n0;
            const unsigned i1 = r % (unsigned)n1;
            const unsigned i2 = r / (unsigned)n1;
            long long pred;
            const long long a = i0 > 0 ? p[j - 1] : 0;
            const long long bq = i1 > 0 ? p[j - n0] : 0;
            const long long ab = (i0 > 0 && i1 > 0) ? p[j - n0 - 1] : 0;
            if (D == 2) {
                pred = a + bq - ab;
            } else {
                const long long cz = i2 > 0 ? p[j - n01] : 0;
                const long long ac = (i0 > 0 && i2 > 0) ? p[j - n01 - 1] : 0;
                const long long bc = (i1 > 0 && i2 > 0) ? p[j - n01 - n0] : 0;
                const long long abc = (i0 > 0 && i1 > 0 && i2 > 0) ? p[j - n01 - n0 - 1] : 0;
                pred = a + bq + cz - ab - ac - bc + abc;
            }
            const long long d = (long long)p[j] - pred;
            if (d >= -(MC_R - 1) && d <= MC_R - 1) {
                codes[j] = (uint16_t)(d + MC_R);
            } else {
                codes[j] = 0;
                flag[i] = true;
                dv[i] = (int)d;
            }
        }
    }
    const int total = tile_ranks(flag, rank, s_cnt);
    const long long excl = tile_prefix(st, tile, total, &s_slot);
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (flag[i]) {
            const long long pos = excl + rank[i];
            if (pos < cap) {
                oidx[pos] = (int32_t)(tile * MC_TILE + i * MC_WG + threadIdx.x);
                odelta[pos] = dv[i];
            }
        }
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) {
        const long long n = excl + total;
        res->n_grid_outliers = n;
        if (n > cap) atomicOr(err, MC_EBIT_GCAP);
    }
}

// ---------------------------------------------------------------------------
// g(x1') at a vertex from the prequantised grid (x1' recomputed on the fly).
template <int D>
__device__ __forceinline__ float back_interp(const float* __restrict__ coords, long long nv, long long v,
                                             const GridGeom& gg, const int32_t* __restrict__ p,
                                             double c, double step1)
{
    int i0, i1, i2 = 0;
    float t0, t1, t2 = 0.0f;
    axis_cell(coords[v], gg.of[0], gg.ihf[0], gg.n0, i0, t0);
    axis_cell(coords[nv + v], gg.of[1], gg.ihf[1], gg.n1, i1, t1);
    if (D == 3) axis_cell(coords[2 * nv + v], gg.of[2], gg.ihf[2], gg.n2, i2, t2);
    const long long n0 = gg.n0, n01 = (long long)gg.n0 * gg.n1;
    const long long j = i0 + n0 * i1 + n01 * i2;
    const float x00 = xhat_of(p[j], c, step1), x10 = xhat_of(p[j + 1], c, step1);
    const float x01 = xhat_of(p[j + n0], c, step1), x11 = xhat_of(p[j + n0 + 1], c, step1);
    const float c00 = lerpf_(x00, x10, t0);
    const float c10 = lerpf_(x01, x11, t0);
    const float c0 = lerpf_(c00, c10, t1);
    if (D == 2) return c0;
    const float y00 = xhat_of(p[j + n01], c, step1), y10 = xhat_of(p[j + n01 + 1], c, step1);
    const float y01 = xhat_of(p[j + n01 + n0], c, step1), y11 = xhat_of(p[j + n01 + n0 + 1], c, step1);
    const float c01 = lerpf_(y00, y10, t0);
    const float c11 = lerpf_(y01, y11, t0);
    const float c1 = lerpf_(c01, c11, t1);
    return lerpf_(c0, c1, t2);
}

__device__ __forceinline__ int zz_bits(int k)
{
    const unsigned z = ((unsigned)k << 1) ^ (unsigned)(k >> 31);
    return 32 - __clz(z);
}

template <typename T, int D, bool LEARNED>
__global__ __launch_bounds__(256) void k_residual(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                  const int32_t* __restrict__ p, const T* __restrict__ x,
                                                  const RangeOut* __restrict__ range, BoundParams bp,
                                                  const int32_t* __restrict__ rho_q,
                                                  uint16_t* __restrict__ codes, int32_t* __restrict__ oidx,
                                                  T* __restrict__ oval, long long cap,
                                                  uint32_t* __restrict__ bflags, float* __restrict__ dbg_g,
                                                  unsigned long long* __restrict__ st,
                                                  unsigned int* __restrict__ ticket, long long ntiles,
                                                  unsigned int* __restrict__ err, mc_result* __restrict__ res)
{
    __shared__ int s_cnt[65];
    __shared__ long long s_slot;
    __shared__ long long s_red[4];
    const DevBound b = make_bound(range, bp);
    const long long tile = take_ticket(ticket, &s_slot);
    bool flag[MC_IPT];
    int rank[MC_IPT];
    int code[MC_IPT];
    const int ocost = 32 + 8 * (int)sizeof(T);
    int cost_p = 0, cost_l = 0;
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        const long long v = tile * MC_TILE + i * MC_WG + threadIdx.x;
        flag[i] = false;
        code[i] = 0;
        if (v < nv && b.ok) {
            const float g = back_interp<D>(coords, nv, v, gg, p, b.c, b.step1);
            if (dbg_g) dbg_g[v] = g;
            const T xv = x[v];
            const double r = (double)xv - (double)g;
            const double q = rint(r * b.inv2);
            const T xr = (T)((double)g + q * b.step2);
            const bool ok = fabs(q) <= (double)(MC_R - 1) && fabs((double)xv - (double)xr) <= b.tau2;
            if (ok) {
                const int qi = (int)q;
                code[i] = qi;
                if (LEARNED) {
                    const int cl = qi - rho_q[v];
                    cost_p += zz_bits(qi);
                    cost_l += (cl >= -(MC_R - 1) && cl <= MC_R - 1) ? zz_bits(cl) : ocost;
                }
            } else {
                flag[i] = true;
                if (LEARNED) { cost_p += ocost; cost_l += ocost; }
            }
        }
    }
    bool learned = false;
    if (LEARNED) {
        const long long cp = block_sum_i64(cost_p, s_red);
        const long long cl = block_sum_i64(cost_l, s_red);
        learned = cl < cp;
        if (learned && threadIdx.x == 0) atomicOr(&bflags[tile >> 5], 1u << (tile & 31));
    }
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        const long long v = tile * MC_TILE + i * MC_WG + threadIdx.x;
        if (v < nv && b.ok) {
            if (LEARNED && learned && !flag[i]) {
                const int cl = code[i] - rho_q[v];
                if (cl >= -(MC_R - 1) && cl <= MC_R - 1) code[i] = cl;
                else flag[i] = true;
            }
            codes[v] = flag[i] ? (uint16_t)0 : (uint16_t)(code[i] + MC_R);
        }
    }
    const int total = tile_ranks(flag, rank, s_cnt);
    // outlier count in bits 0..31, learned-block count in bits 32..61
    const unsigned long long packed = (unsigned long long)total | ((unsigned long long)(learned ? 1 : 0) << 32);
    const unsigned long long exclp = tile_prefix(st, tile, packed, &s_slot);
    const long long excl = (long long)(exclp & 0xffffffffull);
#pragma unroll
    for (int i = 0; i < MC_IPT; ++i) {
        if (flag[i]) {
            const long long pos = excl + rank[i];
            const long long v = tile * MC_TILE + i * MC_WG + threadIdx.x;
            if (pos < cap) {
                oidx[pos] = (int32_t)v;
                oval[pos] = x[v];
            }
        }
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) {
        const unsigned long long incl = exclp + packed;
        const long long n = (long long)(incl & 0xffffffffull);
        res->n_vertex_outliers = n;
        res->n_learned_blocks = (long long)(incl >> 32);
        unsigned int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (n > cap) e |= MC_EBIT_VCAP;
        res->status = status_from_bits(e);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace mck {

hipError_t range(const void* x, int dtype, long long n, unsigned long long* partial, int nblocks,
                 unsigned int* done, RangeOut* out, unsigned long long* zero_a, long long nzero_a,
                 unsigned int* zero_b, long long nzero_b, unsigned int* err, hipStream_t s)
{
    ProfScope ps("k_range", s);
    if (dtype == MC_F64)
        hipLaunchKernelGGL(k_range<double>, dim3(nblocks), dim3(256), 0, s, (const double*)x, n, partial, done,
                           out, zero_a, nzero_a, zero_b, nzero_b, err);
    else
        hipLaunchKernelGGL(k_range<float>, dim3(nblocks), dim3(256), 0, s, (const float*)x, n, partial, done, out,
                           zero_a, nzero_a, zero_b, nzero_b, err);
    return hipGetLastError();
}

hipError_t resample(const int32_t* vid, const float* w, int dim, long long ng, const void* x, int dtype,
                    const RangeOut* range, BoundParams bp, int32_t* p, float* dbg_v, uint32_t* bflags,
                    long long nbflags, unsigned int* err, mc_result* res, hipStream_t s)
{
    ProfScope ps("k_resample", s);
    long long need = ng > nbflags ? ng : nbflags;
    dim3 grid((unsigned)((need + 255) / 256));
#define MC_RS(T, D) hipLaunchKernelGGL((k_resample<T, D>), grid, dim3(256), 0, s, vid, w, ng, (const T*)x, range, bp, \
                                       p, dbg_v, bflags, nbflags, err, res, dtype)
    if (dtype == MC_F64) { if (dim == 2) MC_RS(double, 2); else MC_RS(double, 3); }
    else { if (dim == 2) MC_RS(float, 2); else MC_RS(float, 3); }
#undef MC_RS
    return hipGetLastError();
}

hipError_t lorenzo(const int32_t* p, int dim, int n0, int n1, int n2, long long ng, uint16_t* codes,
                   int32_t* oidx, int32_t* odelta, long long cap, unsigned long long* st, unsigned int* ticket,
                   unsigned int* err, mc_result* res, hipStream_t s)
{
    ProfScope ps("k_lorenzo", s);
    long long ntiles = (ng + MC_TILE - 1) / MC_TILE;
    if (dim == 2)
        hipLaunchKernelGGL(k_lorenzo<2>, dim3((unsigned)ntiles), dim3(256), 0, s, p, n0, n1, n2, ng, codes, oidx,
                           odelta, cap, st, ticket, ntiles, err, res);
    else
        hipLaunchKernelGGL(k_lorenzo<3>, dim3((unsigned)ntiles), dim3(256), 0, s, p, n0, n1, n2, ng, codes, oidx,
                           odelta, cap, st, ticket, ntiles, err, res);
    return hipGetLastError();
}

hipError_t residual(const float* coords, long long nv, GridGeom gg, const int32_t* p, const void* x, int dtype,
                    const RangeOut* range, BoundParams bp, const int32_t* rho_q, uint16_t* codes, int32_t* oidx,
                    void* oval, long long cap, uint32_t* bflags, float* dbg_g, unsigned long long* st,
                    unsigned int* ticket, unsigned int* err, mc_result* res, hipStream_t s)
{
    ProfScope ps(rho_q ? "k_residual_learned" : "k_residual", s);
    long long ntiles = (nv + MC_TILE - 1) / MC_TILE;
    dim3 grid((unsigned)ntiles);
#define MC_RQ(T, D, L) hipLaunchKernelGGL((k_residual<T, D, L>), grid, dim3(256), 0, s, coords, nv, gg, p, (const T*)x, \
                                          range, bp, rho_q, codes, oidx, (T*)oval, cap, bflags, dbg_g, st, ticket,   \
                                          ntiles, err, res)
    const bool L = rho_q != nullptr;
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

}  // namespace mck
