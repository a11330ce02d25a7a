// k_decode.hip -- decompression on gfx950 (paper Alg. 4).
//   k_d2_*     2-D Lorenzo inverse on 256-column row segments (below)
//   k_d3_*     3-D Lorenzo inverse for rows of at most 1024 nodes: tile
//              face sums, their prefixes, then x1' straight from the codes
//              (below)
//   k_dec_xy_* (3-D, longer rows) inverse within each z-plane: d = code - R
//              (outliers by binary search in the ascending outlier list);
//              column totals per chunk of rows, their prefix over the
//              plane's chunks, then running column sums plus a wave scan
//              along x
//   k_dec_z_*  (3-D, longer rows) inclusive prefix along z in chunks of
//              planes: totals, prefix over the chunks, apply; in place
//   k_vdecode  g(x1') at each vertex from the decoded grid, dequantisation
//              x' = (T)(g + q * 2 tau2), raw values for outliers (the
//              learned decode, which adds the network's shift, is
//              k_mlp_vdecode in k_mlp.hip)
#include "mc_dev.h"
#include "mc_kernels.h"

// Exclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ int wave_excl_scan(int v)
{
    return wave_incl_scan(v) - v;
}

// The grid decoder is the inclusive prefix sum of the Lorenzo errors along
// every axis.  Generic 3-D path: the z prefix runs first (on the decoded errors), then
// the 2-D prefix of each plane; the last pass writes x1' = (float)(c + p *
// 2 tau1) directly.  Tiles: (chunk of rows) x (all x) per plane for the xy
// part, (chunk of planes) x (the same chunk of rows) for the z part, so the
// z pass can also emit the xy column totals.
//   k_dec_xy_carry  per (plane, column): exclusive prefix over row chunks
//   k_dec_xy_apply  running column sums from the carry, x-scan of each row,
//                   x1' written (input: the z-prefixed errors)
//   k_dec_z_tot     3-D: per (plane chunk, position): sum of the errors
//   k_dec_z_carry   per position: exclusive prefix over plane chunks
//   k_dec_z_apply   z-prefixed errors + xy column totals of every tile
// Exclusive prefix over chunks, in place: one thread per position, the
// chunk values loaded 32 at a time before any is used.
__device__ __forceinline__ void excl_prefix_strided(int* __restrict__ a, long long first, long long stride, int n)
{
    int run = 0;
    for (int b = 0; b < n; b += 32) {
        int t[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) t[u] = a[first + (long long)min(b + u, n - 1) * stride];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            if (b + u < n) a[first + (long long)(b + u) * stride] = run;
            run += b + u < n ? t[u] : 0;
        }
    }
}

// Exclusive prefix over the nyc row chunks of every (plane, column), in
// place.  A 1,024-thread workgroup takes 64 columns of one plane (lane =
// column, so every load and store is coalesced): in rounds of 256 chunks,
// wave w scans chunks 16w .. 16w+15 of the round in registers (all 16
// loads issued first), the 16 wave totals per column are combined through
// LDS, and a running total per column carries from round to round.
__global__ __launch_bounds__(1024) void k_dec_xy_carry(int* __restrict__ agg, int n0, int n2, int nyc)
{
    __shared__ int s_tot[16][64];
    __shared__ int s_run[64];
    const int l = lane_id(), w = threadIdx.x >> 6;
    const long long ncb = (n0 + 63) / 64;
    const long long z = blockIdx.x / ncb;
    const int c = (int)(blockIdx.x % ncb) * 64 + l;
    const bool act = c < n0 && z < n2;
    int* col = agg + z * (long long)nyc * n0 + (act ? c : 0);
    if (w == 0) s_run[l] = 0;
    for (int r0 = 0; r0 < nyc; r0 += 256) {
        const int j0 = r0 + 16 * w;
        int t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) t[u] = (act && j0 + u < nyc) ? col[(long long)(j0 + u) * n0] : 0;
        int sum = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int v = t[u];
            t[u] = sum;
            sum += v;
        }
        s_tot[w][l] = sum;
        __syncthreads();                            // also orders the first round after s_run's clearing
        int off = s_run[l];
        for (int v = 0; v < w; ++v) off += s_tot[v][l];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (act && j0 + u < nyc) col[(long long)(j0 + u) * n0] = off + t[u];
        __syncthreads();                            // every wave has read s_run and s_tot
        if (w == 15) s_run[l] = off + sum;          // wave 15's offset plus its total: the round's end
        __syncthreads();
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
    excl_prefix_strided(aggz, pos, nxy, nzc);
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

// ---------------------------------------------------------------------------
// 3-D decode on quads of x (n0 <= 1024; when n0 is not a multiple of 4 each
// row ends in a partial quad, and the workspace rows are padded to a
// multiple of 4 so that its 16-byte accesses stay aligned).  Tiles are
// (x range) x (MC_DY rows of row chunk j) x (MC_DZ planes of plane chunk k);
// lanes own four consecutive x (8-byte code loads, 16-byte stores) and
// issue all loads of a sweep before using any.  With d the errors, the
// inclusive prefix p splits at the tile's first row Y0 and first plane Z0:
//   p(x,y,z) = sum_{x' <= x} A(x',y,z),
//   A(x,y,z) = E(x) + sum_{Z0<=z'<=z} Fy(x,z') + sum_{Y0<=y'<=y} R(x,y',z),
//   R(x,y,z) = Fz(x,y) + sum_{Z0<=z'<=z} d(x,y,z'),
// with Fz(x,y) = sum_{z'<Z0} d(x,y,z'), Fy(x,z) = sum_{y'<Y0} d(x,y',z) and
// E(x) = sum_{y'<Y0, z'<Z0} d(x,y',z').  Three launches:
//   k_d3_tot    per tile (256-column segment): the tile's z sums per (x,y)
//               (agg_z), y sums per (x,z) (agg_y, through LDS) and its
//               total per x (agg_t)
//   k_d3_carry  exclusive prefixes: agg_z over plane chunks (-> Fz), agg_y
//               over row chunks (-> Fy), agg_t over both (-> E)
//   k_d3_apply  per tile, whole rows: R by a running sum over the planes,
//               the y prefix across the four waves through LDS (the lead
//               wave adds E + Fy), the x scan of every row, x1' written
// Integer sums wrap as in two's complement; p itself fits in 32 bits, so
// the wrapped partial sums still add up to it.
#define MC_DZ MC_DZ_PLANES
#define MC_DY MC_DY_ROWS
static_assert(MC_DY == 8, "3-D quad decode: 4 waves x 2 rows");
static_assert(MC_DZ % 4 == 0, "3-D quad decode: planes prefetched in quarters");

// Codes of the quad at node j (x, x+1, x+2, x+3 of one row).  AL: the row
// length is a multiple of 4 (one 8-byte load); otherwise `left` = n0 - x
// elements remain in the row and those past its end read as the neutral
// code R (error 0).
template <bool AL>
__device__ __forceinline__ ushort4 ld_codes4(const uint16_t* __restrict__ codes, unsigned j, bool act, unsigned left)
{
    if (!act) return make_ushort4(0, 0, 0, 0);
    if (AL) return *reinterpret_cast<const ushort4*>(codes + j);
    const unsigned short R = (unsigned short)MC_R;
    return make_ushort4(codes[j], left > 1u ? codes[j + 1] : R, left > 2u ? codes[j + 2] : R,
                        left > 3u ? codes[j + 3] : R);
}

// Outliers of the 16 (plane, row) runs of a wave.  Run r covers node
// indices [s_r, e_r); lane r < 16 returns the first outlier position with
// index >= s_r and lane 16 + r that with index >= e_r (the list ascends),
// so a zero code of run r searches positions [lo_r, hi_r) only.  Every lane
// passes its run's bounds for run (lane & 15).
__device__ __forceinline__ int run_bound(const int32_t* __restrict__ oidx, long long nout, long long s, long long e,
                                         bool valid)
{
    const int l = lane_id();
    if (nout == 0 || l >= 32 || !valid) return 0;
    const long long key = l < 16 ? s : e;
    long long lo = 0, hi = nout;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if ((long long)oidx[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (int)lo;
}

// Error of one node of run r: its code, or its entry among the run's
// outliers (positions [lo, hi), read from lanes r and 16 + r of `bounds`).
__device__ __forceinline__ int dec1r(unsigned c, const int32_t* __restrict__ oidx,
                                     const int32_t* __restrict__ odelta, int lo, int hi, unsigned j)
{
    if (c != 0u) return (int)c - MC_R;
    int a = lo, b = hi;
    while (a < b) {
        const int mid = (a + b) >> 1;
        if ((unsigned)oidx[mid] < j) a = mid + 1;
        else b = mid;
    }
    return (a < hi && (unsigned)oidx[a] == j) ? odelta[a] : 0;
}

__device__ __forceinline__ int4 dec4r(ushort4 c, const int32_t* __restrict__ oidx,
                                      const int32_t* __restrict__ odelta, int bounds, int r, unsigned j)
{
    const int lo = __builtin_amdgcn_readlane(bounds, r), hi = __builtin_amdgcn_readlane(bounds, 16 + r);
    if ((c.x != 0u) & (c.y != 0u) & (c.z != 0u) & (c.w != 0u))
        return make_int4((int)c.x - MC_R, (int)c.y - MC_R, (int)c.z - MC_R, (int)c.w - MC_R);
    return make_int4(dec1r(c.x, oidx, odelta, lo, hi, j), dec1r(c.y, oidx, odelta, lo, hi, j + 1),
                     dec1r(c.z, oidx, odelta, lo, hi, j + 2), dec1r(c.w, oidx, odelta, lo, hi, j + 3));
}

__device__ __forceinline__ int4 add4(int4 a, int4 b)
{
    return make_int4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

template <bool AL>
__global__ __launch_bounds__(256) void k_d3_tot(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                const int32_t* __restrict__ odelta, const mc_result* __restrict__ res,
                                                long long gcap, int n0, int n0p, int n1, int n2, int nxs, int nyc,
                                                int nzc, int* __restrict__ agg_z, int* __restrict__ agg_y,
                                                int* __restrict__ agg_t, unsigned remap)
{
    // per plane (then the tile total) and per wave; the planes in two
    // rounds of MC_DZ / 2, so the buffer is half the tile (20 KB: more
    // workgroups per CU)
    constexpr int HZ = MC_DZ / 2;
    static_assert(MC_DZ % 2 == 0, "two rounds of planes");
    __shared__ int4 s_p[HZ + 1][4][64];
    const unsigned t = tile_of(remap);                           // grid = exactly the tiles: no early exit
    const unsigned xs = t % (unsigned)nxs, r = t / (unsigned)nxs;
    const unsigned yc = r % (unsigned)nyc, zc = r / (unsigned)nyc;
    const int w = threadIdx.x >> 6, lane = lane_id();
    const unsigned x = xs * 256u + 4u * (unsigned)lane;
    const bool actx = x < (unsigned)n0;
    const unsigned nxy = (unsigned)n0 * (unsigned)n1, nxyp = (unsigned)n0p * (unsigned)n1;
    const unsigned left = (unsigned)n0 - x;
    const int z0 = (int)zc * MC_DZ, z1 = min(z0 + MC_DZ, n2);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    unsigned rb[2], rp[2];                                       // code index, workspace index of the row
    bool ar[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const unsigned y = yc * MC_DY + 2u * (unsigned)w + (unsigned)q;
        ar[q] = actx && y < (unsigned)n1;
        rb[q] = x + (unsigned)n0 * y;
        rp[q] = x + (unsigned)n0p * y;
    }
    ushort4 c[MC_DZ][2];
#pragma unroll
    for (int k = 0; k < MC_DZ; ++k)
#pragma unroll
        for (int q = 0; q < 2; ++q)
            c[k][q] = ld_codes4<AL>(codes, rb[q] + nxy * (unsigned)(z0 + k), ar[q] && z0 + k < z1, left);
    int bnd;
    {
        const int r = lane & 15, zr = z0 + (r >> 1);
        const unsigned yr = yc * MC_DY + 2u * (unsigned)w + (unsigned)(r & 1);
        const long long s0 = (long long)nxy * zr + (long long)n0 * yr + xs * 256u;
        bnd = run_bound(oidx, nout, s0, s0 + min(256, n0 - (int)xs * 256), yr < (unsigned)n1 && zr < z1);
    }
    int4 sz[2] = {make_int4(0, 0, 0, 0), make_int4(0, 0, 0, 0)};
    int4 cs[MC_DZ];
#pragma unroll
    for (int k = 0; k < MC_DZ; ++k) {
        cs[k] = make_int4(0, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (ar[q] && z0 + k < z1) {
                const int4 d = dec4r(c[k][q], oidx, odelta, bnd, 2 * k + q, rb[q] + nxy * (unsigned)(z0 + k));
                sz[q] = add4(sz[q], d);
                cs[k] = add4(cs[k], d);
            }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
        if (ar[q]) *reinterpret_cast<int4*>(agg_z + (size_t)zc * nxyp + rp[q]) = sz[q];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h) __syncthreads();                                  // the first round's reads are done
#pragma unroll
        for (int k = 0; k < HZ; ++k) s_p[k][w][lane] = cs[h * HZ + k];
        if (h) s_p[HZ][w][lane] = add4(sz[0], sz[1]);
        __syncthreads();
        for (int k = w; k < HZ + h; k += 4) {
            if (!actx) continue;
            int4 a = s_p[k][0][lane];
#pragma unroll
            for (int v = 1; v < 4; ++v) a = add4(a, s_p[k][v][lane]);
            if (k < HZ) {
                const int zk = z0 + h * HZ + k;
                if (zk < z1) *reinterpret_cast<int4*>(agg_y + ((size_t)zk * nyc + yc) * n0p + x) = a;
            } else {
                *reinterpret_cast<int4*>(agg_t + ((size_t)yc * nzc + zc) * n0p + x) = a;
            }
        }
    }
}

// Exclusive prefix of a[0], a[stride], ... a[(n-1) stride] in place, B
// values loaded before any is used (32-bit offsets: every workspace array
// holds fewer than 2^32 entries).
template <int B>
__device__ __forceinline__ void excl_prefix_b(int* __restrict__ a, unsigned stride, int n)
{
    int run = 0;
    for (int b = 0; b < n; b += B) {
        int t[B];
#pragma unroll
        for (int u = 0; u < B; ++u) t[u] = a[(unsigned)min(b + u, n - 1) * stride];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (b + u < n) a[(unsigned)(b + u) * stride] = run;
            run += b + u < n ? t[u] : 0;
        }
    }
}

// Blocks [0, nbt): agg_t, 2^xb_log x per block, the rest of the block's
// threads per x taking the row chunks (pass 1, prefix over plane chunks)
// and then the plane chunks (pass 2, prefix over row chunks) -- the longest
// dependent chain, so dispatched first; [nbt, nbt + nbz): agg_z, one
// position each; the rest: agg_y, one (x, plane) each.  Pass 2 reads what
// other waves of the block wrote in pass 1, after the block barrier (which
// makes a block's global stores visible to the whole block).
__global__ __launch_bounds__(256, 3) void k_d3_carry(int* __restrict__ agg_z, int* __restrict__ agg_y,
                                                     int* __restrict__ agg_t, long long nxy, int n0, int n2, int nyc,
                                                     int nzc, unsigned nbt, unsigned nbz, int xb_log)
{
    const unsigned b = blockIdx.x;
    if (b >= nbt + nbz) {
        const long long i = (long long)(b - nbt - nbz) * 256 + threadIdx.x;
        if (i < (long long)n0 * n2) {
            const long long z = i / n0, c = i % n0;
            excl_prefix_b<32>(agg_y + z * nyc * n0 + c, (unsigned)n0, nyc);
        }
        return;
    }
    if (b >= nbt) {
        const long long pos = (long long)(b - nbt) * 256 + threadIdx.x;
        if (pos < nxy) excl_prefix_b<32>(agg_z + pos, (unsigned)nxy, nzc);
        return;
    }
    const int x = (int)(b << xb_log) + (int)(threadIdx.x & ((1u << xb_log) - 1u));
    const int sl = (int)(threadIdx.x >> xb_log), nsl = 256 >> xb_log;
    const bool act = x < n0;
    if (act)
        for (int j = sl; j < nyc; j += nsl)
            excl_prefix_b<32>(agg_t + (long long)j * nzc * n0 + x, (unsigned)n0, nzc);
    __syncthreads();
    if (act)
        for (int k = sl; k < nzc; k += nsl)
            excl_prefix_b<32>(agg_t + (long long)k * n0 + x, (unsigned)nzc * (unsigned)n0, nyc);
}

// Workgroup = one (row chunk, plane chunk) tile over all x: 4 waves x 2
// rows, NXS 256-column segments per row.  Codes of PF planes are loaded
// before any is used.
template <int NXS, bool AL>
__global__ __launch_bounds__(256, NXS == 1 ? 4 : 2) void k_d3_apply(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                  const int32_t* __restrict__ odelta,
                                                  const mc_result* __restrict__ res, long long gcap, int n0, int n0p,
                                                  int n1, int n2, int nyc, int nzc, const int* __restrict__ agg_z,
                                                  const int* __restrict__ agg_y, const int* __restrict__ agg_t,
                                                  float* __restrict__ xh, unsigned remap)
{
    constexpr int PF = NXS == 1 ? MC_DZ : (NXS == 2 ? MC_DZ / 2 : MC_DZ / 4);
    __shared__ int4 s_cs[2][4][NXS][64];
    const unsigned t = tile_of(remap);                           // grid = exactly the tiles: no early exit
    const unsigned yc = t % (unsigned)nyc, zc = t / (unsigned)nyc;
    const int w = threadIdx.x >> 6, lane = lane_id();
    const bool lead = w == 0;
    const unsigned nxy = (unsigned)n0 * (unsigned)n1, nxyp = (unsigned)n0p * (unsigned)n1;
    const int z0 = (int)zc * MC_DZ, z1 = min(z0 + MC_DZ, n2);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const double c = res->c, step1 = 2.0 * res->tau1;
    unsigned xq[NXS];
    bool ax[NXS];
#pragma unroll
    for (int sg = 0; sg < NXS; ++sg) {
        xq[sg] = (unsigned)sg * 256u + 4u * (unsigned)lane;
        ax[sg] = xq[sg] < (unsigned)n0;
    }
    unsigned yb[2], ybp[2];                                      // row start: codes and x1', workspace
    bool ar[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const unsigned y = yc * MC_DY + 2u * (unsigned)w + (unsigned)q;
        ar[q] = y < (unsigned)n1;
        yb[q] = (unsigned)n0 * y;
        ybp[q] = (unsigned)n0p * y;
    }
    int bnd;
    {
        const int r = lane & 15, zr = z0 + (r >> 1);
        const unsigned yr = yc * MC_DY + 2u * (unsigned)w + (unsigned)(r & 1);
        const long long s0 = (long long)nxy * zr + (long long)n0 * yr;
        bnd = run_bound(oidx, nout, s0, s0 + n0, yr < (unsigned)n1 && zr < z1);
    }
    int4 run[2][NXS], own[NXS];
#pragma unroll
    for (int sg = 0; sg < NXS; ++sg) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
            run[q][sg] = (ar[q] && ax[sg]) ? *reinterpret_cast<const int4*>(agg_z + (size_t)zc * nxyp + ybp[q] + xq[sg])
                                           : make_int4(0, 0, 0, 0);
        own[sg] = (lead && ax[sg]) ? *reinterpret_cast<const int4*>(agg_t + ((size_t)yc * nzc + zc) * n0p + xq[sg])
                                   : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int k0 = 0; k0 < MC_DZ; k0 += PF) {
        if (z0 + k0 >= z1) break;                                // uniform over the workgroup
        ushort4 cc[PF][2][NXS];
        int4 fy[PF][NXS];
#pragma unroll
        for (int kk = 0; kk < PF; ++kk) {
            const int z = z0 + k0 + kk;
#pragma unroll
            for (int sg = 0; sg < NXS; ++sg) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    cc[kk][q][sg] = ld_codes4<AL>(codes, nxy * (unsigned)z + yb[q] + xq[sg], ar[q] && ax[sg] && z < z1,
                                                  (unsigned)n0 - xq[sg]);
                fy[kk][sg] = (lead && ax[sg] && z < z1)
                                 ? *reinterpret_cast<const int4*>(agg_y + ((size_t)z * nyc + yc) * n0p + xq[sg])
                                 : make_int4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int kk = 0; kk < PF; ++kk) {
            const int k = k0 + kk, z = z0 + k;
            if (z >= z1) break;                                  // uniform over the workgroup
#pragma unroll
            for (int sg = 0; sg < NXS; ++sg) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    if (ar[q] && ax[sg])
                        run[q][sg] = add4(run[q][sg], dec4r(cc[kk][q][sg], oidx, odelta, bnd, 2 * k + q,
                                                            nxy * (unsigned)z + yb[q] + xq[sg]));
                own[sg] = add4(own[sg], fy[kk][sg]);
                s_cs[k & 1][w][sg][lane] = add4(own[sg], add4(run[0][sg], run[1][sg]));
            }
            __syncthreads();
            int rowoff[2] = {0, 0};
#pragma unroll
            for (int sg = 0; sg < NXS; ++sg) {
                int4 a = own[sg];
                for (int v = 0; v < w; ++v) a = add4(a, s_cs[k & 1][v][sg][lane]);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    a = add4(a, run[q][sg]);
                    const int a0 = a.x, a1 = a0 + a.y, a2 = a1 + a.z, a3 = a2 + a.w;
                    const int inc = wave_incl_scan(a3);
                    const int off = rowoff[q] + inc - a3;
                    rowoff[q] += __shfl(inc, 63, 64);
                    if (ar[q] && ax[sg]) {
                        float4 o;
                        o.x = xhat_of(off + a0, c, step1);
                        o.y = xhat_of(off + a1, c, step1);
                        o.z = xhat_of(off + a2, c, step1);
                        o.w = xhat_of(off + a3, c, step1);
                        float* dst = xh + nxy * (unsigned)z + yb[q] + xq[sg];
                        if (AL) {
                            *reinterpret_cast<float4*>(dst) = o;
                        } else {
                            const unsigned left = (unsigned)n0 - xq[sg];
                            dst[0] = o.x;
                            if (left > 1u) dst[1] = o.y;
                            if (left > 2u) dst[2] = o.z;
                            if (left > 3u) dst[3] = o.w;
                        }
                    }
                }
            }
        }
    }
}

// VPT vertices per thread (tile of 256 VPT), every load issued before use.
template <typename T, int D, bool NT, int VPT = MC_IPT>
__device__ __forceinline__ void vdecode_block(long long tile, const float* __restrict__ coords, long long nv,
                                              const GridGeom& gg, const float* __restrict__ xh,
                                              const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                              const T* __restrict__ oval, const mc_result* __restrict__ res,
                                              long long vcap, T* __restrict__ xout)
{
    long long v[VPT];
    bool act[VPT];
    int code[VPT];
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        v[i] = tile * (VPT * MC_WG) + i * MC_WG + threadIdx.x;
        act[i] = v[i] < nv;
        code[i] = ld_s<NT>(codes + (act[i] ? v[i] : 0));
    }
    float g[VPT];
    back_interp_n<D, VPT, false, NT>(coords, nv, gg, xh, 0.0, 0.0, v, act, g);
    const double step2 = 2.0 * res->tau2;
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        if (!act[i]) continue;
        if (code[i] == 0) {
            const long long n = res->n_vertex_outliers < vcap ? res->n_vertex_outliers : vcap;
            const long long k = find_outlier(oidx, n, v[i]);
            st_s<NT>(xout + v[i], k >= 0 ? oval[k] : (T)0);
        } else {
            const int q = code[i] - MC_R;
            st_s<NT>(xout + v[i], (T)((double)g[i] + (double)q * step2));
        }
    }
}

template <typename T, int D, bool NT, int VPT>
__global__ __launch_bounds__(256) void k_vdecode(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                 const float* __restrict__ xh, const uint16_t* __restrict__ codes,
                                                 const int32_t* __restrict__ oidx, const T* __restrict__ oval,
                                                 const mc_result* __restrict__ res, long long vcap,
                                                 T* __restrict__ xout, unsigned remap)
{
    vdecode_block<T, D, NT, VPT>(tile_of(remap), coords, nv, gg, xh, codes, oidx, oval, res, vcap, xout);
}

// Batched vertex decode: one launch over the tiles of every field (see the
// batched compress stages in k_compress.hip), plain codes.
template <typename T, int D>
__device__ __forceinline__ void b_vdecode(const mck::BItemD* it, unsigned t)
{
    if (it->knobs & mck::MC_KNOB_NT_VERT)
        vdecode_block<T, D, true>(t, it->coords, it->nv, it->gg, it->xh, it->vcodes, it->vidx,
                                  (const T*)it->vval, it->res, it->vcap, (T*)it->xout);
    else
        vdecode_block<T, D, false>(t, it->coords, it->nv, it->gg, it->xh, it->vcodes, it->vidx,
                                   (const T*)it->vval, it->res, it->vcap, (T*)it->xout);
}

__global__ __launch_bounds__(256) void k_b_vdecode(const mck::BItemD* __restrict__ items,
                                                   const unsigned* __restrict__ base, int n)
{
    const int i = item_of(base, n, blockIdx.x);
    const mck::BItemD* it = items + i;
    const unsigned t = blockIdx.x - base[i];
    switch (it->cls) {
    case 0: b_vdecode<float, 2>(it, t); break;
    case 1: b_vdecode<float, 3>(it, t); break;
    case 2: b_vdecode<double, 2>(it, t); break;
    default: b_vdecode<double, 3>(it, t); break;
    }
}

// ---------------------------------------------------------------------------
// 2-D decode on row segments.  A wave owns a segment of 256 columns (lane l:
// columns 256 sg + l + 64 k, k < 4, so every load and store is coalesced)
// and a chunk of MC_D2_R rows; with Y(x, y) the column prefix of the
// errors (the difference of the decoded grid along x) and S(y, sg) its sum
// over a segment,
//   k_d2_tot    per (segment, chunk): the chunk's column totals of the errors
//   (k_dec_xy_carry: exclusive prefix over the chunks, in place)
//   k_d2_rowsum per (segment, chunk): Y from the carries, S written per row
//   k_d2_apply  per (segment, chunk): Y again, its prefix along the segment
//               (four wave scans) plus the S of the segments to the left:
//               the decoded grid, x1' written
// Rows of at most 16 segments take k_d2_apply_rows after the carries
// instead of the last two (the segment sums exchanged in LDS).
// Every partial sum is a difference of two decoded values, so int32 holds it.
__device__ __forceinline__ void d2_unit(int unit, int nseg, int n0, int n1, int& sg, int& y0, int& y1)
{
    sg = unit % nseg;
    y0 = (unit / nseg) * MC_D2_R;
    y1 = min(n1, y0 + MC_D2_R);
}

// The errors of rows y0 .. y0 + MC_D2_R - 1 (past n1 and past n0: 0) at the
// lane's four columns, every code load issued before any is used.
__device__ __forceinline__ void d2_errors(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                          const int32_t* __restrict__ odelta, long long nout, int n0, int n1, int x0,
                                          int y0, int y1, int (&e)[MC_D2_R][4])
{
    const int l = lane_id();
#pragma unroll
    for (int r = 0; r < MC_D2_R; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = min(x0 + l + 64 * k, n0 - 1), y = min(y0 + r, n1 - 1);
            e[r][k] = codes[(long long)y * n0 + x];
        }
#pragma unroll
    for (int r = 0; r < MC_D2_R; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = x0 + l + 64 * k, y = y0 + r;
            int d = e[r][k] - MC_R;
            if (e[r][k] == 0) {
                const long long o = find_outlier(oidx, nout, (long long)min(y, n1 - 1) * n0 + min(x, n0 - 1));
                d = o >= 0 ? odelta[o] : 0;
            }
            e[r][k] = (x < n0 && y < y1) ? d : 0;
        }
}

__global__ __launch_bounds__(256) void k_d2_tot(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                const int32_t* __restrict__ odelta, const mc_result* __restrict__ res,
                                                long long gcap, int n0, int n1, int nseg, int nunits,
                                                int* __restrict__ agg)
{
    const int unit = (int)xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (unit >= nunits) return;
    int sg, y0, y1;
    d2_unit(unit, nseg, n0, n1, sg, y0, y1);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    int e[MC_D2_R][4];
    d2_errors(codes, oidx, odelta, nout, n0, n1, sg * 256, y0, y1, e);
    const long long row = (long long)(unit / nseg) * n0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int t = 0;
#pragma unroll
        for (int r = 0; r < MC_D2_R; ++r) t += e[r][k];
        const int x = sg * 256 + lane_id() + 64 * k;
        if (x < n0) agg[row + x] = t;
    }
}

__global__ __launch_bounds__(256) void k_d2_rowsum(const uint16_t* __restrict__ codes,
                                                   const int32_t* __restrict__ oidx,
                                                   const int32_t* __restrict__ odelta,
                                                   const mc_result* __restrict__ res, long long gcap, int n0, int n1,
                                                   int nseg, int nunits, const int* __restrict__ carry,
                                                   int* __restrict__ segsum)
{
    const int unit = (int)xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (unit >= nunits) return;
    int sg, y0, y1;
    d2_unit(unit, nseg, n0, n1, sg, y0, y1);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const long long row = (long long)(unit / nseg) * n0;
    int col[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = sg * 256 + lane_id() + 64 * k;
        col[k] = x < n0 ? carry[row + x] : 0;
    }
    int e[MC_D2_R][4];
    d2_errors(codes, oidx, odelta, nout, n0, n1, sg * 256, y0, y1, e);
#pragma unroll
    for (int r = 0; r < MC_D2_R; ++r) {
        int t = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            col[k] += e[r][k];
            t += col[k];
        }
        t = wave_sum(t);
        if (lane_id() == 0 && y0 + r < y1) segsum[(long long)(y0 + r) * nseg + sg] = t;
    }
}

__global__ __launch_bounds__(256) void k_d2_apply(const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
                                                  const int32_t* __restrict__ odelta,
                                                  const mc_result* __restrict__ res, long long gcap, int n0, int n1,
                                                  int nseg, int nunits, const int* __restrict__ carry,
                                                  const int* __restrict__ segsum, float* __restrict__ xh)
{
    const int unit = (int)xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (unit >= nunits) return;
    int sg, y0, y1;
    d2_unit(unit, nseg, n0, n1, sg, y0, y1);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const double c = res->c, step1 = 2.0 * res->tau1;
    const long long row = (long long)(unit / nseg) * n0;
    const int l = lane_id();
    int col[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = sg * 256 + l + 64 * k;
        col[k] = x < n0 ? carry[row + x] : 0;
    }
    // the segment sums to the left of this one, per row (nseg <= 32 lanes)
    int left[MC_D2_R];
#pragma unroll
    for (int r = 0; r < MC_D2_R; ++r)
        left[r] = (l < sg && y0 + r < y1) ? segsum[(long long)(y0 + r) * nseg + l] : 0;
    int e[MC_D2_R][4];
    d2_errors(codes, oidx, odelta, nout, n0, n1, sg * 256, y0, y1, e);
#pragma unroll
    for (int r = 0; r < MC_D2_R; ++r) {
        if (y0 + r >= y1) break;                         // uniform across the wave
        int run = wave_sum(left[r]);
        const long long base = (long long)(y0 + r) * n0 + sg * 256 + l;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            col[k] += e[r][k];
            const int inc = wave_incl_scan(col[k]);
            if (sg * 256 + l + 64 * k < n0) xh[base + 64 * k] = xhat_of(run + inc, c, step1);
            run += __shfl(inc, 63, 64);
        }
    }
}

// Rows of at most MC_D2_SEG_MAX segments: one workgroup per chunk of rows,
// one wave per segment.  After the carries each wave has Y on its segment;
// the per-row segment sums meet in LDS, so the apply needs no separate pass
// for them (k_d2_rowsum) and reads the codes once more instead of twice.
#define MC_D2_SEG_MAX 16
__global__ __launch_bounds__(64 * MC_D2_SEG_MAX) void k_d2_apply_rows(
    const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx, const int32_t* __restrict__ odelta,
    const mc_result* __restrict__ res, long long gcap, int n0, int n1, const int* __restrict__ carry,
    float* __restrict__ xh)
{
    __shared__ int s_sum[MC_D2_R][MC_D2_SEG_MAX];
    const int sg = threadIdx.x >> 6, l = lane_id();
    const int ch = (int)xcd_tile(blockIdx.x, gridDim.x);
    const int y0 = ch * MC_D2_R, y1 = min(n1, y0 + MC_D2_R);
    const long long nout = res->n_grid_outliers < gcap ? res->n_grid_outliers : gcap;
    const double c = res->c, step1 = 2.0 * res->tau1;
    const long long row = (long long)ch * n0;
    int col[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = sg * 256 + l + 64 * k;
        col[k] = x < n0 ? carry[row + x] : 0;
    }
    int e[MC_D2_R][4];
    d2_errors(codes, oidx, odelta, nout, n0, n1, sg * 256, y0, y1, e);
    {
        int cy[4] = {col[0], col[1], col[2], col[3]};
#pragma unroll
        for (int r = 0; r < MC_D2_R; ++r) {
            int t = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                cy[k] += e[r][k];
                t += cy[k];
            }
            t = wave_sum(t);
            if (l == 0) s_sum[r][sg] = t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < MC_D2_R; ++r) {
        if (y0 + r >= y1) break;                         // uniform across the workgroup
        int run = wave_sum(l < sg ? s_sum[r][l] : 0);
        const long long base = (long long)(y0 + r) * n0 + sg * 256 + l;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            col[k] += e[r][k];
            const int inc = wave_incl_scan(col[k]);
            if (sg * 256 + l + 64 * k < n0) xh[base + 64 * k] = xhat_of(run + inc, c, step1);
            run += __shfl(inc, 63, 64);
        }
    }
}

namespace mck {

hipError_t grid_decode(const uint16_t* codes, const int32_t* oidx, const int32_t* odelta, long long gcap,
                       const mc_result* res, int dim, int n0, int n1, int n2, int32_t* pz, float* xh, DecodeWs& ws,
                       unsigned remap, hipStream_t s)
{
    hipError_t e;
    const int cpt = (n0 + 63) / 64;
    const unsigned nb_xy = (unsigned)((ws.ntiles_xy + 3) / 4);
    if (dim == 2) {
        const int nseg = (n0 + 255) / 256, nunits = nseg * ws.nyc;
        const dim3 g((unsigned)((nunits + 3) / 4));
        {
            ProfScope ps("k_dec_xy_tot", s);
            hipLaunchKernelGGL(k_d2_tot, g, dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, n1, nseg, nunits,
                               ws.agg_xy);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        {
            ProfScope ps("k_dec_xy_carry", s);
            hipLaunchKernelGGL(k_dec_xy_carry, dim3((unsigned)((n0 + 63) / 64)), dim3(1024), 0, s, ws.agg_xy, n0, 1,
                               ws.nyc);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (nseg <= MC_D2_SEG_MAX) {
            ProfScope ps("k_dec_xy_apply", s);
            hipLaunchKernelGGL(k_d2_apply_rows, dim3((unsigned)ws.nyc), dim3(64 * nseg), 0, s, codes, oidx, odelta,
                               res, gcap, n0, n1, ws.agg_xy, xh);
            return hipGetLastError();
        }
        {
            ProfScope ps("k_dec_xy_rowsum", s);
            hipLaunchKernelGGL(k_d2_rowsum, g, dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, n1, nseg, nunits,
                               ws.agg_xy, ws.segsum);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        ProfScope ps("k_dec_xy_apply", s);
        hipLaunchKernelGGL(k_d2_apply, g, dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, n1, nseg, nunits,
                           ws.agg_xy, ws.segsum, xh);
        return hipGetLastError();
    }
    if (ws.fast3) {
        const int n0p = ws.pitch;                                // workspace row pitch: n0 rounded up to 4
        const long long nxyp = (long long)n0p * n1;
        const int nxs = (n0 + 255) / 256;
        const bool al = n0 % 4 == 0;
        {
            ProfScope ps("k_dec3_tot", s);
            const unsigned ntiles = (unsigned)((long long)nxs * ws.nyc * ws.nzc);
            const unsigned rm = remap & MC_KNOB_DZTOT;
#define MC_D3T(A) hipLaunchKernelGGL(k_d3_tot<A>, dim3(ntiles), dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, n0p, \
                                     n1, n2, nxs, ws.nyc, ws.nzc, ws.agg_z, ws.agg_xy, ws.agg_t, rm)
            if (al) MC_D3T(true);
            else MC_D3T(false);
#undef MC_D3T
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        {
            ProfScope ps("k_dec3_carry", s);
            const unsigned nbz = (unsigned)((nxyp + 255) / 256), nby = (unsigned)(((long long)n0p * n2 + 255) / 256);
            const int mx = ws.nyc > ws.nzc ? ws.nyc : ws.nzc;   // longest run of the tile-total prefix
            int xb_log = 4;                                      // x per block: 256 / xb >= mx when it can be
            while (xb_log > 0 && (256 >> xb_log) < mx) --xb_log;
            const unsigned nbt = (unsigned)((n0p + (1 << xb_log) - 1) >> xb_log);
            hipLaunchKernelGGL(k_d3_carry, dim3(nbt + nbz + nby), dim3(256), 0, s, ws.agg_z, ws.agg_xy, ws.agg_t, nxyp,
                               n0p, n2, ws.nyc, ws.nzc, nbt, nbz, xb_log);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        {
            ProfScope ps("k_dec3_apply", s);
            const dim3 g((unsigned)((long long)ws.nyc * ws.nzc));
            const unsigned rm = remap & MC_KNOB_DZAPPLY;
#define MC_D3A(X, A) hipLaunchKernelGGL((k_d3_apply<X, A>), g, dim3(256), 0, s, codes, oidx, odelta, res, gcap, n0, \
                                        n0p, n1, n2, ws.nyc, ws.nzc, ws.agg_z, ws.agg_xy, ws.agg_t, xh, rm)
            if (nxs == 1) { if (al) MC_D3A(1, true); else MC_D3A(1, false); }
            else if (nxs == 2) { if (al) MC_D3A(2, true); else MC_D3A(2, false); }
            else { if (al) MC_D3A(4, true); else MC_D3A(4, false); }
#undef MC_D3A
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        return hipSuccess;
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
        hipLaunchKernelGGL(k_dec_xy_carry, dim3((unsigned)((long long)((n0 + 63) / 64) * n2)), dim3(1024), 0, s,
                           ws.agg_xy, n0, n2, ws.nyc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        ProfScope ps("k_dec_xy_apply", s);
#define MC_DXA(C, F) hipLaunchKernelGGL((k_dec_xy_apply<C, F>), dim3(nb_xy), dim3(256), 0, s, codes, oidx, odelta, pz, res, \
                                        gcap, n0, n1, ws.rows, ws.nyc, ws.ntiles_xy, ws.agg_xy, xh)
#define MC_DXA2(C) MC_DXA(C, false)
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

hipError_t batch_vdecode(const BItemD* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s)
{
    ProfScope ps("k_b_vdecode", s);
    hipLaunchKernelGGL(k_b_vdecode, dim3(nblocks), dim3(256), 0, s, items, base, n);
    return hipGetLastError();
}

hipError_t vertex_decode(const float* coords, long long nv, GridGeom gg, const float* xh, const uint16_t* codes,
                         const int32_t* oidx, const void* oval, long long vcap, const mc_result* res, void* xout,
                         int dtype, unsigned remap, hipStream_t s)
{
    const bool nt = (remap & MC_KNOB_NT_VERT) != 0;
    const int vpt = knob_vpt(remap);
    remap &= MC_KNOB_VDECODE;
    ProfScope ps("k_vdecode", s);
    const long long per = 256LL * vpt;
    dim3 grid((unsigned)((nv + per - 1) / per));
#define MC_VD0(T, D, NT, V) hipLaunchKernelGGL((k_vdecode<T, D, NT, V>), grid, dim3(256), 0, s, coords, nv, gg, xh, \
                                               codes, oidx, (const T*)oval, res, vcap, (T*)xout, remap)
#define MC_VD1(T, D, V) do { if (nt) MC_VD0(T, D, true, V); else MC_VD0(T, D, false, V); } while (0)
#define MC_VD(T, D) do { if (vpt == 2) MC_VD1(T, D, 2); else if (vpt == 8) MC_VD1(T, D, 8); else MC_VD1(T, D, 4); } \
                    while (0)
    if (dtype == MC_F64) { if (gg.dim == 2) MC_VD(double, 2); else MC_VD(double, 3); }
    else { if (gg.dim == 2) MC_VD(float, 2); else MC_VD(float, 3); }
#undef MC_VD
#undef MC_VD1
#undef MC_VD0
    return hipGetLastError();
}

}  // namespace mck
