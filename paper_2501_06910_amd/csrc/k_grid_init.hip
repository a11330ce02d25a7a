// k_grid_init.hip -- the grid initialisation of Alg. 1 on gfx950: the
// spacing of each axis is a percentile of the cells' edge extents along it.
// The percentile is an exact radix select over the FP32 bit patterns of the
// extents (non-negative floats order like their bits), computed on the fly
// from the cells and coordinates in three passes of 11, 11 and 10 bits:
// each pass histograms the extents whose higher bits match the prefix
// chosen so far (per-workgroup LDS histogram, flushed with 64-bit atomics).
#include "mc_dev.h"
#include "mc_kernels.h"

#define MC_GI_BINS 2048

template <int D>
__global__ __launch_bounds__(256) void k_edge_hist(const float* __restrict__ coords, const int32_t* __restrict__ cells,
                                                   long long nv, long long nc, int axis, unsigned shift,
                                                   unsigned nbits, unsigned pmask, unsigned pval,
                                                   unsigned long long* __restrict__ hist,
                                                   unsigned int* __restrict__ bad)
{
    constexpr int NE = D == 2 ? 3 : 6;
    __shared__ unsigned s_h[MC_GI_BINS];
    for (int i = threadIdx.x; i < MC_GI_BINS; i += 256) s_h[i] = 0u;
    __syncthreads();
    const unsigned bmask = (1u << nbits) - 1u;
    const float* __restrict__ c = coords + (long long)axis * nv;
    bool badv = false;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < nc; k += (long long)gridDim.x * 256) {
        int v[D + 1];
#pragma unroll
        for (int q = 0; q <= D; ++q) v[q] = cells[(long long)q * nc + k];
        bool ok = true;
#pragma unroll
        for (int q = 0; q <= D; ++q) ok = ok && v[q] >= 0 && (long long)v[q] < nv;
        if (!ok) {
            badv = true;
            continue;
        }
        float p[D + 1];
#pragma unroll
        for (int q = 0; q <= D; ++q) p[q] = c[v[q]];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            // edges (0,1) (0,2) [(0,3)] (1,2) [(1,3) (2,3)]
            const int a = D == 2 ? (e < 2 ? 0 : 1) : (e < 3 ? 0 : (e < 5 ? 1 : 2));
            const int b = D == 2 ? (e == 0 ? 1 : 2) : (e < 3 ? e + 1 : (e < 5 ? e - 1 : 3));
            const unsigned key = __float_as_uint(fabsf(p[a] - p[b]));
            if ((key & pmask) == pval) atomicAdd(&s_h[(key >> shift) & bmask], 1u);
        }
    }
    if (badv) atomicOr(bad, 1u);
    __syncthreads();
    for (int i = threadIdx.x; i <= (int)bmask; i += 256)
        if (s_h[i]) atomicAdd(&hist[i], (unsigned long long)s_h[i]);
}

namespace mck {

hipError_t edge_hist(const float* coords, const int32_t* cells, int dim, long long nv, long long nc, int axis,
                     unsigned shift, unsigned nbits, unsigned pmask, unsigned pval, unsigned long long* hist,
                     unsigned* bad, hipStream_t s)
{
    ProfScope ps("k_edge_hist", s);
    long long nb = (nc + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (dim == 2)
        hipLaunchKernelGGL(k_edge_hist<2>, dim3((unsigned)nb), dim3(256), 0, s, coords, cells, nv, nc, axis, shift,
                           nbits, pmask, pval, hist, bad);
    else
        hipLaunchKernelGGL(k_edge_hist<3>, dim3((unsigned)nb), dim3(256), 0, s, coords, cells, nv, nc, axis, shift,
                           nbits, pmask, pval, hist, bad);
    return hipGetLastError();
}

}  // namespace mck
