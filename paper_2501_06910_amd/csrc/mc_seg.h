// mc_seg.h -- segmented running sums on gfx950 wavefronts: an element is
// (f, v) = (restart here, value); combining a then b gives
// (a.f | b.f, b.f ? b.v : a.v + b.v), an associative operation with (0, 0)
// neutral, so a prefix over it rebuilds a running sum that restarts at
// every flagged element.
#pragma once
#include "mc_dev.h"

struct Seg {
    int f, v;
};

__device__ __forceinline__ Seg seg_op(Seg a, Seg b)
{
    return Seg{a.f | b.f, b.f ? b.v : a.v + b.v};
}

__device__ __forceinline__ Seg wave_seg_incl(Seg s)
{
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        Seg o;
        o.f = __shfl_up(s.f, d, 64);
        o.v = __shfl_up(s.v, d, 64);
        if (l >= d) s = seg_op(o, s);
    }
    return s;
}

// Workgroup-wide exclusive segmented scan of one Seg per thread (NW waves),
// started from `init`; *total receives init combined with every thread's.
template <int NW>
__device__ __forceinline__ Seg block_seg_excl(Seg s, Seg init, Seg* s_w, Seg* total)
{
    const int l = lane_id(), w = threadIdx.x >> 6;
    const Seg inc = wave_seg_incl(s);
    if (l == 63) s_w[w] = inc;
    __syncthreads();
    Seg pre = init, all = init;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const Seg a = s_w[k];
        if (k < w) pre = seg_op(pre, a);
        all = seg_op(all, a);
    }
    *total = all;
    Seg ex;
    ex.f = __shfl_up(inc.f, 1, 64);
    ex.v = __shfl_up(inc.v, 1, 64);
    if (l == 0) ex = Seg{0, 0};
    return seg_op(pre, ex);
}

