// mc_interp.h -- the multilevel interpolation and the time-axis grid
// predictors on the prequantised grid p (the SZ family's interpolation
// predictor, Sec. II; any grid compressor may stand in for C(x1),
// Sec. IV-D).  Shared by their encoders and decoders (k_interp.hip) and the
// outlier gather (k_compress.hip).
//
// With L the least integer such that 2^L >= n_d on every axis, the strides
// run s = 2^(L-1) .. 1.  The origin is predicted by 0; every other node
// belongs to the class (s, a) where s = 2^t, t the fewest trailing zero
// bits among its non-zero coordinates, and a the highest axis whose
// coordinate is non-zero with t trailing zeros (an odd multiple of s).  Its
// prediction interpolates along a from the nodes at -s and +s (and -3s,
// +3s for the cubic rule), all of them in classes decoded before it:
//   +s outside the grid:             p[-s]
//   cubic and -3s, +3s inside:       floor((-p[-3s] + 9 p[-s] + 9 p[+s] - p[+3s] + 8) / 16)
//   otherwise:                       floor((p[-s] + p[+s]) / 2)
// Decoding runs the origin, then the classes in the order s = 2^(L-1) .. 1
// and, within a stride, a = 0 .. D-1.  Integer arithmetic throughout.
#pragma once
#include <stdint.h>

// Trailing zeros of a non-zero coordinate, 31 for zero.
__device__ __forceinline__ int ip_tz(int v)
{
    return v ? __builtin_ctz((unsigned)v) : 31;
}

// log2 of the class stride (-1 for the origin) and the class axis.
__device__ __forceinline__ int ip_class(int i0, int i1, int i2, int& axis)
{
    const int t0 = ip_tz(i0), t1 = ip_tz(i1), t2 = ip_tz(i2);
    const int t = min(t0, min(t1, t2));
    axis = t2 == t ? 2 : (t1 == t ? 1 : 0);
    return t == 31 ? -1 : t;
}

// Prediction of the node at flat index j, coordinate x along its class axis
// (extent n), stride s, flat distance ds = s * (flat step along the axis);
// indices fit in int (fewer than 2^31 nodes), sums are taken in int64.
// All four neighbour loads are issued unconditionally and together (a
// neighbour a rule does not use reads the -s node again, which is always
// inside the grid) and the rule is chosen with bitwise masks, not selects,
// so that the compiler keeps the loads out of branches.  Without a +s
// neighbour b reads a, and floor((a + a) / 2) = a is that case's rule.
template <bool CUBIC>
__device__ __forceinline__ long long ip_predict(const int32_t* __restrict__ p, int j, int x, int n, int ds, int s)
{
    const bool hb = x + s <= n - 1;
    const bool h3 = CUBIC && x >= 3 * s && x + 3 * s <= n - 1;
    const int ia = j - ds;
    const long long a = p[ia];
    const long long b = p[hb ? j + ds : ia];
    const long long lin = (a + b) >> 1;
    if (!CUBIC) return lin;
    const long long a3 = p[h3 ? j - 3 * ds : ia];
    const long long b3 = p[h3 ? j + 3 * ds : ia];
    const long long cub = (9 * (a + b) - a3 - b3 + 8) >> 4;
    const long long m3 = -(long long)h3;
    return (cub & m3) | (lin & ~m3);
}

// Prediction error of node j from the fully known grid p (encoder side).
// The origin (prediction 0) takes the same loads at distance 0.
template <bool CUBIC>
__device__ __forceinline__ long long ip_delta(const int32_t* __restrict__ p, int j, int i0, int i1, int i2, int n0,
                                              int n1, int n2)
{
    int a;
    const int t = ip_class(i0, i1, i2, a);
    const bool org = t < 0;
    const int tt = org ? 0 : t;
    const int st = a == 0 ? 1 : (a == 1 ? n0 : n0 * n1);
    const int x = a == 0 ? i0 : (a == 1 ? i1 : i2), n = a == 0 ? n0 : (a == 1 ? n1 : n2);
    const long long self = p[j];
    const long long pred = ip_predict<CUBIC>(p, j, x, n, org ? 0 : st << tt, 1 << tt);
    return self - (org ? 0ll : pred);
}

// Time-axis prediction of a node from its reference grid value r (the
// previous timestep's x1'): rint((r - c) * inv1) when that is below 2^27 in
// magnitude, else 0 (a non-finite r included).
__device__ __forceinline__ long long tp_pred(float r, double c, double inv1)
{
    const double s = ((double)r - c) * inv1;
    return fabs(s) < 134217728.0 ? (long long)rint(s) : 0ll;
}
