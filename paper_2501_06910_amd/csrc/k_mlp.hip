// k_mlp.hip -- learned residual predictor on gfx950 matrix cores.
//
// Network: in -> 64 -> 64 -> 64 -> 1, ReLU; weights BF16, accumulation
// FP32, hidden activations re-rounded to BF16 after bias and ReLU.  Inputs
// of a vertex: bf16((x1'[n] - g) * kappa) for the 4^D grid nodes around its
// grid cell (indices clamped), then bf16(t_d - 0.5), zero padded to KPAD.
//
// Layout.  A wave owns 64 vertices (4 column blocks of 16).  Every layer is
// computed transposed, H^T = W . X^T, with v_mfma_f32_16x16x16_bf16: A = a
// 16x16 block of W (from LDS), B = 16 vertices x 16 inputs.  The output
// fragment of one layer (lane l holds rows 4(l/16)..+3 of column l%16) is
// exactly the B fragment the next layer needs, so activations never leave
// registers in the forward pass.  Input fragments are built directly in that
// layout: lane l computes inputs 4(l/16)+16kb+i of vertex l%16 of each block.
//
// Training (one step): each wave takes 64 samples drawn with SplitMix64,
// runs the forward pass, then backward: dZ = dH * [h > 0]; weight gradients
// dW = dZ^T . H need both operands transposed, so dZ^T and H^T are staged in
// LDS ([unit][sample], BF16) and read back as fragments; input gradients
// dH = W^T . dZ use a transposed weight copy in LDS.  Each wave writes its
// whole gradient to its own slot; a second kernel sums the slots in a fixed
// order (deterministic) and applies Adam.
#include "mc_dev.h"
#include "mc_kernels.h"

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define HID 64

__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u = u + 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ float bfround(float f) { return bf2f(f2bf(f)); }

// Four floats to BF16 (round to nearest even) with the hardware's packed
// conversion (v_cvt_pk_bf16_f32); the same rounding as f2bf on every
// finite value.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d)
{
    const bf16x2_t lo = __builtin_convertvector((f32x2_t){a, b}, bf16x2_t);
    const bf16x2_t hi = __builtin_convertvector((f32x2_t){c, d}, bf16x2_t);
    const unsigned ul = __builtin_bit_cast(unsigned, lo), uh = __builtin_bit_cast(unsigned, hi);
    bf16x4 r;
    r[0] = (short)(ul & 0xffffu);
    r[1] = (short)(ul >> 16);
    r[2] = (short)(uh & 0xffffu);
    r[3] = (short)(uh >> 16);
    return r;
}

// ReLU of four BF16 values as packed signed 16-bit maxima with zero
// (v_pk_max_i16, two values per instruction): a BF16 value is negative
// exactly when its sign bit is set, i.e. when it is negative as an int16, so
// max(v, 0) keeps positive values and gives +0 for the rest.  Rounding and
// ReLU commute (rounding keeps the sign; -0 and +0 both become +0), so
// relu_bf(pack4(x)) equals pack4(relu(x)) for every value that is not a NaN.
__device__ __forceinline__ bf16x4 relu_bf(bf16x4 v)
{
    return __builtin_elementwise_max(v, (bf16x4){0, 0, 0, 0});
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// K = 32 products per instruction (gfx950).  Each lane supplies 8 values of
// A and 8 of B; the instruction pairs A's and B's values of the same lane
// group and slot, so any assignment of the 32 k indices to (lane group,
// slot) gives the full sum as long as A and B use the same one.  Here slot
// i < 4 of lane group g is k = 4g + i of the first 16-block and slot 4 + i
// the same of the second: the B operand is then just two 16-wide fragments
// side by side (the output of the 16-row MFMA layout), and the weights are
// stored in that order.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x8 cat8(bf16x4 a, bf16x4 b)
{
    typedef short s8 __attribute__((ext_vector_type(8)));
    const s8 v = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int D> struct MlpShape {
    static constexpr int NN = D == 2 ? 16 : 64;     // neighbourhood nodes
    static constexpr int KIN = NN + D;
    static constexpr int KPAD = D == 2 ? 32 : 96;
    static constexpr int KB = KPAD / 16;
};

// Weights in LDS: bf16 W1[64][KPAD], W2[64][64], W3[64][64] (output-major),
// optionally the transposes W2T, W3T; fp32 b1..b3, W4 (bf16 values), b4.
template <int D, bool TRANSPOSED> struct LdsWeights {
    unsigned short w1[HID * MlpShape<D>::KPAD];
    unsigned short w2[HID * HID];
    unsigned short w3[HID * HID];
    unsigned short w2t[TRANSPOSED ? HID * HID : 1];
    unsigned short w3t[TRANSPOSED ? HID * HID : 1];
    float b1[HID], b2[HID], b3[HID], w4[HID];
    float b4;
};

template <int D, bool TRANSPOSED>
__device__ void load_weights(LdsWeights<D, TRANSPOSED>& s, const mck::MlpDev& m)
{
    constexpr int KPAD = MlpShape<D>::KPAD;
    for (int i = threadIdx.x; i < HID * KPAD; i += blockDim.x) s.w1[i] = m.w1[i];
    for (int i = threadIdx.x; i < HID * HID; i += blockDim.x) {
        s.w2[i] = m.w2[i];
        s.w3[i] = m.w3[i];
        if (TRANSPOSED) {
            const int r = i / HID, c = i % HID;
            s.w2t[c * HID + r] = m.w2[i];
            s.w3t[c * HID + r] = m.w3[i];
        }
    }
    for (int i = threadIdx.x; i < HID; i += blockDim.x) {
        s.b1[i] = m.b1[i];
        s.b2[i] = m.b2[i];
        s.b3[i] = m.b3[i];
        s.w4[i] = bf2f(m.w4[i]);
    }
    if (threadIdx.x == 0) s.b4 = m.b4[0];
    __syncthreads();
}

// Inference copy of the weights in LDS, fragment-major for the K = 32
// instruction: the A fragment of row block mb and k pair c (16-blocks 2c
// and 2c + 1) for lane l is entry (mb * KC + c) * 64 + l, so a wave reads
// 1 KB of consecutive bytes per fragment (no bank conflicts).
template <int D> struct LdsFrag {
    bf16x8 w1[4 * (MlpShape<D>::KB / 2) * 64];
    bf16x8 w2[8 * 64];
    bf16x8 w3[8 * 64];
    bf16x8 w4f[2 * 64];          // the head as a 16 x 64 A operand: row 0 = W4, rows 1..15 zero
    float b1[HID], b2[HID], b3[HID], w4[HID];
    float b4;
};

__device__ __forceinline__ bf16x8 frag8_of(const unsigned short* w, int ld, int kpairs, int idx)
{
    const int l = idx & 63, c = (idx >> 6) % kpairs, mb = (idx >> 6) / kpairs, g = l >> 4;
    const unsigned short* row = w + (mb * 16 + (l & 15)) * ld;
    typedef short s8 __attribute__((ext_vector_type(8)));
    s8 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        r[i] = (short)row[(2 * c) * 16 + 4 * g + i];
        r[4 + i] = (short)row[(2 * c + 1) * 16 + 4 * g + i];
    }
    return __builtin_bit_cast(bf16x8, r);
}

template <int D>
__device__ void load_frag(LdsFrag<D>& s, const mck::MlpDev& m)
{
    constexpr int KC = MlpShape<D>::KB / 2, KPAD = MlpShape<D>::KPAD;
    for (int i = threadIdx.x; i < 4 * KC * 64; i += blockDim.x) s.w1[i] = frag8_of(m.w1, KPAD, KC, i);
    for (int i = threadIdx.x; i < 8 * 64; i += blockDim.x) {
        s.w2[i] = frag8_of(m.w2, HID, 2, i);
        s.w3[i] = frag8_of(m.w3, HID, 2, i);
    }
    for (int i = threadIdx.x; i < HID; i += blockDim.x) {
        s.b1[i] = m.b1[i];
        s.b2[i] = m.b2[i];
        s.b3[i] = m.b3[i];
        s.w4[i] = bf2f(m.w4[i]);
    }
    for (int i = threadIdx.x; i < 2 * 64; i += blockDim.x) {
        const int l = i & 63, c = i >> 6, g = l >> 4;
        typedef short s8 __attribute__((ext_vector_type(8)));
        s8 r;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r[k] = (l & 15) == 0 ? (short)m.w4[32 * c + 4 * g + k] : (short)0;
            r[4 + k] = (l & 15) == 0 ? (short)m.w4[32 * c + 16 + 4 * g + k] : (short)0;
        }
        s.w4f[i] = __builtin_bit_cast(bf16x8, r);
    }
    if (threadIdx.x == 0) s.b4 = m.b4[0];
    __syncthreads();
}

// A fragment: rows r0..r0+15 of a row-major bf16 matrix with leading
// dimension ld, columns c0 + 4(l/16) .. +3 for lane l.
__device__ __forceinline__ bf16x4 afrag(const unsigned short* w, int ld, int r0, int c0)
{
    const int l = lane_id();
    return *(const bf16x4*)(w + (r0 + (l & 15)) * ld + c0 + 4 * (l >> 4));
}

// Geometry of one vertex: grid cell, in-cell offsets and g(x1').
struct VGeom {
    int i0, i1, i2;
    float t0, t1, t2, g;
};

template <int D>
__device__ __forceinline__ VGeom vertex_geom(const float* __restrict__ coords, long long nv, long long v,
                                             const GridGeom& gg, const float* __restrict__ xh)
{
    VGeom q;
    q.i2 = 0;
    q.t2 = 0.0f;
    // coordinates, then the cell's corners, each batch issued before use
    const float p0 = coords[v], p1 = coords[nv + v], p2 = D == 3 ? coords[2 * nv + v] : 0.0f;
    axis_cell(p0, gg.of[0], gg.ihf[0], gg.n0, q.i0, q.t0);
    axis_cell(p1, gg.of[1], gg.ihf[1], gg.n1, q.i1, q.t1);
    if (D == 3) axis_cell(p2, gg.of[2], gg.ihf[2], gg.n2, q.i2, q.t2);
    const int n0 = gg.n0;
    const unsigned n01 = (unsigned)gg.n0 * (unsigned)gg.n1;
    const unsigned j = (unsigned)q.i0 + (unsigned)n0 * (unsigned)q.i1 + n01 * (unsigned)q.i2;
    float c[8];
    const f2a4 e0 = *reinterpret_cast<const f2a4*>(xh + j);       // x-adjacent corners: one 8-byte load
    const f2a4 e1 = *reinterpret_cast<const f2a4*>(xh + j + n0);
    c[0] = e0.x;
    c[1] = e0.y;
    c[2] = e1.x;
    c[3] = e1.y;
    if (D == 3) {
        const f2a4 e2 = *reinterpret_cast<const f2a4*>(xh + j + n01);
        const f2a4 e3 = *reinterpret_cast<const f2a4*>(xh + j + n01 + n0);
        c[4] = e2.x;
        c[5] = e2.y;
        c[6] = e3.x;
        c[7] = e3.y;
    }
    const float c00 = lerpf_(c[0], c[1], q.t0);
    const float c10 = lerpf_(c[2], c[3], q.t0);
    float g = lerpf_(c00, c10, q.t1);
    if (D == 3) {
        const float c01 = lerpf_(c[4], c[5], q.t0);
        const float c11 = lerpf_(c[6], c[7], q.t0);
        g = lerpf_(g, lerpf_(c01, c11, q.t1), q.t2);
    }
    q.g = g;
    return q;
}

__device__ __forceinline__ VGeom shfl_geom(const VGeom& a, int src)
{
    VGeom b;
    b.i0 = __shfl(a.i0, src, 64);
    b.i1 = __shfl(a.i1, src, 64);
    b.i2 = __shfl(a.i2, src, 64);
    b.t0 = __shfl(a.t0, src, 64);
    b.t1 = __shfl(a.t1, src, 64);
    b.t2 = __shfl(a.t2, src, 64);
    b.g = __shfl(a.g, src, 64);
    return b;
}

// Input k of a vertex (before BF16 rounding).
template <int D>
__device__ __forceinline__ float feature(int k, const VGeom& q, const GridGeom& gg, const float* __restrict__ xh,
                                         float kappa)
{
    constexpr int NN = MlpShape<D>::NN;
    if (k < NN) {
        const int a0 = k & 3, a1 = (k >> 2) & 3, a2 = k >> 4;
        const int n0 = min(max(q.i0 - 1 + a0, 0), gg.n0 - 1);
        const int n1 = min(max(q.i1 - 1 + a1, 0), gg.n1 - 1);
        const int n2 = D == 3 ? min(max(q.i2 - 1 + a2, 0), gg.n2 - 1) : 0;
        const float d = xh[(unsigned)n0 + (unsigned)gg.n0 * ((unsigned)n1 + (unsigned)gg.n1 * (unsigned)n2)] - q.g;
        return d * kappa;
    }
    if (k < NN + D) {
        const float t = (k - NN) == 0 ? q.t0 : ((k - NN) == 1 ? q.t1 : q.t2);
        return t - 0.5f;
    }
    return 0.0f;
}

// Four consecutive floats at a 4-byte aligned address.
typedef float f4a4 __attribute__((ext_vector_type(4), aligned(4)));

// Input fragments of the wave's 4 column blocks: zf[nb][kb].  Inputs
// k < NN are neighbourhood differences (one gather each), the next D the
// in-cell offsets, the rest zero padding; which fragment holds which is the
// same for every lane (16 inputs per fragment, NN a multiple of 16), so the
// gathers are issued NBB column blocks at a time, all before any is used,
// with no branch around them (an invalid vertex gathers a clamped node and
// its inputs are zeroed afterwards).
template <int D>
__device__ __forceinline__ void build_inputs(bf16x4 (&zf)[4][MlpShape<D>::KB], const VGeom& mine, bool valid_any,
                                             const GridGeom& gg, const float* __restrict__ xh, float kappa,
                                             const bool (&valid)[4])
{
    constexpr int NN = MlpShape<D>::NN, KB = MlpShape<D>::KB, KG = NN / 16;   // fragments with gathers
    constexpr int NBB = D == 2 ? 4 : 2;                                          // column blocks per batch
    const int l = lane_id(), g4 = 4 * (l >> 4);
#pragma unroll
    for (int nb0 = 0; nb0 < 4; nb0 += NBB) {
        VGeom q[NBB];
        float val[NBB][KG][4];
        // a lane's four inputs of a fragment are the x-neighbours i0-1 .. i0+2
        // of one (y, z) row: one 16-byte load when the whole wave is away from
        // the grid's x ends, else one clamped load each
#pragma unroll
        for (int u = 0; u < NBB; ++u) q[u] = shfl_geom(mine, (nb0 + u) * 16 + (l & 15));
        bool inner = true;
#pragma unroll
        for (int u = 0; u < NBB; ++u) inner = inner && q[u].i0 >= 1 && q[u].i0 + 2 <= gg.n0 - 1;
        if (__all(inner)) {
#pragma unroll
            for (int u = 0; u < NBB; ++u)
#pragma unroll
                for (int kb = 0; kb < KG; ++kb) {
                    const int a1 = (l >> 4) & 3, a2 = kb;
                    const int n1 = min(max(q[u].i1 - 1 + a1, 0), gg.n1 - 1);
                    const int n2 = D == 3 ? min(max(q[u].i2 - 1 + a2, 0), gg.n2 - 1) : 0;
                    const f4a4 r = *reinterpret_cast<const f4a4*>(
                        xh + ((unsigned)(q[u].i0 - 1) + (unsigned)gg.n0 * ((unsigned)n1 + (unsigned)gg.n1 * (unsigned)n2)));
                    val[u][kb][0] = r.x;
                    val[u][kb][1] = r.y;
                    val[u][kb][2] = r.z;
                    val[u][kb][3] = r.w;
                }
        } else {
#pragma unroll
            for (int u = 0; u < NBB; ++u)
#pragma unroll
                for (int kb = 0; kb < KG; ++kb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int k = kb * 16 + g4 + i;
                        const int a0 = k & 3, a1 = (k >> 2) & 3, a2 = k >> 4;
                        const int n0 = min(max(q[u].i0 - 1 + a0, 0), gg.n0 - 1);
                        const int n1 = min(max(q[u].i1 - 1 + a1, 0), gg.n1 - 1);
                        const int n2 = D == 3 ? min(max(q[u].i2 - 1 + a2, 0), gg.n2 - 1) : 0;
                        val[u][kb][i] =
                            xh[(unsigned)n0 + (unsigned)gg.n0 * ((unsigned)n1 + (unsigned)gg.n1 * (unsigned)n2)];
                    }
        }
#pragma unroll
        for (int u = 0; u < NBB; ++u) {
            const int nb = nb0 + u;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                float f[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = kb * 16 + g4 + i;
                    float x;
                    if (kb < KG) {
                        x = (val[u][kb < KG ? kb : 0][i] - q[u].g) * kappa;
                    } else if (k < NN + D) {
                        const float t = (k - NN) == 0 ? q[u].t0 : ((k - NN) == 1 ? q[u].t1 : q[u].t2);
                        x = t - 0.5f;
                    } else {
                        x = 0.0f;
                    }
                    f[i] = valid[nb] ? x : 0.0f;
                }
                zf[nb][kb] = pack4(f[0], f[1], f[2], f[3]);
            }
        }
    }
    (void)valid_any;
}

// One hidden layer: out[mb][nb] = bf16(relu(W[mb-block] . in[.][nb] + b)).
template <int KBLK>
__device__ __forceinline__ void hidden_layer(const unsigned short* w, int ld, const float* b,
                                             const bf16x4 (&in)[4][KBLK], bf16x4 (&out)[4][4], f32x4 (&pre)[4][4])
{
    const int g4 = 4 * (lane_id() >> 4);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        f32x4 acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KBLK; ++kb) {
            const bf16x4 a = afrag(w, ld, mb * 16, kb * 16);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma16(a, in[nb][kb], acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            float h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float x = acc[nb][i] + b[mb * 16 + g4 + i];
                h[i] = x > 0.0f ? x : 0.0f;
            }
            pre[mb][nb] = (f32x4){h[0], h[1], h[2], h[3]};
            out[nb][mb] = pack4(h[0], h[1], h[2], h[3]);
        }
    }
}

// The same layer with the weights in fragment-major LDS and the K = 32
// instruction (inference): KBLK 16-blocks of input, taken in pairs.
template <int KBLK>
__device__ __forceinline__ void hidden_layer_f(const bf16x8* wf, const float* b, const bf16x4 (&in)[4][KBLK],
                                               bf16x4 (&out)[4][4])
{
    constexpr int KC = KBLK / 2;
    const int l = lane_id(), g4 = 4 * (l >> 4);
    bf16x8 bin[4][KC];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int c = 0; c < KC; ++c) bin[nb][c] = cat8(in[nb][2 * c], in[nb][2 * c + 1]);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        // the bias starts the accumulation (one rounding order among others:
        // the forward pass is compared with a tolerance)
        const f32x4 bias = (f32x4){b[mb * 16 + g4], b[mb * 16 + g4 + 1], b[mb * 16 + g4 + 2], b[mb * 16 + g4 + 3]};
        f32x4 acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = bias;
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            const bf16x8 a = wf[(mb * KC + c) * 64 + l];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma32(a, bin[nb][c], acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
            out[nb][mb] = relu_bf(pack4(acc[nb][0], acc[nb][1], acc[nb][2], acc[nb][3]));
    }
}

// Head on the matrix cores: W4 as row 0 of a 16 x 64 A operand (the other
// rows zero), two K = 32 instructions per column block; rho of vertex
// nb*16 + c sits in lane c, element 0, and is broadcast to every lane.
__device__ __forceinline__ void head_f(const bf16x8* w4f, float b4, const bf16x4 (&h3)[4][4], float (&rho)[4])
{
    const int l = lane_id();
    const bf16x8 a0 = w4f[l], a1 = w4f[64 + l];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        f32x4 acc = (f32x4){b4, b4, b4, b4};
        acc = mfma32(a0, cat8(h3[nb][0], h3[nb][1]), acc);
        acc = mfma32(a1, cat8(h3[nb][2], h3[nb][3]), acc);
        rho[nb] = __shfl(acc[0], l & 15, 64);
    }
}

// Head: rho of vertex nb*16 + l%16 for every nb, summed over the 64 units in
// a fixed order (lane-local, then across the 4 row groups).
__device__ __forceinline__ void head(const float* w4, float b4, const bf16x4 (&h3)[4][4], float (&rho)[4])
{
    const int g4 = 4 * (lane_id() >> 4);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        float s = 0.0f;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) s = s + w4[mb * 16 + g4 + i] * bf2f((unsigned short)h3[nb][mb][i]);
        s = s + __shfl_xor(s, 16, 64);
        s = s + __shfl_xor(s, 32, 64);
        rho[nb] = s + b4;
    }
}

template <int D>
__device__ __forceinline__ void forward(const LdsWeights<D, false>* sw0, const unsigned short* w1,
                                        const unsigned short* w2, const unsigned short* w3, const float* b1,
                                        const float* b2, const float* b3, const float* w4, float b4,
                                        const bf16x4 (&zf)[4][MlpShape<D>::KB], bf16x4 (&h1)[4][4],
                                        bf16x4 (&h2)[4][4], bf16x4 (&h3)[4][4], float (&rho)[4])
{
    f32x4 pre[4][4];
    hidden_layer<MlpShape<D>::KB>(w1, MlpShape<D>::KPAD, b1, zf, h1, pre);
    hidden_layer<4>(w2, HID, b2, h1, h2, pre);
    hidden_layer<4>(w3, HID, b3, h2, h3, pre);
    head(w4, b4, h3, rho);
    (void)sw0;
}

template <int D>
__device__ __forceinline__ void forward_f(const LdsFrag<D>& sw, const bf16x4 (&zf)[4][MlpShape<D>::KB],
                                          float (&rho)[4])
{
    bf16x4 h1[4][4], h2[4][4], h3[4][4];
    hidden_layer_f<MlpShape<D>::KB>(sw.w1, sw.b1, zf, h1);
    hidden_layer_f<4>(sw.w2, sw.b2, h1, h2);
    hidden_layer_f<4>(sw.w3, sw.b3, h2, h3);
    head_f(sw.w4f, sw.b4, h3, rho);
}

__device__ __forceinline__ int rho_quant(float r)
{
    const double q = rint((double)r);
    if (!(q == q) || isinf(q)) return 0;
    if (q > (double)(MC_R - 1)) return MC_R - 1;
    if (q < -(double)(MC_R - 1)) return -(MC_R - 1);
    return (int)q;
}

// ---------------------------------------------------------------------------
// inference: rho_q for every vertex (or only those in learned blocks)
// ---------------------------------------------------------------------------
// Register use is capped at 128 (4 waves per SIMD): the inputs, the layer
// activations and the accumulators of a 64-vertex tile fit without spills.
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_mlp_infer(
    mck::MlpDev m, const float* __restrict__ coords, long long nv, GridGeom gg, const float* __restrict__ xh,
    const uint32_t* __restrict__ only_blocks, int32_t* __restrict__ rho_q)
{
    __shared__ LdsFrag<D> sw;
    load_frag<D>(sw, m);
    const long long ntiles = (nv + 63) / 64;
    const int l = lane_id();
    for (long long tile = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles;
         tile += (long long)gridDim.x * 4) {
        const long long v0 = tile * 64;
        if (only_blocks) {
            const long long blk = v0 / MC_LBLOCK;
            if (!((only_blocks[blk >> 5] >> (blk & 31)) & 1u)) continue;
        }
        const long long v = v0 + l;
        const VGeom mine = vertex_geom<D>(coords, nv, v < nv ? v : nv - 1, gg, xh);
        bool valid[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) valid[nb] = v0 + nb * 16 + (l & 15) < nv;
        bf16x4 zf[4][MlpShape<D>::KB];
        build_inputs<D>(zf, mine, true, gg, xh, m.kappa, valid);
        float rho[4];
        forward_f<D>(sw, zf, rho);
        // lane l holds vertex l of the tile as rho[l / 16]
        float r = rho[0];
        if ((l >> 4) == 1) r = rho[1];
        if ((l >> 4) == 2) r = rho[2];
        if ((l >> 4) == 3) r = rho[3];
        if (v < nv) rho_q[v] = rho_quant(r);
    }
}

// Inputs of vertices [v0, v0 + count) as floats [count][KPAD].
template <int D>
__global__ __launch_bounds__(256) void k_mlp_features(float kappa, const float* __restrict__ coords, long long nv,
                                                      GridGeom gg, const float* __restrict__ xh, long long v0,
                                                      long long count, float* __restrict__ z)
{
    constexpr int KPAD = MlpShape<D>::KPAD;
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= count) return;
    const VGeom q = vertex_geom<D>(coords, nv, v0 + s, gg, xh);
    for (int k = 0; k < KPAD; ++k) z[s * KPAD + k] = bfround(feature<D>(k, q, gg, xh, kappa));
}

// Forward pass on given inputs z[batch][KPAD] (already BF16-valued).
template <int D>
__global__ __launch_bounds__(256) void k_mlp_forward_z(mck::MlpDev m, const float* __restrict__ z, long long batch,
                                                       float* __restrict__ out)
{
    __shared__ LdsFrag<D> sw;
    load_frag<D>(sw, m);
    constexpr int KB = MlpShape<D>::KB, KPAD = MlpShape<D>::KPAD;
    const long long ntiles = (batch + 63) / 64;
    const int l = lane_id(), g4 = 4 * (l >> 4);
    for (long long tile = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles;
         tile += (long long)gridDim.x * 4) {
        bf16x4 zf[4][KB];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const long long s = tile * 64 + nb * 16 + (l & 15);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                float f[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) f[i] = s < batch ? z[s * KPAD + kb * 16 + g4 + i] : 0.0f;
                zf[nb][kb] = pack4(f[0], f[1], f[2], f[3]);
            }
        }
        float rho[4];
        forward_f<D>(sw, zf, rho);
        float r = rho[0];
        if ((l >> 4) == 1) r = rho[1];
        if ((l >> 4) == 2) r = rho[2];
        if ((l >> 4) == 3) r = rho[3];
        const long long s = tile * 64 + l;
        if (s < batch) out[s] = r;
    }
}

// Sum of (x1'[n] - g)^2 over every vertex and its 4^D neighbourhood nodes,
// FP64, per block (fixed assignment: the sum is the same on every run).
template <int D>
__global__ __launch_bounds__(256) void k_mlp_sumsq(const float* __restrict__ coords, long long nv, GridGeom gg,
                                                   const float* __restrict__ xh, double* __restrict__ partial)
{
    __shared__ double s_red[4];
    constexpr int NN = MlpShape<D>::NN;
    double acc = 0.0;
    for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < nv; v += (long long)gridDim.x * 256) {
        const VGeom q = vertex_geom<D>(coords, nv, v, gg, xh);
        for (int k = 0; k < NN; ++k) {
            const int a0 = k & 3, a1 = (k >> 2) & 3, a2 = k >> 4;
            const int n0 = min(max(q.i0 - 1 + a0, 0), gg.n0 - 1);
            const int n1 = min(max(q.i1 - 1 + a1, 0), gg.n1 - 1);
            const int n2 = D == 3 ? min(max(q.i2 - 1 + a2, 0), gg.n2 - 1) : 0;
            const double d = (double)xh[(unsigned)n0 + (unsigned)gg.n0 * ((unsigned)n1 + (unsigned)gg.n1 * (unsigned)n2)]
                             - (double)q.g;
            acc += d * d;
        }
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
        long long cnt = 0;
        for (long long v = (long long)blockIdx.x * 256; v < nv; v += (long long)gridDim.x * 256)
            cnt += (nv - v < 256 ? nv - v : 256);
        partial[2 * blockIdx.x + 1] = (double)(cnt * NN);
    }
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long splitmix64_dev(unsigned long long seed, unsigned long long ctr)
{
    // SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output number ctr+1 of
    // the generator whose state starts at seed
    unsigned long long z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct ParamOffsets {
    int w1, b1, w2, b2, w3, b3, w4, b4, n;
};

template <int D> __device__ __forceinline__ ParamOffsets param_offsets()
{
    ParamOffsets o;
    o.w1 = 0;
    o.b1 = HID * MlpShape<D>::KIN;
    o.w2 = o.b1 + HID;
    o.b2 = o.w2 + HID * HID;
    o.w3 = o.b2 + HID;
    o.b3 = o.w3 + HID * HID;
    o.w4 = o.b3 + HID;
    o.b4 = o.w4 + HID;
    o.n = o.b4 + 1;
    return o;
}

// Stages a D-layout fragment set (rows = units or inputs, cols = samples)
// into LDS as bf16 [row][64 samples].
__device__ __forceinline__ void stage_frag(unsigned short* buf, int r0, const bf16x4& f, int nb)
{
    const int l = lane_id(), g4 = 4 * (l >> 4), col = nb * 16 + (l & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) buf[(r0 + g4 + i) * 64 + col] = (unsigned short)f[i];
}

// dW[rows of A][rows of B] = sum over the 64 samples of A^T B (both staged
// [row][sample]); writes the result to grad (row-major, ldg columns, only
// columns < ncols).
template <int NBB>
__device__ __forceinline__ void weight_grad(const unsigned short* a, const unsigned short* b, float* grad, int ldg,
                                            int ncols)
{
    const int l = lane_id(), g4 = 4 * (l >> 4);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBB; ++nb) {
            f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const bf16x4 fa = *(const bf16x4*)(a + (mb * 16 + (l & 15)) * 64 + kb * 16 + g4);
                const bf16x4 fb = *(const bf16x4*)(b + (nb * 16 + (l & 15)) * 64 + kb * 16 + g4);
                acc = mfma16(fa, fb, acc);
            }
            const int col = nb * 16 + (l & 15);
            if (col < ncols)
#pragma unroll
                for (int i = 0; i < 4; ++i) grad[(mb * 16 + g4 + i) * ldg + col] = acc[i];
        }
}

// dH = W^T . dZ, then dZ_prev = dH * [h > 0].  The A fragment of W^T
// (rows = inputs k, columns = units u) is gathered from the row-major W.
__device__ __forceinline__ void input_grad(const unsigned short* w, const bf16x4 (&dz)[4][4], const bf16x4 (&h)[4][4],
                                           f32x4 (&dzp)[4][4])
{
    const int l = lane_id(), g4 = 4 * (l >> 4);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        f32x4 acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            bf16x4 a;
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = (short)w[(kb * 16 + g4 + i) * HID + mb * 16 + (l & 15)];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma16(a, dz[nb][kb], acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int i = 0; i < 4; ++i) dzp[mb][nb][i] = bf2f((unsigned short)h[nb][mb][i]) > 0.0f ? acc[nb][i] : 0.0f;
    }
}

// Sum over the 16 lanes that share l/16 (one row group), fixed order.
__device__ __forceinline__ float group16_sum(float s)
{
    s = s + __shfl_xor(s, 1, 64);
    s = s + __shfl_xor(s, 2, 64);
    s = s + __shfl_xor(s, 4, 64);
    s = s + __shfl_xor(s, 8, 64);
    return s;
}

// Bias gradient of one layer from its dZ (D-layout [mb][nb][i]): rows
// mb*16 + 4(l/16) + i, summed over the 64 samples.
__device__ __forceinline__ void bias_grad(const f32x4 (&dz)[4][4], float* grad)
{
    const int l = lane_id(), g4 = 4 * (l >> 4);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float s = ((dz[mb][0][i] + dz[mb][1][i]) + dz[mb][2][i]) + dz[mb][3][i];
            s = group16_sum(s);
            if ((l & 15) == 0) grad[mb * 16 + g4 + i] = s;
        }
}

template <int D>
__global__ __launch_bounds__(64) void k_mlp_train(mck::MlpDev m, const float* __restrict__ coords, long long nv,
                                                   GridGeom gg, const float* __restrict__ xh,
                                                   const mc_result* __restrict__ res, const void* __restrict__ xfield,
                                                   int dtype, const float* __restrict__ zin,
                                                   const float* __restrict__ yin, long long batch,
                                                   unsigned long long seed, long long step,
                                                   float* __restrict__ grad_part, float* __restrict__ loss_part)
{
    constexpr int KB = MlpShape<D>::KB, KPAD = MlpShape<D>::KPAD, KIN = MlpShape<D>::KIN;
    // one wave per workgroup: weights plus two staging buffers stay well
    // inside 64 KiB of LDS
    __shared__ LdsWeights<D, false> sw;
    constexpr int BROWS = KPAD > HID ? KPAD : HID;   // H^T (64 rows) or Z^T (KPAD rows)
    __shared__ unsigned short sbuf[HID * 64 + BROWS * 64];
    load_weights<D, false>(sw, m);
    const int l = lane_id(), g4 = 4 * (l >> 4);
    const long long part = blockIdx.x;                             // one wave = 64 samples
    const bool active = part * 64 < batch;
    unsigned short* bufA = sbuf;                 // dZ^T  [64 units][64 samples]
    unsigned short* bufB = sbuf + HID * 64;      // H^T or Z^T [BROWS][64 samples]
    const ParamOffsets po = param_offsets<D>();
    float* grad = grad_part + part * po.n;

    // ---- inputs and targets ----
    bf16x4 zf[4][KB];
    float y = 0.0f;
    const long long s = part * 64 + l;
    if (zin) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const long long sn = part * 64 + nb * 16 + (l & 15);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                float f[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) f[i] = (active && sn < batch) ? zin[sn * KPAD + kb * 16 + g4 + i] : 0.0f;
                zf[nb][kb] = pack4(f[0], f[1], f[2], f[3]);
            }
        }
        y = (active && s < batch) ? yin[s] : 0.0f;
    } else {
        const unsigned long long r = splitmix64_dev(seed, (unsigned long long)(step * batch + s));
        const long long v = (long long)(((r >> 32) * (unsigned long long)nv) >> 32);
        const VGeom mine = vertex_geom<D>(coords, nv, v, gg, xh);
        bool valid[4] = {active, active, active, active};
        build_inputs<D>(zf, mine, true, gg, xh, m.kappa, valid);
        const double inv2 = 1.0 / (2.0 * res->tau2);
        const double xv = dtype == MC_F64 ? ((const double*)xfield)[v] : (double)((const float*)xfield)[v];
        y = (float)((xv - (double)mine.g) * inv2);
    }

    // ---- forward ----
    bf16x4 h1[4][4], h2[4][4], h3[4][4];
    float rho[4];
    forward<D>(nullptr, sw.w1, sw.w2, sw.w3, sw.b1, sw.b2, sw.b3, sw.w4, sw.b4, zf, h1, h2, h3, rho);
    float r = rho[0];
    if ((l >> 4) == 1) r = rho[1];
    if ((l >> 4) == 2) r = rho[2];
    if ((l >> 4) == 3) r = rho[3];
    const bool mine_ok = active && s < batch;
    const float e = mine_ok ? r - y : 0.0f;
    const float dr_mine = mine_ok ? 2.0f * e / (float)batch : 0.0f;
    const float lsum = wave_sum(e * e);

    // dr of vertex nb*16 + l%16
    float dr[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) dr[nb] = __shfl(dr_mine, nb * 16 + (l & 15), 64);

    // ---- head gradients and dZ3 ----
    f32x4 dz[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int u = mb * 16 + g4 + i;
            float gw = 0.0f;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const float h = bf2f((unsigned short)h3[nb][mb][i]);
                gw = gw + dr[nb] * h;
                dz[mb][nb][i] = h > 0.0f ? sw.w4[u] * dr[nb] : 0.0f;
            }
            gw = group16_sum(gw);
            if ((l & 15) == 0 && active) grad[po.w4 + u] = gw;
        }
    {
        // dr[nb] is the same in the 4 row groups: sum one group's 16 lanes
        float sb = (((dr[0] + dr[1]) + dr[2]) + dr[3]);
        sb = group16_sum(sb);
        if (l == 0 && active) {
            grad[po.b4] = sb;
            loss_part[part] = lsum;
        }
    }
    if (active) bias_grad(dz, grad + po.b3);

    // ---- layer 3: dW3 = dZ3^T . H2, dZ2 = (W3^T dZ3) * [h2 > 0] ----
    bf16x4 dzf[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            dzf[nb][mb] = pack4(dz[mb][nb][0], dz[mb][nb][1], dz[mb][nb][2], dz[mb][nb][3]);
            stage_frag(bufA, mb * 16, dzf[nb][mb], nb);
            stage_frag(bufB, mb * 16, h2[nb][mb], nb);
        }
    __syncthreads();
    if (active) weight_grad<4>(bufA, bufB, grad + po.w3, HID, HID);
    input_grad(sw.w3, dzf, h2, dz);
    __syncthreads();
    if (active) bias_grad(dz, grad + po.b2);

    // ---- layer 2 ----
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            dzf[nb][mb] = pack4(dz[mb][nb][0], dz[mb][nb][1], dz[mb][nb][2], dz[mb][nb][3]);
            stage_frag(bufA, mb * 16, dzf[nb][mb], nb);
            stage_frag(bufB, mb * 16, h1[nb][mb], nb);
        }
    __syncthreads();
    if (active) weight_grad<4>(bufA, bufB, grad + po.w2, HID, HID);
    input_grad(sw.w2, dzf, h1, dz);
    __syncthreads();
    if (active) bias_grad(dz, grad + po.b1);

    // ---- layer 1: dW1 = dZ1^T . Z ----
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const bf16x4 f = pack4(dz[mb][nb][0], dz[mb][nb][1], dz[mb][nb][2], dz[mb][nb][3]);
            stage_frag(bufA, mb * 16, f, nb);
        }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) stage_frag(bufB, kb * 16, zf[nb][kb], nb);
    __syncthreads();
    if (active) weight_grad<KB>(bufA, bufB, grad + po.w1, KIN, KIN);
}

// Sums the per-wave gradients in a fixed order; optionally one Adam step on
// the FP32 master parameters.
__global__ __launch_bounds__(256) void k_mlp_reduce_adam(int np, int nparts, const float* __restrict__ grad_part,
                                                         const float* __restrict__ loss_part, float* __restrict__ grad,
                                                         float* __restrict__ loss_out, float* __restrict__ params,
                                                         float* __restrict__ mom, float* __restrict__ vel, float lr,
                                                         float bc1, float bc2, int apply, float inv_batch)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k == 0) {
        float ls = 0.0f;
        for (int p = 0; p < nparts; ++p) ls = ls + loss_part[p];
        *loss_out = ls * inv_batch;
    }
    if (k >= np) return;
    float g = 0.0f;
    for (int p = 0; p < nparts; ++p) g = g + grad_part[(long long)p * np + k];
    grad[k] = g;
    if (apply) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float mk = b1 * mom[k] + (1.0f - b1) * g;
        const float vk = b2 * vel[k] + (1.0f - b2) * (g * g);
        mom[k] = mk;
        vel[k] = vk;
        const float mh = mk / bc1, vh = vk / bc2;
        params[k] = params[k] - lr * mh / (sqrtf(vh) + eps);
    }
}

// Master FP32 parameters -> the device model (bf16 weights, fp32 biases).
template <int D>
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ p, uint16_t* __restrict__ w1,
                                                  uint16_t* __restrict__ w2, uint16_t* __restrict__ w3,
                                                  uint16_t* __restrict__ w4, float* __restrict__ b1,
                                                  float* __restrict__ b2, float* __restrict__ b3, float* __restrict__ b4)
{
    constexpr int KIN = MlpShape<D>::KIN, KPAD = MlpShape<D>::KPAD;
    const ParamOffsets o = param_offsets<D>();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < HID * KPAD) {
        const int u = i / KPAD, k = i % KPAD;
        w1[i] = k < KIN ? f2bf(p[o.w1 + u * KIN + k]) : (uint16_t)0;
    }
    if (i < HID * HID) {
        w2[i] = f2bf(p[o.w2 + i]);
        w3[i] = f2bf(p[o.w3 + i]);
    }
    if (i < HID) {
        w4[i] = f2bf(p[o.w4 + i]);
        b1[i] = p[o.b1 + i];
        b2[i] = p[o.b2 + i];
        b3[i] = p[o.b3 + i];
    }
    if (i == 0) b4[0] = p[o.b4];
}

// ---------------------------------------------------------------------------
namespace mck {

static int n_params(int dim) { return dim == 2 ? (64 * 18 + 64 + 4096 + 64 + 4096 + 64 + 64 + 1)
                                               : (64 * 67 + 64 + 4096 + 64 + 4096 + 64 + 64 + 1); }

hipError_t mlp_pack(const float* params, int dim, uint16_t* w1, uint16_t* w2, uint16_t* w3, uint16_t* w4, float* b1,
                    float* b2, float* b3, float* b4, hipStream_t s)
{
    const int n = 64 * 96;
    if (dim == 2)
        hipLaunchKernelGGL(k_mlp_pack<2>, dim3((n + 255) / 256), dim3(256), 0, s, params, w1, w2, w3, w4, b1, b2, b3, b4);
    else
        hipLaunchKernelGGL(k_mlp_pack<3>, dim3((n + 255) / 256), dim3(256), 0, s, params, w1, w2, w3, w4, b1, b2, b3, b4);
    return hipGetLastError();
}

hipError_t mlp_infer(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh,
                     const uint32_t* only_blocks, int32_t* rho_q, hipStream_t s)
{
    ProfScope ps(only_blocks ? "k_mlp_infer_d" : "k_mlp_infer_c", s);
    long long nb = (nv + 255) / 256;
    if (nb > 2048) nb = 2048;
    if (nb < 1) nb = 1;
    if (m.dim == 2)
        hipLaunchKernelGGL(k_mlp_infer<2>, dim3((unsigned)nb), dim3(256), 0, s, m, coords, nv, gg, xh, only_blocks, rho_q);
    else
        hipLaunchKernelGGL(k_mlp_infer<3>, dim3((unsigned)nb), dim3(256), 0, s, m, coords, nv, gg, xh, only_blocks, rho_q);
    return hipGetLastError();
}

hipError_t mlp_features(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh, long long v0,
                        long long count, float* z, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    dim3 grid((unsigned)((count + 255) / 256));
    if (m.dim == 2)
        hipLaunchKernelGGL(k_mlp_features<2>, grid, dim3(256), 0, s, m.kappa, coords, nv, gg, xh, v0, count, z);
    else
        hipLaunchKernelGGL(k_mlp_features<3>, grid, dim3(256), 0, s, m.kappa, coords, nv, gg, xh, v0, count, z);
    return hipGetLastError();
}

hipError_t mlp_forward_z(const MlpDev& m, const float* z, long long batch, float* rho, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    long long nb = (batch + 255) / 256;
    if (nb > 2048) nb = 2048;
    if (m.dim == 2)
        hipLaunchKernelGGL(k_mlp_forward_z<2>, dim3((unsigned)nb), dim3(256), 0, s, m, z, batch, rho);
    else
        hipLaunchKernelGGL(k_mlp_forward_z<3>, dim3((unsigned)nb), dim3(256), 0, s, m, z, batch, rho);
    return hipGetLastError();
}

hipError_t mlp_feature_sumsq(const float* coords, long long nv, GridGeom gg, const float* xh, int dim,
                             double* partial, int nblocks, hipStream_t s)
{
    if (dim == 2)
        hipLaunchKernelGGL(k_mlp_sumsq<2>, dim3(nblocks), dim3(256), 0, s, coords, nv, gg, xh, partial);
    else
        hipLaunchKernelGGL(k_mlp_sumsq<3>, dim3(nblocks), dim3(256), 0, s, coords, nv, gg, xh, partial);
    return hipGetLastError();
}

hipError_t train_step_grad(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh,
                           const mc_result* res, const float* z_given, const float* y_given, const void* x, int dtype,
                           long long batch, unsigned long long seed, long long step, float* grad_part,
                           float* loss_part, int nparts, hipStream_t s)
{
    ProfScope ps("k_mlp_train", s);
    dim3 grid((unsigned)nparts);
    if (m.dim == 2)
        hipLaunchKernelGGL(k_mlp_train<2>, grid, dim3(64), 0, s, m, coords, nv, gg, xh, res, x, dtype, z_given,
                           y_given, batch, seed, step, grad_part, loss_part);
    else
        hipLaunchKernelGGL(k_mlp_train<3>, grid, dim3(64), 0, s, m, coords, nv, gg, xh, res, x, dtype, z_given,
                           y_given, batch, seed, step, grad_part, loss_part);
    return hipGetLastError();
}

hipError_t train_reduce_adam(int nparams, int nparts, const float* grad_part, const float* loss_part, float* grad,
                             float* loss_out, float* params, float* m, float* v, long long t, float lr, int apply,
                             long long batch, hipStream_t s)
{
    ProfScope ps("k_mlp_adam", s);
    const float bc1 = (float)(1.0 - pow(0.9, (double)(t > 0 ? t : 1)));
    const float bc2 = (float)(1.0 - pow(0.999, (double)(t > 0 ? t : 1)));
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((nparams + 255) / 256), dim3(256), 0, s, nparams, nparts, grad_part,
                       loss_part, grad, loss_out, params, m, v, lr, bc1, bc2, apply, 1.0f / (float)batch);
    (void)n_params;
    return hipGetLastError();
}

}  // namespace mck
