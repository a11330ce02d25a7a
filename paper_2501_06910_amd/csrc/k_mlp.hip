// k_mlp.hip -- learned residual predictor on gfx950 matrix cores.
//
// Network: in -> 64 -> 64 -> 64 -> 1, ReLU; weights BF16, accumulation
// FP32, hidden activations re-rounded to BF16 after bias and ReLU.  Inputs
// of a vertex: bf16((x1'[n] - g) * kappa) for the 4^D grid nodes around its
// grid cell (indices clamped), then bf16(t_d - 0.5), zero padded to KPAD.
//
// Layout.  In inference a wave owns 64 vertices (4 column blocks of 16).
// Every layer is computed transposed, H^T = W . X^T, with
// v_mfma_f32_16x16x32_bf16: A = a 16-row block of W (from the fragment
// image in LDS), B = 16 vertices x 32 inputs.  The output fragment of one
// layer (lane l holds rows 4(l/16)..+3 of column l%16) is exactly half of
// the B fragment the next layer needs, so activations never leave registers
// in the forward pass.  Input fragments are built directly in that layout:
// lane l computes inputs 4(l/16)+16kb+i of vertex l%16 of each block.
//
// Kernels: k_mlp_residual (compress: the network on every vertex of a
// 4,096-vertex decision block, then the block's codes) and k_mlp_vdecode
// (decompress: the network on the learned blocks, every vertex decoded);
// training: see the block comment above stage_frag.
#include <type_traits>

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

// Weights as MFMA A fragments for the K = 32 instruction ("fragment
// image"): the fragment of row block mb and k pair c (16-blocks 2c and
// 2c + 1) for lane l is entry (mb * KC + c) * 64 + l, so a wave reads 1 KB
// of consecutive bytes per fragment (no LDS bank conflicts).  The image is
// built once per model change in device memory and copied to LDS with
// 16-byte loads.  LdsFrag is what inference needs; training also needs the
// transposes of W2 and W3 (A operands of dH = W^T dZ).
template <int D> struct LdsFrag {
    bf16x8 w1[4 * (MlpShape<D>::KB / 2) * 64];
    bf16x8 w2[8 * 64];
    bf16x8 w3[8 * 64];
    bf16x8 w4f[2 * 64];          // the head as a 16 x 64 A operand: row 0 = W4, rows 1..15 zero
    float b1[HID], b2[HID], b3[HID], w4[HID];
    float b4;
};
template <int D> struct FragImg {
    LdsFrag<D> f;
    bf16x8 w2t[8 * 64];
    bf16x8 w3t[8 * 64];
};

// Short index of element (r, c) of a row-major matrix in its fragment
// image with kpairs 32-wide column pairs: lane 16(c%16/4) + r%16 of entry
// (r/16, c/32), slot 4((c/16)%2) + c%4.
__device__ __forceinline__ int frag_pos(int r, int c, int kpairs)
{
    const int kb = c >> 4, within = c & 15;
    const int lane = (within >> 2) * 16 + (r & 15);
    return ((((r >> 4) * kpairs + (kb >> 1)) * 64 + lane) << 3) + ((kb & 1) << 2) + (within & 3);
}
// Short index of W4[u] in the head operand (row 0 of a 16 x 64 A operand).
__device__ __forceinline__ int head_pos(int u)
{
    return (((u >> 5) * 64 + ((u & 15) >> 2) * 16) << 3) + (((u >> 4) & 1) << 2) + (u & 3);
}

// Copies NBYTES (a multiple of 16) from global memory to LDS with NT
// threads, all loads issued before the stores.
template <int NBYTES, int NT>
__device__ __forceinline__ void copy_to_lds(void* dst, const void* src)
{
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    constexpr int N = NBYTES / 16, PER = (N + NT - 1) / NT;
    static_assert(NBYTES % 16 == 0, "16-byte granules");
    const u32x4* s = (const u32x4*)src;
    u32x4* d = (u32x4*)dst;
    u32x4 v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = j * NT + (int)threadIdx.x;
        if (i < N) v[j] = s[i];
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = j * NT + (int)threadIdx.x;
        if (i < N) d[i] = v[j];
    }
}

template <int D, int NT>
__device__ __forceinline__ void load_frag(LdsFrag<D>& s, const mck::MlpDev& m)
{
    copy_to_lds<sizeof(LdsFrag<D>), NT>(&s, m.img);
    __syncthreads();
}

// Builds the fragment image from the row-major BF16 weights and FP32
// biases of a model (one thread per short of the image).
template <int D>
__global__ __launch_bounds__(256) void k_mlp_image(mck::MlpDev m, FragImg<D>* __restrict__ img)
{
    constexpr int KC = MlpShape<D>::KB / 2, KPAD = MlpShape<D>::KPAD;
    unsigned short* w1 = (unsigned short*)img->f.w1;
    unsigned short* w2 = (unsigned short*)img->f.w2;
    unsigned short* w3 = (unsigned short*)img->f.w3;
    unsigned short* w4f = (unsigned short*)img->f.w4f;
    unsigned short* w2t = (unsigned short*)img->w2t;
    unsigned short* w3t = (unsigned short*)img->w3t;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < HID * KPAD) {
        const int r = i / KPAD, c = i % KPAD;
        w1[frag_pos(r, c, KC)] = m.w1[i];
    }
    if (i < HID * HID) {
        const int r = i >> 6, c = i & 63;
        w2[frag_pos(r, c, 2)] = m.w2[i];
        w3[frag_pos(r, c, 2)] = m.w3[i];
        w2t[frag_pos(c, r, 2)] = m.w2[i];
        w3t[frag_pos(c, r, 2)] = m.w3[i];
    }
    if (i < 2 * 64 * 8) {                    // head operand: W4 in row 0, zeros elsewhere
        const int l = (i >> 3) & 63, c = i >> 9, slot = i & 7;
        w4f[i] = (l & 15) == 0 ? m.w4[32 * c + 16 * (slot >> 2) + 4 * (l >> 4) + (slot & 3)] : (unsigned short)0;
    }
    if (i < HID) {
        img->f.b1[i] = m.b1[i];
        img->f.b2[i] = m.b2[i];
        img->f.b3[i] = m.b3[i];
        img->f.w4[i] = bf2f(m.w4[i]);
    }
    if (i == 0) img->f.b4 = m.b4[0];
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
template <int D, bool MASK = true>
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
                    f[i] = (!MASK || valid[nb]) ? x : 0.0f;
                }
                zf[nb][kb] = pack4(f[0], f[1], f[2], f[3]);
            }
        }
    }
    (void)valid_any;
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

// clamp(rint(r), -(R-1), R-1), 0 for a non-finite r.  Rounding in FP32 is
// exact (every float of magnitude >= 2^23 is an integer already), so this
// equals rounding the value widened to FP64.
__device__ __forceinline__ int rho_quant(float r)
{
    const float q = rintf(r);
    if (!(q == q) || isinf(q)) return 0;
    if (q > (float)(MC_R - 1)) return MC_R - 1;
    if (q < -(float)(MC_R - 1)) return -(MC_R - 1);
    return (int)q;
}

// Cell and in-cell offsets of one vertex, with its g(x1') given.
template <int D>
__device__ __forceinline__ VGeom vertex_cell(const float* __restrict__ coords, long long nv, long long v,
                                             const GridGeom& gg, float g)
{
    VGeom q;
    q.i2 = 0;
    q.t2 = 0.0f;
    const float p0 = coords[v], p1 = coords[nv + v], p2 = D == 3 ? coords[2 * nv + v] : 0.0f;
    axis_cell(p0, gg.of[0], gg.ihf[0], gg.n0, q.i0, q.t0);
    axis_cell(p1, gg.of[1], gg.ihf[1], gg.n1, q.i1, q.t1);
    if (D == 3) axis_cell(p2, gg.of[2], gg.ihf[2], gg.n2, q.i2, q.t2);
    q.g = g;
    return q;
}

// Learned vertex codes in one kernel: one 512-thread workgroup per
// 4,096-vertex decision block, two workgroups per CU so that one's memory
// phase overlaps the other's network.
//   phase 0  g(x1') and the plain code q of the block's first 512 vertices;
//            if one of them is not zero, the block is coded directly
//            (phase 1 recomputes g with the network's inputs, pass A
//            quantises the rest).  Otherwise the rest of the block too: a
//            block whose plain codes are all zero (no outlier) costs 0
//            bits, so the shifted codes cannot be strictly cheaper: its
//            plain codes are written and the network is not run (unless
//            the shifts are asked for, rho_out)
//   phase 1  the network on the block's 64-vertex tiles (8 per wave), the
//            shift rho_q of every vertex kept in LDS
//   pass A   the block's cost of the plain and of the shifted codes
//            (bitlen(zigzag(code)) per coded vertex plus (32 + 8 sizeof(T))
//            per outlier)
//   pass B   the codes of the cheaper choice (shifted only when strictly
//            cheaper) and each 1,024-vertex tile's outlier count, bit 31
//            marking the first tile of a learned block
// rho_out (optional) receives rho_q.
template <typename T, int D>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_mlp_residual(
    mck::MlpDev m, const float* __restrict__ coords, long long nv, GridGeom gg, const float* __restrict__ xh,
    const T* __restrict__ x, const DevBound* __restrict__ bnd, uint16_t* __restrict__ codes,
    uint32_t* __restrict__ bflags, float* __restrict__ dbg_g, int32_t* __restrict__ rho_out,
    unsigned int* __restrict__ count, unsigned int* __restrict__ vsum, long long ntv)
{
    constexpr int NT = 512, NW = NT / 64, PT = MC_LBLOCK / NT, LT = MC_LBLOCK / MC_TILE;
    static_assert(MC_LBLOCK % NT == 0 && MC_TILE % NT == 0 && LT <= NW && PT == 8, "block layout: rows 1..7 as 4 + 3");
    static_assert(MC_R - 1 <= 32767, "codes and shifts fit int16");
    constexpr short OUT = -32768;                               // q marker of an outlier
    __shared__ LdsFrag<D> sw;
    __shared__ float s_g[MC_LBLOCK];
    __shared__ short s_q[MC_LBLOCK], s_rq[MC_LBLOCK];
    __shared__ long long s_sp[NW], s_sl[NW];
    __shared__ int s_cnt[LT][NW];
    const long long blk = blockIdx.x, vb = blk * MC_LBLOCK;
    const int w = threadIdx.x >> 6, l = lane_id();
    const DevBound b = *bnd;
    bool nz = false;
    // g and the plain code of vertices vb + k, k = i NT + tid for i in [i0, i0 + N)
    auto quantize_rows = [&](auto n_tag, int i0) {
        constexpr int N = decltype(n_tag)::value;
        long long v[N];
        bool act[N];
        T xv[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            v[i] = vb + (i0 + i) * NT + (int)threadIdx.x;
            act[i] = v[i] < nv;
            xv[i] = x[act[i] ? v[i] : 0];
        }
        float g[N];
        back_interp_n<D, N, false>(coords, nv, gg, xh, 0.0, 0.0, v, act, g);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            if (!act[i]) continue;
            const int k = (i0 + i) * NT + (int)threadIdx.x;
            s_g[k] = g[i];
            if (!b.ok) continue;
            int q;
            const bool ok = quantize_residual<T>(xv[i], g[i], b, q);
            s_q[k] = ok ? (short)q : OUT;
            nz = nz || !ok || q != 0;
            if (dbg_g) dbg_g[v[i]] = g[i];
        }
    };
    // the network's weights are copied to LDS first, so that their loads
    // overlap phase 0; the barrier after phase 0 completes the copy
    copy_to_lds<sizeof(LdsFrag<D>), NT>(&sw, m.img);
    quantize_rows(std::integral_constant<int, 1>{}, 0);          // phase 0
    const bool direct = __syncthreads_or(nz) != 0;              // uniform over the workgroup
    if (!direct) {
        quantize_rows(std::integral_constant<int, 4>{}, 1);
        quantize_rows(std::integral_constant<int, 3>{}, 5);
        const bool any = __syncthreads_or(nz) != 0;
        if (!any && !rho_out) {
#pragma unroll
            for (int i = 0; i < PT; ++i) {
                const long long v = vb + i * NT + (int)threadIdx.x;
                if (v < nv && b.ok) codes[v] = (uint16_t)MC_R;
            }
            const long long tile = blk * LT + threadIdx.x;
            if (threadIdx.x < LT && tile < ntv) count[tile] = 0u;
            return;
        }
    }
    for (int t = w; t < MC_LBLOCK / 64; t += NW) {               // phase 1
        const long long v0 = vb + t * 64;
        if (v0 >= nv) break;                                     // uniform over the wave
        const long long v = v0 + l;
        const long long vc = v < nv ? v : nv - 1;
        const VGeom mine = direct ? vertex_geom<D>(coords, nv, vc, gg, xh)
                                  : vertex_cell<D>(coords, nv, vc, gg, v < nv ? s_g[t * 64 + l] : 0.0f);
        if (direct && v < nv) s_g[t * 64 + l] = mine.g;
        bool valid[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) valid[nb] = v0 + nb * 16 + (l & 15) < nv;
        bf16x4 zf[4][MlpShape<D>::KB];
        if (D == 2 && v0 + 64 <= nv)
            build_inputs<D, false>(zf, mine, true, gg, xh, m.kappa, valid);
        else
            build_inputs<D, true>(zf, mine, true, gg, xh, m.kappa, valid);
        float rho[4];
        forward_f<D>(sw, zf, rho);
        float r = rho[0];
        if ((l >> 4) == 1) r = rho[1];
        if ((l >> 4) == 2) r = rho[2];
        if ((l >> 4) == 3) r = rho[3];
        const int rq = rho_quant(r);
        s_rq[t * 64 + l] = (short)rq;
        if (rho_out && v < nv) rho_out[v] = rq;
    }
    __syncthreads();
    const int ocost = 32 + 8 * (int)sizeof(T);
    long long cp = 0, cl = 0;
#pragma unroll
    for (int i = 0; i < PT; ++i) {                               // pass A
        const int k = i * NT + (int)threadIdx.x;
        const long long v = vb + k;
        if (v >= nv || !b.ok) continue;
        if (direct && i > 0) {                                   // not quantised in phase 0
            const float g = s_g[k];
            int qq;
            const bool ok = quantize_residual<T>(x[v], g, b, qq);
            s_q[k] = ok ? (short)qq : OUT;
            if (dbg_g) dbg_g[v] = g;
        }
        const int q = s_q[k];
        if (q != OUT) {
            const int lq = q - s_rq[k];
            cp += zz_bits(q);
            cl += (lq >= -(MC_R - 1) && lq <= MC_R - 1) ? zz_bits(lq) : ocost;
        } else {
            cp += ocost;
            cl += ocost;
        }
    }
    cp = wave_sum(cp);
    cl = wave_sum(cl);
    if (l == 0) { s_sp[w] = cp; s_sl[w] = cl; }
    __syncthreads();
    long long sp = 0, sl = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) { sp += s_sp[k]; sl += s_sl[k]; }
    const bool learned = sl < sp;                                // uniform over the workgroup
    int nout[LT] = {};
#pragma unroll
    for (int i = 0; i < PT; ++i) {                               // pass B
        const int k = i * NT + (int)threadIdx.x;
        const long long v = vb + k;
        if (v >= nv || !b.ok) continue;
        int q = s_q[k];
        bool ok = q != OUT;
        if (ok && learned) {
            q -= s_rq[k];
            ok = q >= -(MC_R - 1) && q <= MC_R - 1;
        }
        codes[v] = ok ? (uint16_t)(q + MC_R) : (uint16_t)0;
        nout[k / MC_TILE] += ok ? 0 : 1;
    }
#pragma unroll
    for (int tl = 0; tl < LT; ++tl) {
        const int c = wave_sum(nout[tl]);
        if (l == 0) s_cnt[tl][w] = c;
    }
    __syncthreads();
    const long long tile = blk * LT + threadIdx.x;
    if (threadIdx.x < LT && tile < ntv) {
        unsigned c = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) c += (unsigned)s_cnt[threadIdx.x][k];
        if (c) atomicAdd(&vsum[tile / MC_SC_TILES], c);
        if (learned && threadIdx.x == 0) {
            c |= 0x80000000u;
            atomicOr(&bflags[blk >> 5], 1u << (blk & 31));
        }
        count[tile] = c;
    }
}

// Learned decompress in one pass: every 64-vertex tile decodes its
// vertices, x' = (T)(g + (q + rho_q) * 2 tau2) with q = code - R (raw values
// for outliers), where g is the back-interpolation the network's inputs
// already need (the same operations as the vertex decoder's, so the same
// bits) and rho_q is the network's shift in learned blocks, 0 elsewhere (no
// network evaluation there).  The shifts never reach memory.
template <int D, typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_mlp_vdecode(
    mck::MlpDev m, const float* __restrict__ coords, long long nv, GridGeom gg, const float* __restrict__ xh,
    const uint32_t* __restrict__ bflags, const uint16_t* __restrict__ codes, const int32_t* __restrict__ oidx,
    const T* __restrict__ oval, const mc_result* __restrict__ res, long long vcap, T* __restrict__ xout)
{
    __shared__ LdsFrag<D> sw;
    load_frag<D, 256>(sw, m);
    const long long ntiles = (nv + 63) / 64;
    const int l = lane_id();
    const double step2 = 2.0 * res->tau2;
    const long long nout = res->n_vertex_outliers < vcap ? res->n_vertex_outliers : vcap;
    for (long long tile = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles;
         tile += (long long)gridDim.x * 4) {
        const long long v0 = tile * 64;
        const long long blk = v0 / MC_LBLOCK;                    // a tile lies inside one block
        const bool learned = (bflags[blk >> 5] >> (blk & 31)) & 1u;
        const long long v = v0 + l;
        const long long vc = v < nv ? v : nv - 1;
        const VGeom mine = vertex_geom<D>(coords, nv, vc, gg, xh);
        const float g = mine.g;
        int rq = 0;
        if (learned) {                                           // uniform over the wave
            bool valid[4];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) valid[nb] = v0 + nb * 16 + (l & 15) < nv;
            bf16x4 zf[4][MlpShape<D>::KB];
            if (D == 2 && v0 + 64 <= nv)
                build_inputs<D, false>(zf, mine, true, gg, xh, m.kappa, valid);
            else
                build_inputs<D, true>(zf, mine, true, gg, xh, m.kappa, valid);
            float rho[4];
            forward_f<D>(sw, zf, rho);
            float r = rho[0];
            if ((l >> 4) == 1) r = rho[1];
            if ((l >> 4) == 2) r = rho[2];
            if ((l >> 4) == 3) r = rho[3];
            rq = rho_quant(r);
        }
        if (v < nv) {
            const int code = codes[v];                           // loaded after the network: fewer live registers
            if (code == 0) {
                const long long k = find_outlier(oidx, nout, v);
                xout[v] = k >= 0 ? oval[k] : (T)0;
            } else {
                const int q = code - MC_R + rq;
                xout[v] = (T)((double)g + (double)q * step2);
            }
        }
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
    load_frag<D, 256>(sw, m);
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

// Training, one step of minibatch B:
//  * k_mlp_sample draws the samples of several steps in one launch (a wave
//    per 64 samples: SplitMix64 vertex, inputs as B fragments, target in
//    code units), so no gather latency sits inside a step;
//  * k_mlp_train: one workgroup of 8 waves per 64 samples.  Wave w takes
//    column block nb = w % 4 (16 samples) and unit half mh = w / 4 (row
//    blocks 2mh, 2mh + 1) of every layer; the halves of a layer's output
//    meet in LDS as B fragments for the next layer.  Backward: dZ = dH *
//    [h > 0]; dW = dZ^T . H with the samples as the K dimension (dZ^T and
//    H^T staged [unit][sample] in LDS), dH = W^T . dZ from the transposed
//    weight fragments.  Each workgroup writes its gradient to its own slot;
//  * k_mlp_adam sums the slots in a fixed order (the same gradient on every
//    run), applies Adam to the FP32 master parameters and writes the BF16
//    weights both row-major and into the fragment image.

// LDS row stride of the [row][sample] staging buffers: 72 shorts keeps the
// 16 rows of a fragment read on different banks.
#define SP 72

// Stages a fragment (rows r0 + 4(l/16) + i, sample column nb*16 + l%16)
// into a [row][sample] buffer.
__device__ __forceinline__ void stage_frag(unsigned short* buf, int r0, const bf16x4& f, int nb)
{
    const int l = lane_id(), g4 = 4 * (l >> 4), col = nb * 16 + (l & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) buf[(r0 + g4 + i) * SP + col] = (unsigned short)f[i];
}

// K = 32 operand of rows r0..r0+15 of a [row][sample] buffer, samples
// 32c .. 32c+31 (the same slot order as cat8 of two 16-wide fragments).
__device__ __forceinline__ bf16x8 staged8(const unsigned short* buf, int r0, int c)
{
    const int l = lane_id(), g4 = 4 * (l >> 4);
    const unsigned short* row = buf + (r0 + (l & 15)) * SP + 32 * c + g4;
    return cat8(*(const bf16x4*)row, *(const bf16x4*)(row + 16));
}

// One 16 x 16 tile of dW = A^T B over the 64 staged samples: rows of A
// (units) ra..ra+15, rows of B cb..cb+15; written to grad[u * ldg + k] for
// k < ncols.
__device__ __forceinline__ void weight_tile(const unsigned short* a, int ra, const unsigned short* b, int cb,
                                            float* grad, int ldg, int ncols)
{
    const int l = lane_id(), g4 = 4 * (l >> 4);
    f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
    acc = mfma32(staged8(a, ra, 0), staged8(b, cb, 0), acc);
    acc = mfma32(staged8(a, ra, 1), staged8(b, cb, 1), acc);
    const int k = cb + (l & 15);
    if (k < ncols)
#pragma unroll
        for (int i = 0; i < 4; ++i) grad[(ra + g4 + i) * ldg + k] = acc[i];
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

// Samples of steps [t0, t0 + nsteps): inputs as B fragments
// zfr[((step * nparts + part) * 4 + nb) * KB + kb][lane] and targets
// y[step * batch + s], s = part * 64 + lane (one wave per 64 samples).
template <int D>
__global__ __launch_bounds__(256) void k_mlp_sample(float kappa, const float* __restrict__ coords, long long nv,
                                                    GridGeom gg, const float* __restrict__ xh,
                                                    const mc_result* __restrict__ res, const void* __restrict__ xfield,
                                                    int dtype, long long batch, unsigned long long seed, long long t0,
                                                    long long nsteps, bf16x4* __restrict__ zfr, float* __restrict__ y)
{
    constexpr int KB = MlpShape<D>::KB;
    const long long nparts = batch / 64;
    const long long wv = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wv >= nsteps * nparts) return;
    const long long st = wv / nparts, part = wv % nparts;
    const int l = lane_id();
    const long long s = part * 64 + l;
    const unsigned long long r = splitmix64_dev(seed, (unsigned long long)((t0 + st) * batch + s));
    const long long v = (long long)(((r >> 32) * (unsigned long long)nv) >> 32);
    const VGeom mine = vertex_geom<D>(coords, nv, v, gg, xh);
    bf16x4 zf[4][KB];
    const bool valid[4] = {true, true, true, true};
    build_inputs<D>(zf, mine, true, gg, xh, kappa, valid);
    bf16x4* out = zfr + (st * nparts + part) * 4 * KB * 64;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) out[(nb * KB + kb) * 64 + l] = zf[nb][kb];
    const double inv2 = 1.0 / (2.0 * res->tau2);
    const double xv = dtype == MC_F64 ? ((const double*)xfield)[v] : (double)((const float*)xfield)[v];
    y[st * batch + s] = (float)((xv - (double)mine.g) * inv2);
}

// Given inputs z[batch][KPAD] (BF16 values) and targets -> the fragment
// layout of k_mlp_sample, zero padded to whole 64-sample parts.
template <int D>
__global__ __launch_bounds__(256) void k_mlp_zfrag(const float* __restrict__ z, const float* __restrict__ yin,
                                                   long long batch, bf16x4* __restrict__ zfr, float* __restrict__ y)
{
    constexpr int KB = MlpShape<D>::KB, KPAD = MlpShape<D>::KPAD;
    const long long wv = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wv * 64 >= batch) return;
    const int l = lane_id(), g4 = 4 * (l >> 4);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const long long sn = wv * 64 + nb * 16 + (l & 15);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            float f[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) f[i] = sn < batch ? z[sn * KPAD + kb * 16 + g4 + i] : 0.0f;
            zfr[(wv * 4 + nb) * KB * 64 + kb * 64 + l] = pack4(f[0], f[1], f[2], f[3]);
        }
    }
    const long long s = wv * 64 + l;
    y[s] = s < batch ? yin[s] : 0.0f;
}

template <int D> struct TrainLds {
    FragImg<D> w;
    bf16x4 x[2][4][4][64];                          // exchange [buffer][nb][mb][lane]
    unsigned short h1s[HID * SP], h2s[HID * SP];    // H1^T, H2^T [unit][sample]
    unsigned short zs[MlpShape<D>::KPAD * SP];      // Z^T [input][sample]
    unsigned short dzs[2][HID * SP];                // dZ^T of the current layers
    float part[4][4][HID];                          // dW4, db3, db2, db1 over 16 samples: [quantity][nb][unit]
    float dsum[4], loss[4];                         // db4 and squared error over 16 samples
};

template <int D>
__global__ __launch_bounds__(512) void k_mlp_train(const FragImg<D>* __restrict__ img,
                                                   const bf16x4* __restrict__ zfr, const float* __restrict__ y,
                                                   long long batch, float* __restrict__ grad_part,
                                                   float* __restrict__ loss_part)
{
    constexpr int KB = MlpShape<D>::KB, KC = KB / 2, KIN = MlpShape<D>::KIN;
    __shared__ TrainLds<D> S;
    const int l = lane_id(), g4 = 4 * (l >> 4), w = threadIdx.x >> 6;
    const int nb = w & 3, mh = w >> 2;
    const long long part = blockIdx.x;
    const ParamOffsets po = param_offsets<D>();
    float* grad = grad_part + part * po.n;
    const FragImg<D>& W = S.w;

    // inputs of the wave's 16 samples (issued before the weight copy)
    bf16x4 zf[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) zf[kb] = zfr[((part * 4 + nb) * KB + kb) * 64 + l];
    const long long s = part * 64 + nb * 16 + (l & 15);
    const bool ok = s < batch;
    const float yv = y[s];
    copy_to_lds<sizeof(FragImg<D>), 512>(&S.w, img);
    if (mh == 0)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) stage_frag(S.zs, kb * 16, zf[kb], nb);
    __syncthreads();

    // ---- forward: the wave's two row blocks of each layer ----
    bf16x4 h1m[2], h2m[2], h3m[2];
    {
        bf16x8 bin[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) bin[c] = cat8(zf[2 * c], zf[2 * c + 1]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int mb = 2 * mh + j;
            f32x4 acc = (f32x4){W.f.b1[mb * 16 + g4], W.f.b1[mb * 16 + g4 + 1], W.f.b1[mb * 16 + g4 + 2],
                                W.f.b1[mb * 16 + g4 + 3]};
#pragma unroll
            for (int c = 0; c < KC; ++c) acc = mfma32(W.f.w1[(mb * KC + c) * 64 + l], bin[c], acc);
            h1m[j] = relu_bf(pack4(acc[0], acc[1], acc[2], acc[3]));
            S.x[0][nb][mb][l] = h1m[j];
            stage_frag(S.h1s, mb * 16, h1m[j], nb);
        }
    }
    __syncthreads();
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const bf16x8* wf = layer == 0 ? W.f.w2 : W.f.w3;
        const float* b = layer == 0 ? W.f.b2 : W.f.b3;
        const bf16x8 bin0 = cat8(S.x[layer][nb][0][l], S.x[layer][nb][1][l]);
        const bf16x8 bin1 = cat8(S.x[layer][nb][2][l], S.x[layer][nb][3][l]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int mb = 2 * mh + j;
            f32x4 acc = (f32x4){b[mb * 16 + g4], b[mb * 16 + g4 + 1], b[mb * 16 + g4 + 2], b[mb * 16 + g4 + 3]};
            acc = mfma32(wf[(mb * 2 + 0) * 64 + l], bin0, acc);
            acc = mfma32(wf[(mb * 2 + 1) * 64 + l], bin1, acc);
            const bf16x4 h = relu_bf(pack4(acc[0], acc[1], acc[2], acc[3]));
            if (layer == 0) {
                h2m[j] = h;
                stage_frag(S.h2s, mb * 16, h, nb);
            } else {
                h3m[j] = h;
            }
            S.x[1 - layer][nb][mb][l] = h;
        }
        __syncthreads();
    }

    // ---- head, loss and dZ3 ----
    float dr;
    {
        f32x4 acc = (f32x4){W.f.b4, W.f.b4, W.f.b4, W.f.b4};
        acc = mfma32(W.f.w4f[l], cat8(S.x[0][nb][0][l], S.x[0][nb][1][l]), acc);
        acc = mfma32(W.f.w4f[64 + l], cat8(S.x[0][nb][2][l], S.x[0][nb][3][l]), acc);
        const float rho = __shfl(acc[0], l & 15, 64);      // sample l%16 of the block, in every row group
        const float e = ok ? rho - yv : 0.0f;
        dr = ok ? 2.0f * e / (float)batch : 0.0f;
        const float se = group16_sum(e * e), sd = group16_sum(dr);
        if (mh == 0 && l == 0) {
            S.loss[nb] = se;
            S.dsum[nb] = sd;
        }
    }
    f32x4 dz[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int mb = 2 * mh + j;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int u = mb * 16 + g4 + i;
            const float h = bf2f((unsigned short)h3m[j][i]);
            dz[j][i] = h > 0.0f ? W.f.w4[u] * dr : 0.0f;
            const float gw4 = group16_sum(dr * h), gb3 = group16_sum(dz[j][i]);
            if ((l & 15) == 0) {
                S.part[0][nb][u] = gw4;
                S.part[1][nb][u] = gb3;
            }
        }
        const bf16x4 f = pack4(dz[j][0], dz[j][1], dz[j][2], dz[j][3]);
        stage_frag(S.dzs[0], mb * 16, f, nb);
        S.x[1][nb][mb][l] = f;           // x[1] (H2) was last read before the previous barrier
    }
    __syncthreads();

    // ---- layers 3 and 2: dW = dZ^T H, dZ_prev = (W^T dZ) * [h_prev > 0] ----
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const unsigned short* dzcur = S.dzs[layer];
        const unsigned short* hprev = layer == 0 ? S.h2s : S.h1s;
        float* gw = grad + (layer == 0 ? po.w3 : po.w2);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int t = 2 * w + j;                       // 16 tiles over the 8 waves
            weight_tile(dzcur, (t >> 2) * 16, hprev, (t & 3) * 16, gw, HID, HID);
        }
        const bf16x8* wt = layer == 0 ? W.w3t : W.w2t;
        const int xin = 1 - layer, xout = layer;          // dZ3 in x[1] -> dZ2 in x[0]
        const bf16x8 bin0 = cat8(S.x[xin][nb][0][l], S.x[xin][nb][1][l]);
        const bf16x8 bin1 = cat8(S.x[xin][nb][2][l], S.x[xin][nb][3][l]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int mb = 2 * mh + j;
            f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
            acc = mfma32(wt[(mb * 2 + 0) * 64 + l], bin0, acc);
            acc = mfma32(wt[(mb * 2 + 1) * 64 + l], bin1, acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = mb * 16 + g4 + i;
                const bf16x4 hp = layer == 0 ? h2m[j] : h1m[j];
                dz[j][i] = bf2f((unsigned short)hp[i]) > 0.0f ? acc[i] : 0.0f;
                const float gb = group16_sum(dz[j][i]);
                if ((l & 15) == 0) S.part[2 + layer][nb][u] = gb;
            }
            const bf16x4 f = pack4(dz[j][0], dz[j][1], dz[j][2], dz[j][3]);
            stage_frag(S.dzs[1 - layer], mb * 16, f, nb);   // dzs[1 - layer] was last read two barriers ago
            if (layer == 0) S.x[xout][nb][mb][l] = f;
        }
        __syncthreads();
    }

    // ---- layer 1: dW1 = dZ1^T Z over the KPAD inputs (columns < KIN kept) ----
    for (int t = w; t < 4 * KB; t += 8) weight_tile(S.dzs[0], (t / KB) * 16, S.zs, (t % KB) * 16, grad + po.w1, KIN, KIN);
    // biases, W4 and the loss: the four 16-sample sums in a fixed order
    if (w < 4) {
        const float (&p)[4][HID] = S.part[w];
        const float v = ((p[0][l] + p[1][l]) + p[2][l]) + p[3][l];
        const int off = w == 0 ? po.w4 : (w == 1 ? po.b3 : (w == 2 ? po.b2 : po.b1));
        grad[off + l] = v;
    } else if (w == 4 && l == 0) {
        grad[po.b4] = ((S.dsum[0] + S.dsum[1]) + S.dsum[2]) + S.dsum[3];
        loss_part[part] = ((S.loss[0] + S.loss[1]) + S.loss[2]) + S.loss[3];
    }
}

// Position of parameter k in the row-major device model and the fragment
// image: writes the BF16 weight (or FP32 bias) of value p.
template <int D>
__device__ __forceinline__ void store_param(int k, float p, const ParamOffsets& o, uint16_t* w1, uint16_t* w2,
                                            uint16_t* w3, uint16_t* w4, float* b1, float* b2, float* b3, float* b4,
                                            FragImg<D>* img)
{
    constexpr int KIN = MlpShape<D>::KIN, KPAD = MlpShape<D>::KPAD, KC = MlpShape<D>::KB / 2;
    const unsigned short h = f2bf(p);
    if (k < o.b1) {
        const int u = k / KIN, c = k % KIN;
        w1[u * KPAD + c] = h;
        ((unsigned short*)img->f.w1)[frag_pos(u, c, KC)] = h;
    } else if (k < o.w2) {
        b1[k - o.b1] = p;
        img->f.b1[k - o.b1] = p;
    } else if (k < o.b2) {
        const int i = k - o.w2, u = i >> 6, c = i & 63;
        w2[i] = h;
        ((unsigned short*)img->f.w2)[frag_pos(u, c, 2)] = h;
        ((unsigned short*)img->w2t)[frag_pos(c, u, 2)] = h;
    } else if (k < o.w3) {
        b2[k - o.b2] = p;
        img->f.b2[k - o.b2] = p;
    } else if (k < o.b3) {
        const int i = k - o.w3, u = i >> 6, c = i & 63;
        w3[i] = h;
        ((unsigned short*)img->f.w3)[frag_pos(u, c, 2)] = h;
        ((unsigned short*)img->w3t)[frag_pos(c, u, 2)] = h;
    } else if (k < o.w4) {
        b3[k - o.b3] = p;
        img->f.b3[k - o.b3] = p;
    } else if (k < o.b4) {
        const int u = k - o.w4;
        w4[u] = h;
        ((unsigned short*)img->f.w4f)[head_pos(u)] = h;
        img->f.w4[u] = bf2f(h);
    } else {
        b4[0] = p;
        img->f.b4 = p;
    }
}

// Sums the per-workgroup gradient slots in a fixed order (8 waves take
// consecutive slot ranges, 8 running sums each, combined in a fixed tree);
// optionally one Adam step on the FP32 master parameters, whose new values
// go straight into the device model and its fragment image.
template <int D>
__global__ __launch_bounds__(512) void k_mlp_adam(int nparts, const float* __restrict__ grad_part,
                                                  const float* __restrict__ loss_part, float* __restrict__ grad,
                                                  float* __restrict__ loss_out, float inv_batch,
                                                  float* __restrict__ params, float* __restrict__ mom,
                                                  float* __restrict__ vel, float lr, float bc1, float bc2, int apply,
                                                  mck::MlpDev md, FragImg<D>* __restrict__ img)
{
    __shared__ float red[8][64];
    const ParamOffsets o = param_offsets<D>();
    const int l = lane_id(), w = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + l;
    const int p0 = (int)((long long)w * nparts / 8), p1 = (int)((long long)(w + 1) * nparts / 8);
    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (k < o.n) {
        int p = p0;
        for (; p + 8 <= p1; p += 8)
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = a[j] + grad_part[(long long)(p + j) * o.n + k];
#pragma unroll
        for (int j = 0; j < 7; ++j)
            if (p + j < p1) a[j] = a[j] + grad_part[(long long)(p + j) * o.n + k];
    }
    red[w][l] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    if (blockIdx.x == 0 && w == 1) {
        float ls = 0.0f;
        for (int p = l; p < nparts; p += 64) ls = ls + loss_part[p];
        ls = wave_sum(ls);
        if (l == 0) *loss_out = ls * inv_batch;
    }
    if (w != 0 || k >= o.n) return;
    const float g = (((red[0][l] + red[1][l]) + (red[2][l] + red[3][l])) +
                     ((red[4][l] + red[5][l]) + (red[6][l] + red[7][l])));
    if (grad) grad[k] = g;
    if (!apply) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mk = b1 * mom[k] + (1.0f - b1) * g;
    const float vk = b2 * vel[k] + (1.0f - b2) * (g * g);
    mom[k] = mk;
    vel[k] = vk;
    const float mh = mk / bc1, vh = vk / bc2;
    const float pk = params[k] - lr * mh / (sqrtf(vh) + eps);
    params[k] = pk;
    store_param<D>(k, pk, o, (uint16_t*)md.w1, (uint16_t*)md.w2, (uint16_t*)md.w3, (uint16_t*)md.w4, (float*)md.b1,
                   (float*)md.b2, (float*)md.b3, (float*)md.b4, img);
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

hipError_t mlp_residual(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh,
                        const void* x, int dtype, const DevBound* bnd, uint16_t* codes, uint32_t* bflags,
                        float* dbg_g, int32_t* rho_out, unsigned int* count, unsigned int* vsum, hipStream_t s)
{
    ProfScope ps("k_mlp_residual", s);
    const long long ntv = (nv + MC_TILE - 1) / MC_TILE;
    const dim3 grid((unsigned)((nv + MC_LBLOCK - 1) / MC_LBLOCK));
#define MC_MR(T, D) hipLaunchKernelGGL((k_mlp_residual<T, D>), grid, dim3(512), 0, s, m, coords, nv, gg, xh, \
                                       (const T*)x, bnd, codes, bflags, dbg_g, rho_out, count, vsum, ntv)
    if (m.dim == 2) { if (dtype == MC_F64) MC_MR(double, 2); else MC_MR(float, 2); }
    else { if (dtype == MC_F64) MC_MR(double, 3); else MC_MR(float, 3); }
#undef MC_MR
    return hipGetLastError();
}

hipError_t mlp_vdecode(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh,
                       const uint32_t* bflags, const uint16_t* codes, const int32_t* oidx, const void* oval,
                       const mc_result* res, long long vcap, void* xout, int dtype, hipStream_t s)
{
    ProfScope ps("k_mlp_vdecode", s);
    long long nb = (nv + 255) / 256;
    if (nb > 2048) nb = 2048;
    if (nb < 1) nb = 1;
#define MC_MVD(D, T) hipLaunchKernelGGL((k_mlp_vdecode<D, T>), dim3((unsigned)nb), dim3(256), 0, s, m, coords, nv, gg, \
                                        xh, bflags, codes, oidx, (const T*)oval, res, vcap, (T*)xout)
    if (m.dim == 2) { if (dtype == MC_F64) MC_MVD(2, double); else MC_MVD(2, float); }
    else { if (dtype == MC_F64) MC_MVD(3, double); else MC_MVD(3, float); }
#undef MC_MVD
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

size_t mlp_image_bytes(int dim) { return dim == 2 ? sizeof(FragImg<2>) : sizeof(FragImg<3>); }

hipError_t mlp_image(const MlpDev& m, hipStream_t s)
{
    const int n = 64 * 96;
    if (m.dim == 2)
        hipLaunchKernelGGL(k_mlp_image<2>, dim3((n + 255) / 256), dim3(256), 0, s, m, (FragImg<2>*)m.img);
    else
        hipLaunchKernelGGL(k_mlp_image<3>, dim3((n + 255) / 256), dim3(256), 0, s, m, (FragImg<3>*)m.img);
    return hipGetLastError();
}

size_t train_sample_bytes(int dim, long long batch)
{
    const long long kb = dim == 2 ? MlpShape<2>::KB : MlpShape<3>::KB;
    return (size_t)((batch + 63) / 64) * 4 * kb * 64 * 8;
}

hipError_t train_sample(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh,
                        const mc_result* res, const void* x, int dtype, long long batch, unsigned long long seed,
                        long long t0, long long nsteps, void* zfr, float* y, hipStream_t s)
{
    ProfScope ps("k_mlp_sample", s);
    const long long waves = nsteps * (batch / 64);
    dim3 grid((unsigned)((waves + 3) / 4));
    if (m.dim == 2)
        hipLaunchKernelGGL(k_mlp_sample<2>, grid, dim3(256), 0, s, m.kappa, coords, nv, gg, xh, res, x, dtype, batch,
                           seed, t0, nsteps, (bf16x4*)zfr, y);
    else
        hipLaunchKernelGGL(k_mlp_sample<3>, grid, dim3(256), 0, s, m.kappa, coords, nv, gg, xh, res, x, dtype, batch,
                           seed, t0, nsteps, (bf16x4*)zfr, y);
    return hipGetLastError();
}

hipError_t train_zfrag(int dim, const float* z, const float* y, long long batch, void* zfr, float* ypad,
                       hipStream_t s)
{
    dim3 grid((unsigned)(((batch + 63) / 64 + 3) / 4));
    if (dim == 2)
        hipLaunchKernelGGL(k_mlp_zfrag<2>, grid, dim3(256), 0, s, z, y, batch, (bf16x4*)zfr, ypad);
    else
        hipLaunchKernelGGL(k_mlp_zfrag<3>, grid, dim3(256), 0, s, z, y, batch, (bf16x4*)zfr, ypad);
    return hipGetLastError();
}

hipError_t train_grad(const MlpDev& m, const void* zfr, const float* y, long long batch, float* grad_part,
                      float* loss_part, hipStream_t s)
{
    ProfScope ps("k_mlp_train", s);
    dim3 grid((unsigned)((batch + 63) / 64));
    if (m.dim == 2)
        hipLaunchKernelGGL(k_mlp_train<2>, grid, dim3(512), 0, s, (const FragImg<2>*)m.img, (const bf16x4*)zfr, y,
                           batch, grad_part, loss_part);
    else
        hipLaunchKernelGGL(k_mlp_train<3>, grid, dim3(512), 0, s, (const FragImg<3>*)m.img, (const bf16x4*)zfr, y,
                           batch, grad_part, loss_part);
    return hipGetLastError();
}

hipError_t train_adam(const MlpDev& m, int nparts, const float* grad_part, const float* loss_part, float* grad,
                      float* loss_out, float* params, float* mom, float* vel, long long t, float lr, int apply,
                      long long batch, hipStream_t s)
{
    ProfScope ps("k_mlp_adam", s);
    const float bc1 = (float)(1.0 - pow(0.9, (double)(t > 0 ? t : 1)));
    const float bc2 = (float)(1.0 - pow(0.999, (double)(t > 0 ? t : 1)));
    const int np = n_params(m.dim);
    dim3 grid((unsigned)((np + 63) / 64));
    if (m.dim == 2)
        hipLaunchKernelGGL(k_mlp_adam<2>, grid, dim3(512), 0, s, nparts, grad_part, loss_part, grad, loss_out,
                           1.0f / (float)batch, params, mom, vel, lr, bc1, bc2, apply, m, (FragImg<2>*)m.img);
    else
        hipLaunchKernelGGL(k_mlp_adam<3>, grid, dim3(512), 0, s, nparts, grad_part, loss_part, grad, loss_out,
                           1.0f / (float)batch, params, mom, vel, lr, bc1, bc2, apply, m, (FragImg<3>*)m.img);
    return hipGetLastError();
}

}  // namespace mck
