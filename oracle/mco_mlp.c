/*
 * mco_mlp.c -- oracle of the learned residual predictor: a multilayer
 * perceptron in -> 64 -> 64 -> 64 -> 1 (ReLU) that predicts a vertex's
 * residual, in quantisation-code units, from the reconstructed grid around
 * it and its offset inside the grid cell.  The paper has no learned part;
 * this is the learned extension of the residual compressor C(x2).
 *
 * TEST INFRASTRUCTURE (see mco.h).
 *
 * Parameter layout (flat FP32, shared with the library's model format):
 *   W1[64][Kin] (output-major), b1[64], W2[64][64], b2[64], W3[64][64],
 *   b3[64], W4[64], b4[1];  Kin = 4^dim + dim.
 * Arithmetic ("mode 1"): weight matrices rounded to BF16 (RNE), inputs and
 * hidden activations BF16, products exact in FP32, sums in FP32 in
 * ascending input order, biases FP32, output FP32.  "Mode 0" is the same
 * network with no rounding at all (FP64), used for finite-difference
 * checks of the backward pass.
 */
#include "mco.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define H 64

uint64_t mco_splitmix64(uint64_t seed, uint64_t counter)
{
    /* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output number counter+1
     * of the generator whose state starts at seed. */
    uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

float mco_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return f;
    u = u + 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return f;
}

int mco_mlp_kin(int dim) { return dim == 2 ? 18 : 67; }
int mco_mlp_kpad(int dim) { return dim == 2 ? 32 : 96; }

int64_t mco_mlp_nparams(int dim)
{
    int64_t kin = mco_mlp_kin(dim);
    return H * kin + H + H * H + H + H * H + H + H + 1;
}

typedef struct {
    int64_t w1, b1, w2, b2, w3, b3, w4, b4;
} offsets;

static offsets param_offsets(int dim)
{
    int64_t kin = mco_mlp_kin(dim);
    offsets o;
    o.w1 = 0;
    o.b1 = o.w1 + H * kin;
    o.w2 = o.b1 + H;
    o.b2 = o.w2 + H * H;
    o.w3 = o.b2 + H;
    o.b3 = o.w3 + H * H;
    o.w4 = o.b3 + H;
    o.b4 = o.w4 + H;
    return o;
}

/* Kaiming-uniform initialisation from SplitMix64 counters 2^40 + k:
 * u = top 24 bits * 2^-24, w = (float)((2u - 1) * bound), bound
 * sqrt(6/fan_in) for the hidden layers and sqrt(3/fan_in) for the head;
 * biases zero. */
void mco_mlp_init(int dim, uint64_t seed, float* params)
{
    offsets o = param_offsets(dim);
    int64_t kin = mco_mlp_kin(dim);
    int64_t n = mco_mlp_nparams(dim);
    for (int64_t k = 0; k < n; ++k) {
        double bound;
        if (k < o.b1) bound = sqrt(6.0 / (double)kin);
        else if (k >= o.w2 && k < o.b2) bound = sqrt(6.0 / H);
        else if (k >= o.w3 && k < o.b3) bound = sqrt(6.0 / H);
        else if (k >= o.w4 && k < o.b4) bound = sqrt(3.0 / H);
        else { params[k] = 0.0f; continue; }
        uint64_t r = mco_splitmix64(seed, (1ull << 40) + (uint64_t)k);
        double u = (double)(r >> 40) * 0x1p-24;
        params[k] = (float)((2.0 * u - 1.0) * bound);
    }
}

static int64_t clampi(int64_t a, int64_t lo, int64_t hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* Inputs of vertex v: for the 4^dim grid nodes n = (i_d - 1 + a_d) clamped
 * to the grid (a_d in 0..3, a_0 fastest), bf16((x1'[n] - g_v) * kappa); then
 * bf16(t_d - 0.5) for each axis; zero padding up to Kpad. */
void mco_mlp_features(const float* coords, int dim, int64_t nv, const mco_grid* g,
                      const float* xhat, const float* gv, float kappa, int64_t v0,
                      int64_t count, float* z)
{
    int kpad = mco_mlp_kpad(dim);
    int side2 = dim == 3 ? 4 : 1;
    for (int64_t s = 0; s < count; ++s) {
        int64_t v = v0 + s;
        float* zz = z + s * kpad;
        int32_t idx[3];
        float t[3];
        mco_vertex_cell(coords, dim, nv, g, v, idx, t);
        int f = 0;
        for (int a2 = 0; a2 < side2; ++a2)
            for (int a1 = 0; a1 < 4; ++a1)
                for (int a0 = 0; a0 < 4; ++a0) {
                    int64_t n0 = clampi(idx[0] - 1 + a0, 0, g->n[0] - 1);
                    int64_t n1 = clampi(idx[1] - 1 + a1, 0, g->n[1] - 1);
                    int64_t n2 = dim == 3 ? clampi(idx[2] - 1 + a2, 0, g->n[2] - 1) : 0;
                    float d = xhat[n0 + g->n[0] * (n1 + g->n[1] * n2)] - gv[v];
                    zz[f++] = mco_bf16(d * kappa);
                }
        for (int d = 0; d < dim; ++d) zz[f++] = mco_bf16(t[d] - 0.5f);
        while (f < kpad) zz[f++] = 0.0f;
    }
}

/* Root mean square of (x1'[n] - g_v) over every vertex and its 4^dim
 * neighbourhood nodes, in FP64; the model's input scale is 1/rms. */
double mco_mlp_feature_rms(const float* coords, int dim, int64_t nv, const mco_grid* g,
                           const float* xhat, const float* gv)
{
    int side2 = dim == 3 ? 4 : 1;
    double acc = 0.0;
    int64_t cnt = 0;
    for (int64_t v = 0; v < nv; ++v) {
        int32_t idx[3];
        float t[3];
        mco_vertex_cell(coords, dim, nv, g, v, idx, t);
        for (int a2 = 0; a2 < side2; ++a2)
            for (int a1 = 0; a1 < 4; ++a1)
                for (int a0 = 0; a0 < 4; ++a0) {
                    int64_t n0 = clampi(idx[0] - 1 + a0, 0, g->n[0] - 1);
                    int64_t n1 = clampi(idx[1] - 1 + a1, 0, g->n[1] - 1);
                    int64_t n2 = dim == 3 ? clampi(idx[2] - 1 + a2, 0, g->n[2] - 1) : 0;
                    double d = (double)xhat[n0 + g->n[0] * (n1 + g->n[1] * n2)] - (double)gv[v];
                    acc += d * d;
                    ++cnt;
                }
    }
    return sqrt(acc / (double)cnt);
}

/* ---------------------------------------------------------------------- */

typedef struct {
    int mode;
} arith;

static double rf(const arith* a, double x) { return a->mode ? (double)(float)x : x; }
static double rb(const arith* a, double x) { return a->mode ? (double)mco_bf16((float)x) : x; }

/* Forward pass of one sample (z has Kin meaningful inputs). */
static void fwd_one(const arith* ar, int dim, const double* P, const double* z, double* h1,
                    double* h2, double* h3, double* rho)
{
    offsets o = param_offsets(dim);
    int kin = mco_mlp_kin(dim);
    for (int u = 0; u < H; ++u) {
        double acc = 0.0;
        for (int k = 0; k < kin; ++k) acc = rf(ar, acc + rb(ar, P[o.w1 + u * kin + k]) * z[k]);
        double pre = rf(ar, acc + P[o.b1 + u]);
        h1[u] = rb(ar, pre > 0.0 ? pre : 0.0);
    }
    for (int u = 0; u < H; ++u) {
        double acc = 0.0;
        for (int k = 0; k < H; ++k) acc = rf(ar, acc + rb(ar, P[o.w2 + u * H + k]) * h1[k]);
        double pre = rf(ar, acc + P[o.b2 + u]);
        h2[u] = rb(ar, pre > 0.0 ? pre : 0.0);
    }
    for (int u = 0; u < H; ++u) {
        double acc = 0.0;
        for (int k = 0; k < H; ++k) acc = rf(ar, acc + rb(ar, P[o.w3 + u * H + k]) * h2[k]);
        double pre = rf(ar, acc + P[o.b3 + u]);
        h3[u] = rb(ar, pre > 0.0 ? pre : 0.0);
    }
    double acc = 0.0;
    for (int k = 0; k < H; ++k) acc = rf(ar, acc + rb(ar, P[o.w4 + k]) * h3[k]);
    *rho = rf(ar, acc + P[o.b4]);
}

/* Mean-squared-error loss and its gradient over a batch.  The gradient
 * treats the BF16 roundings as identity (straight-through) and uses the
 * rounded activations and weights of the forward pass; ReLU'(h) = [h > 0].
 * Sums are accumulated in ascending sample order. */
static double loss_grad(const arith* ar, int dim, const double* P, const double* z,
                        int64_t zstride, int64_t batch, const double* y, double* G)
{
    offsets o = param_offsets(dim);
    int kin = mco_mlp_kin(dim);
    int64_t np = mco_mlp_nparams(dim);
    if (G) memset(G, 0, (size_t)np * sizeof(double));
    double h1[H], h2[H], h3[H], d1[H], d2[H], d3[H], rho, loss = 0.0;
    for (int64_t b = 0; b < batch; ++b) {
        const double* zb = z + b * zstride;
        fwd_one(ar, dim, P, zb, h1, h2, h3, &rho);
        double e = rho - y[b];
        loss += e * e;
        if (!G) continue;
        double dr = rf(ar, 2.0 * e / (double)batch);
        for (int k = 0; k < H; ++k) {
            G[o.w4 + k] = rf(ar, G[o.w4 + k] + dr * h3[k]);
            d3[k] = h3[k] > 0.0 ? rf(ar, dr * rb(ar, P[o.w4 + k])) : 0.0;
        }
        G[o.b4] = rf(ar, G[o.b4] + dr);
        for (int k = 0; k < H; ++k) {
            double acc = 0.0;
            for (int u = 0; u < H; ++u) acc = rf(ar, acc + d3[u] * rb(ar, P[o.w3 + u * H + k]));
            d2[k] = h2[k] > 0.0 ? acc : 0.0;
        }
        for (int u = 0; u < H; ++u) {
            for (int k = 0; k < H; ++k)
                G[o.w3 + u * H + k] = rf(ar, G[o.w3 + u * H + k] + d3[u] * h2[k]);
            G[o.b3 + u] = rf(ar, G[o.b3 + u] + d3[u]);
        }
        for (int k = 0; k < H; ++k) {
            double acc = 0.0;
            for (int u = 0; u < H; ++u) acc = rf(ar, acc + d2[u] * rb(ar, P[o.w2 + u * H + k]));
            d1[k] = h1[k] > 0.0 ? acc : 0.0;
        }
        for (int u = 0; u < H; ++u) {
            for (int k = 0; k < H; ++k)
                G[o.w2 + u * H + k] = rf(ar, G[o.w2 + u * H + k] + d2[u] * h1[k]);
            G[o.b2 + u] = rf(ar, G[o.b2 + u] + d2[u]);
        }
        for (int u = 0; u < H; ++u) {
            for (int k = 0; k < kin; ++k)
                G[o.w1 + u * kin + k] = rf(ar, G[o.w1 + u * kin + k] + d1[u] * zb[k]);
            G[o.b1 + u] = rf(ar, G[o.b1 + u] + d1[u]);
        }
    }
    return loss / (double)batch;
}

static double* to_double(const float* a, int64_t n)
{
    double* d = (double*)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) d[i] = a[i];
    return d;
}

/* Forward pass in mode 1 for a batch of padded inputs z[batch][Kpad];
 * h1..h3 ([batch][64]) may be NULL. */
void mco_mlp_forward(int dim, const float* params, const float* z, int64_t batch,
                     float* h1, float* h2, float* h3, float* rho)
{
    arith ar = {1};
    int kpad = mco_mlp_kpad(dim);
    double* P = to_double(params, mco_mlp_nparams(dim));
    double zz[96], a1[H], a2[H], a3[H], r;
    for (int64_t b = 0; b < batch; ++b) {
        for (int k = 0; k < kpad; ++k) zz[k] = z[b * kpad + k];
        fwd_one(&ar, dim, P, zz, a1, a2, a3, &r);
        for (int k = 0; k < H; ++k) {
            if (h1) h1[b * H + k] = (float)a1[k];
            if (h2) h2[b * H + k] = (float)a2[k];
            if (h3) h3[b * H + k] = (float)a3[k];
        }
        rho[b] = (float)r;
    }
    free(P);
}

/* Loss and gradient over a batch z[batch][Kpad], targets y[batch].
 * round_bf16 = 1: mode 1 arithmetic; 0: exact FP64 (mode 0). */
double mco_mlp_backward(int dim, const float* params, const float* z, int64_t batch,
                        const float* y, int round_bf16, float* grad)
{
    arith ar = {round_bf16 ? 1 : 0};
    int kpad = mco_mlp_kpad(dim);
    int64_t np = mco_mlp_nparams(dim);
    double* P = to_double(params, np);
    double* Z = to_double(z, batch * kpad);
    double* Y = to_double(y, batch);
    double* G = (double*)malloc((size_t)np * sizeof(double));
    double loss = loss_grad(&ar, dim, P, Z, kpad, batch, Y, G);
    for (int64_t k = 0; k < np; ++k) grad[k] = (float)G[k];
    free(P); free(Z); free(Y); free(G);
    return loss;
}

/* Exact (FP64, unrounded) loss and gradient for finite-difference checks. */
double mco_mlp_loss_exact(int dim, const double* params, const double* z, int64_t batch,
                          const double* y, double* grad)
{
    arith ar = {0};
    return loss_grad(&ar, dim, params, z, mco_mlp_kpad(dim), batch, y, grad);
}

/* Adam (Kingma & Ba), FP32: m = b1*m + (1-b1)*g; v = b2*v + (1-b2)*g*g;
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
void mco_adam_step(int64_t n, float* params, float* m, float* v, const float* grad,
                   int64_t t, float lr, float beta1, float beta2, float eps)
{
    float bc1 = (float)(1.0 - pow((double)beta1, (double)t));
    float bc2 = (float)(1.0 - pow((double)beta2, (double)t));
    for (int64_t k = 0; k < n; ++k) {
        m[k] = beta1 * m[k] + (1.0f - beta1) * grad[k];
        v[k] = beta2 * v[k] + (1.0f - beta2) * (grad[k] * grad[k]);
        float mh = m[k] / bc1;
        float vh = v[k] / bc2;
        params[k] = params[k] - lr * mh / (sqrtf(vh) + eps);
    }
}

/* Integer shift applied to a vertex's residual code:
 * clamp((int32) rint(rho), -(R-1), R-1); non-finite rho gives 0. */
int32_t mco_rho_quantize(float rho)
{
    double r = rint((double)rho);
    if (!(r == r) || isinf(r)) return 0;
    if (r > (double)(MCO_RADIUS - 1)) return MCO_RADIUS - 1;
    if (r < -(double)(MCO_RADIUS - 1)) return -(MCO_RADIUS - 1);
    return (int32_t)r;
}

/* Minibatch sample i of step s: vertex ((splitmix64(seed, s*batch + i) >> 32)
 * * n) >> 32, uniform with replacement. */
void mco_sample_indices(uint64_t seed, int64_t step, int64_t batch, int64_t n, int64_t* idx)
{
    for (int64_t i = 0; i < batch; ++i) {
        uint64_t r = mco_splitmix64(seed, (uint64_t)(step * batch + i));
        idx[i] = (int64_t)(((r >> 32) * (uint64_t)n) >> 32);
    }
}
