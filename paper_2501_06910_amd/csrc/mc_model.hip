// mc_model.hip -- learned residual predictor objects: creation from a
// parameter vector, serialisation, inference on a plan, GPU training.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "mc_internal.h"

static int kin_of(int dim) { return dim == 2 ? 18 : 67; }
static int kpad_of(int dim) { return dim == 2 ? 32 : 96; }

extern "C" int64_t mc_model_param_count(int32_t dim)
{
    if (dim != 2 && dim != 3) return -1;
    const int64_t kin = kin_of(dim);
    return 64 * kin + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1;
}

int mc_model_dim(mc_model m) { return m ? m->dim : 0; }

// Device copy: bf16 W1[64][kpad] (zero padded), W2, W3 [64][64], W4 [64],
// fp32 b1, b2, b3 [64], b4 [1].
static mc_status model_upload(mc_model m)
{
    const size_t nw = 64 * (size_t)m->kpad + 64 * 64 * 2 + 64;
    const size_t img_off = (nw * 2 + (64 * 3 + 4) * 4 + (size_t)mc_model_param_count(m->dim) * 4 + 255) & ~(size_t)255;
    const size_t bytes = img_off + mck::mlp_image_bytes(m->dim);
    if (!m->dev) {
        hipError_t e = hipMalloc(&m->dev, bytes);
        if (e != hipSuccess) return mc_fail(MC_ERR_NOMEM, "model upload: %s", hipGetErrorString(e));
    }
    uint16_t* w1 = (uint16_t*)m->dev;
    uint16_t* w2 = w1 + 64 * m->kpad;
    uint16_t* w3 = w2 + 64 * 64;
    uint16_t* w4 = w3 + 64 * 64;
    float* b1 = (float*)(w4 + 64);
    float* b2 = b1 + 64;
    float* b3 = b2 + 64;
    float* b4 = b3 + 64;
    float* master = b4 + 4;
    hipError_t e = hipMemcpy(master, m->params.data(), m->params.size() * 4, hipMemcpyHostToDevice);
    m->md.dim = m->dim;
    m->md.kin = m->kin;
    m->md.kpad = m->kpad;
    m->md.kappa = m->kappa;
    m->md.w1 = w1; m->md.w2 = w2; m->md.w3 = w3; m->md.w4 = w4;
    m->md.b1 = b1; m->md.b2 = b2; m->md.b3 = b3; m->md.b4 = b4;
    m->md.img = (char*)m->dev + img_off;
    if (e == hipSuccess) e = mck::mlp_pack(master, m->dim, w1, w2, w3, w4, b1, b2, b3, b4, nullptr);
    if (e == hipSuccess) e = mck::mlp_image(m->md, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "model upload: %s", hipGetErrorString(e));
    return MC_OK;
}

extern "C" mc_status mc_model_create(int32_t dim, const float* h_params, float kappa, mc_model* out)
{
    if (!out) return mc_fail(MC_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return mc_fail(MC_ERR_ARG, "dim must be 2 or 3");
    if (!h_params) return mc_fail(MC_ERR_ARG, "params is NULL");
    if (!(kappa > 0.0f) || !std::isfinite(kappa)) return mc_fail(MC_ERR_ARG, "kappa must be finite and > 0");
    const int64_t n = mc_model_param_count(dim);
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(h_params[i])) return mc_fail(MC_ERR_ARG, "non-finite parameter %lld", (long long)i);
    mc_model m = new mc_model_s();
    m->dim = dim;
    m->kin = kin_of(dim);
    m->kpad = kpad_of(dim);
    m->kappa = kappa;
    m->params.assign(h_params, h_params + n);
    mc_status st = model_upload(m);
    if (st != MC_OK) {
        mc_model_destroy(m);
        return st;
    }
    *out = m;
    return MC_OK;
}

extern "C" mc_status mc_model_destroy(mc_model m)
{
    if (!m) return MC_OK;
    mc_batch_forget(m);
    if (m->dev) hipFree(m->dev);
    delete m;
    return MC_OK;
}

extern "C" mc_status mc_model_get_params(mc_model m, float* h_params, float* kappa)
{
    if (!m) return mc_fail(MC_ERR_ARG, "model is NULL");
    if (h_params) memcpy(h_params, m->params.data(), m->params.size() * 4);
    if (kappa) *kappa = m->kappa;
    return MC_OK;
}

// Model file: "MCMLP1\0\0", i32 dim, f32 kappa, then the FP32 parameter
// vector.  The stored form of the compressed stream keeps only the BF16
// weights (what inference reads) and the FP32 biases.
static const char kMagic[8] = {'M', 'C', 'M', 'L', 'P', '1', 0, 0};

extern "C" mc_status mc_model_export(mc_model m, void* h_buf, size_t cap, size_t* written)
{
    if (!m || !written) return mc_fail(MC_ERR_ARG, "model/written is NULL");
    const size_t need = 8 + 4 + 4 + m->params.size() * 4;
    *written = need;
    if (!h_buf) return MC_OK;
    if (cap < need) return mc_fail(MC_ERR_CAPACITY, "export needs %zu bytes", need);
    char* b = (char*)h_buf;
    memcpy(b, kMagic, 8);
    int32_t d = m->dim;
    memcpy(b + 8, &d, 4);
    memcpy(b + 12, &m->kappa, 4);
    memcpy(b + 16, m->params.data(), m->params.size() * 4);
    return MC_OK;
}

extern "C" mc_status mc_model_import(const void* h_buf, size_t n, mc_model* out)
{
    if (!h_buf || !out) return mc_fail(MC_ERR_ARG, "buffer/out is NULL");
    *out = nullptr;
    const char* b = (const char*)h_buf;
    if (n < 16 || memcmp(b, kMagic, 8) != 0) return mc_fail(MC_ERR_FORMAT, "not a model file");
    int32_t d;
    float kappa;
    memcpy(&d, b + 8, 4);
    memcpy(&kappa, b + 12, 4);
    if (d != 2 && d != 3) return mc_fail(MC_ERR_FORMAT, "bad model dim");
    const int64_t np = mc_model_param_count(d);
    if (n != 16 + (size_t)np * 4) return mc_fail(MC_ERR_FORMAT, "model file size mismatch");
    std::vector<float> p((size_t)np);
    memcpy(p.data(), b + 16, (size_t)np * 4);
    mc_status st = mc_model_create(d, p.data(), kappa, out);
    return st == MC_ERR_ARG ? mc_fail(MC_ERR_FORMAT, "model file holds invalid values") : st;
}

extern "C" mc_status mc_model_forward(mc_model m, const float* d_z, int64_t batch, float* d_rho, hipStream_t s)
{
    if (!m || !d_z || !d_rho || batch < 0) return mc_fail(MC_ERR_ARG, "invalid forward arguments");
    hipError_t e = mck::mlp_forward_z(m->md, d_z, batch, d_rho, s);
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "mlp_forward: %s", hipGetErrorString(e));
    return MC_OK;
}

extern "C" mc_status mc_model_features(mc_model m, mc_plan p, const mc_codes* codes, int64_t v0, int64_t count,
                                       float* d_z, hipStream_t s)
{
    if (!m || !p || !codes || !codes->result || !d_z) return mc_fail(MC_ERR_ARG, "invalid feature arguments");
    if (m->dim != p->dim) return mc_fail(MC_ERR_ARG, "model dim does not match the plan");
    if (p->ops != MC_OPS_LINEAR) return mc_fail(MC_ERR_UNSUPPORTED, "the learned predictor needs an MC_OPS_LINEAR plan");
    if (v0 < 0 || count < 0 || v0 + count > p->nv) return mc_fail(MC_ERR_ARG, "vertex range outside the mesh");
    mc_status st = mc_plan_ensure_xh(p, s);
    if (st != MC_OK) return st;
    hipError_t e = mck::mlp_features(m->md, p->coords, p->nv, p->gg, p->xh, v0, count, d_z, s);
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "mlp_features: %s", hipGetErrorString(e));
    return MC_OK;
}

// Per-workgroup gradient partials (64 samples each) are reduced in a fixed
// order, so the gradient is the same on every run.
static int parts_of(long long batch) { return (int)((batch + 63) / 64); }

extern "C" mc_status mc_model_loss_grad(mc_model m, const float* d_z, const float* d_y, int64_t batch, float* d_grad,
                                        float* d_loss, hipStream_t s)
{
    if (!m || !d_z || !d_y || !d_grad || batch <= 0) return mc_fail(MC_ERR_ARG, "invalid loss_grad arguments");
    const int np = (int)mc_model_param_count(m->dim);
    const int nparts = parts_of(batch);
    float *gp = nullptr, *lp = nullptr, *lo = nullptr, *yp = nullptr;
    void* zf = nullptr;
    hipError_t e = hipMalloc(&gp, (size_t)nparts * np * 4);
    if (e == hipSuccess) e = hipMalloc(&lp, (size_t)nparts * 4);
    if (e == hipSuccess) e = hipMalloc(&lo, 4);
    if (e == hipSuccess) e = hipMalloc(&yp, (size_t)nparts * 64 * 4);
    if (e == hipSuccess) e = hipMalloc(&zf, mck::train_sample_bytes(m->dim, batch));
    if (e == hipSuccess) e = mck::train_zfrag(m->dim, d_z, d_y, batch, zf, yp, s);
    if (e == hipSuccess) e = mck::train_grad(m->md, zf, yp, batch, gp, lp, s);
    if (e == hipSuccess)
        e = mck::train_adam(m->md, nparts, gp, lp, d_grad, d_loss ? d_loss : lo, nullptr, nullptr, nullptr, 0, 0.f, 0,
                            batch, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(gp);
    hipFree(lp);
    hipFree(lo);
    hipFree(yp);
    hipFree(zf);
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "loss_grad: %s", hipGetErrorString(e));
    return MC_OK;
}

static void host_init(int dim, uint64_t seed, std::vector<float>& p);

extern "C" mc_status mc_model_train(mc_plan plan, const void* d_field, mc_dtype dtype, const mc_params* prm,
                                    const mc_train_opts* opts, hipStream_t s, mc_model* out)
{
    if (!out) return mc_fail(MC_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!plan) return mc_fail(MC_ERR_ARG, "plan is NULL");
    if (plan->ops != MC_OPS_LINEAR) return mc_fail(MC_ERR_UNSUPPORTED, "the learned predictor needs an MC_OPS_LINEAR plan");
    if (prm && prm->model) return mc_fail(MC_ERR_ARG, "training compresses plainly: params.model must be NULL");
    const int steps = opts && opts->steps > 0 ? opts->steps : 2000;
    const int batch = opts && opts->batch > 0 ? opts->batch : 8192;
    const float lr = opts && opts->lr > 0.f ? opts->lr : 1e-3f;
    const uint64_t seed = opts ? opts->seed : 0;
    if (batch % 64 != 0) return mc_fail(MC_ERR_ARG, "batch must be a multiple of 64");
    if (!plan->xh) return mc_fail(MC_ERR_ARG, "plan has no workspace");
    const int dim = plan->dim;
    const int np = (int)mc_model_param_count(dim);
    // 1) plain compression of the training field into scratch codes
    std::vector<void*> tmp;
    auto dalloc = [&](size_t bytes) -> void* {
        void* q = nullptr;
        if (hipMalloc(&q, bytes ? bytes : 16) != hipSuccess) return nullptr;
        tmp.push_back(q);
        return q;
    };
    auto cleanup = [&]() { for (void* q : tmp) hipFree(q); };
    const size_t tsz = dtype == MC_F64 ? 8 : 4;
    mc_codes c{};
    c.grid_codes = (uint16_t*)dalloc((size_t)plan->ng * 2);
    c.g_out_cap = plan->ng;
    c.g_out_idx = (int32_t*)dalloc((size_t)plan->ng * 4);
    c.g_out_delta = (int32_t*)dalloc((size_t)plan->ng * 4);
    c.vert_codes = (uint16_t*)dalloc((size_t)plan->nv * 2);
    c.v_out_cap = plan->nv;
    c.v_out_idx = (int32_t*)dalloc((size_t)plan->nv * 4);
    c.v_out_val = dalloc((size_t)plan->nv * tsz);
    c.result = (mc_result*)dalloc(sizeof(mc_result));
    const int nparts = parts_of(batch);
    float* gp = (float*)dalloc((size_t)nparts * np * 4);
    float* lp = (float*)dalloc((size_t)nparts * 4);
    float* dev_state = (float*)dalloc((size_t)np * 4 * 4 + 64 * 4);
    // samples of up to `chunk` steps are drawn in one launch (<= 256 MB)
    const size_t zstep = mck::train_sample_bytes(dim, batch), ystep = (size_t)batch * 4;
    int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)steps, ((size_t)256 << 20) / (zstep + ystep)));
    if (opts && opts->sample_steps > 0) chunk = std::min(steps, (int)opts->sample_steps);
    char* zbuf = (char*)dalloc(zstep * chunk);
    float* ybuf = (float*)dalloc(ystep * chunk);
    double* ssq = (double*)dalloc(2048 * 8);
    for (void* q : tmp)
        if (!q) { cleanup(); return mc_fail(MC_ERR_NOMEM, "training scratch allocation failed"); }
    mc_params pp{};
    if (prm) pp = *prm;
    else { pp.eb = 1e-4; pp.eb_mode = MC_EB_REL; pp.grid_share = 0.5; }
    pp.model = nullptr;
    mc_status st = mc_check_params(plan, d_field, dtype, &pp, &c);
    if (st != MC_OK) { cleanup(); return st; }
    if ((st = mc_compress_enqueue(plan, d_field, dtype, &pp, &c, s)) != MC_OK) { cleanup(); return st; }
    if ((st = mc_plan_ensure_xh(plan, s)) != MC_OK) { cleanup(); return st; }
    // 2) input scale: 1 / rms of (x1'[n] - g) over vertices and neighbourhoods
    hipError_t e = mck::mlp_feature_sumsq(plan->coords, plan->nv, plan->gg, plan->xh, dim, ssq, 1024, s);
    std::vector<double> h(2048);
    mc_result hres{};
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), ssq, 2048 * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&hres, c.result, sizeof hres, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { cleanup(); return mc_fail(MC_ERR_DEVICE, "training setup: %s", hipGetErrorString(e)); }
    if (hres.status != MC_OK) { cleanup(); return mc_fail((mc_status)hres.status, "plain compression of the training field failed"); }
    double sum = 0.0, cnt = 0.0;
    for (int k = 0; k < 1024; ++k) { sum += h[2 * k]; cnt += h[2 * k + 1]; }
    const double rms = cnt > 0 ? std::sqrt(sum / cnt) : 0.0;
    const float kappa = rms > 0.0 && std::isfinite(rms) ? (float)(1.0 / rms) : 1.0f;
    // 3) model with a seeded initialisation, Adam state on the device
    std::vector<float> init((size_t)np);
    host_init(dim, seed, init);
    mc_model m = nullptr;
    if ((st = mc_model_create(dim, init.data(), kappa, &m)) != MC_OK) { cleanup(); return st; }
    float* master = (float*)((char*)m->dev + (64 * (size_t)m->kpad + 64 * 64 * 2 + 64) * 2 + (64 * 3 + 4) * 4);
    float* am = dev_state;
    float* av = dev_state + np;
    float* grad = dev_state + 2 * np;
    float* loss = dev_state + 3 * np;
    e = hipMemsetAsync(am, 0, (size_t)np * 2 * 4, s);
    for (int t = 0; t < steps && e == hipSuccess; ++t) {
        const int tc = t % chunk;
        if (tc == 0)
            e = mck::train_sample(m->md, plan->coords, plan->nv, plan->gg, plan->xh, c.result, d_field, dtype, batch,
                                  seed, t, std::min(chunk, steps - t), zbuf, ybuf, s);
        if (e == hipSuccess) e = mck::train_grad(m->md, zbuf + zstep * tc, ybuf + (size_t)batch * tc, batch, gp, lp, s);
        if (e == hipSuccess)
            e = mck::train_adam(m->md, nparts, gp, lp, grad, loss + (t % 64), master, am, av, t + 1, lr, 1, batch, s);
        if (e == hipSuccess && opts && opts->h_loss_out && (t % 64 == 63 || t == steps - 1)) {
            const int first = t - (t % 64);
            e = hipMemcpyAsync(opts->h_loss_out + first, loss, (size_t)(t - first + 1) * 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(m->params.data(), master, (size_t)np * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) {
        mc_model_destroy(m);
        return mc_fail(MC_ERR_DEVICE, "training: %s", hipGetErrorString(e));
    }
    *out = m;
    return MC_OK;
}

// Kaiming-uniform initialisation from SplitMix64 (Steele, Lea, Flood 2014)
// counters 2^40 + k: bound sqrt(6/fan_in) for the hidden layers, sqrt(3/64)
// for the head, zero biases.
static uint64_t splitmix64_at(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void host_init(int dim, uint64_t seed, std::vector<float>& p)
{
    const int64_t kin = kin_of(dim);
    const int64_t w1 = 0, b1 = 64 * kin, w2 = b1 + 64, b2 = w2 + 4096, w3 = b2 + 64, b3 = w3 + 4096, w4 = b3 + 64,
                  b4 = w4 + 64;
    for (int64_t k = 0; k < (int64_t)p.size(); ++k) {
        double bound;
        if (k >= w1 && k < b1) bound = std::sqrt(6.0 / (double)kin);
        else if ((k >= w2 && k < b2) || (k >= w3 && k < b3)) bound = std::sqrt(6.0 / 64.0);
        else if (k >= w4 && k < b4) bound = std::sqrt(3.0 / 64.0);
        else { p[k] = 0.0f; continue; }
        const uint64_t r = splitmix64_at(seed, (1ull << 40) + (uint64_t)k);
        const double u = (double)(r >> 40) * 0x1p-24;
        p[k] = (float)((2.0 * u - 1.0) * bound);
    }
}

// Batched compression and decompression (HIP graphs of per-stage work-list
// launches) are in mc_batch.hip.
