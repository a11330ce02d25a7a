// mc_api.hip -- host side of the C ABI declared in include/mc.h: argument
// validation (before any HIP call), plan construction, the compress and
// decompress sequences, models, batching and the kernel profiler.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "mc_internal.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

mc_status mc_fail(mc_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

extern "C" const char* mc_last_error(void) { return g_last_error.c_str(); }
extern "C" int32_t mc_abi_version(void) { return 1; }

extern "C" const char* mc_status_string(mc_status s)
{
    switch (s) {
    case MC_OK: return "ok";
    case MC_ERR_ARG: return "invalid argument";
    case MC_ERR_RANGE: return "error bound too small for the data range";
    case MC_ERR_CAPACITY: return "outlier capacity exceeded";
    case MC_ERR_NOMEM: return "device allocation failed";
    case MC_ERR_DEVICE: return "HIP call failed";
    case MC_ERR_FORMAT: return "malformed serialized data";
    case MC_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

// ---------------------------------------------------------------------------
// profiler: HIP events around each launch, on the launch stream
// ---------------------------------------------------------------------------
namespace {
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_pm;
bool g_prof_on = false;
std::string g_prof_only;        // empty: every kernel; else only launches of this name
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t pool_get()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence at record, which would write back
    // and invalidate the caches between the launch and its neighbours
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

mck::ProfScope::ProfScope(const char* n, hipStream_t s) : name(n), stream(s), idx(-1)
{
    if (!g_prof_on || mc_capturing) return;
    std::lock_guard<std::mutex> lk(g_pm);
    if (!g_prof_only.empty() && g_prof_only != n) return;
    hipEvent_t a = pool_get(), b = pool_get();
    if (!a || !b) return;
    (void)hipEventRecord(a, s);
    idx = (int)g_recs.size();
    g_recs.push_back({n, a, b});
}

mck::ProfScope::~ProfScope()
{
    if (idx < 0) return;
    std::lock_guard<std::mutex> lk(g_pm);
    (void)hipEventRecord(g_recs[idx].b, stream);
}

namespace {
struct ProfAgg {
    const char* name;
    long long count;
    double ms;
};
std::vector<ProfAgg> g_agg;

void prof_drain()
{
    for (auto& r : g_recs) {
        (void)hipEventSynchronize(r.b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        bool found = false;
        for (auto& a : g_agg)
            if (strcmp(a.name, r.name) == 0) { a.count++; a.ms += ms; found = true; break; }
        if (!found) g_agg.push_back({r.name, 1, (double)ms});
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
}
}  // namespace

extern "C" mc_status mc_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_pm);
    g_prof_on = on != 0;
    return MC_OK;
}

extern "C" mc_status mc_profile_only(const char* name)
{
    std::lock_guard<std::mutex> lk(g_pm);
    g_prof_only = name ? name : "";
    return MC_OK;
}

extern "C" mc_status mc_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_pm);
    prof_drain();
    g_agg.clear();
    return MC_OK;
}

extern "C" int32_t mc_profile_read(const char** names, int64_t* counts, double* total_ms, int32_t cap)
{
    std::lock_guard<std::mutex> lk(g_pm);
    prof_drain();
    int32_t n = 0;
    for (auto& a : g_agg) {
        if (n >= cap) break;
        if (names) names[n] = a.name;
        if (counts) counts[n] = a.count;
        if (total_ms) total_ms[n] = a.ms;
        ++n;
    }
    return n;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
struct TempAllocs {
    std::vector<void*> ptrs;
    ~TempAllocs()
    {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T> T* get(size_t n, hipError_t& err)
    {
        void* p = nullptr;
        err = hipMalloc(&p, n * sizeof(T) > 0 ? n * sizeof(T) : 16);
        if (err != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return (T*)p;
    }
};

template <typename T> static hipError_t plan_alloc(mc_plan p, T** out, size_t n)
{
    void* q = nullptr;
    size_t bytes = n * sizeof(T) > 0 ? n * sizeof(T) : 16;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return e;
    p->allocs.push_back(q);
    p->bytes += bytes;
    *out = (T*)q;
    return hipSuccess;
}

static float fkey_inv(unsigned k)
{
    unsigned b = (k >> 31) ? (k & 0x7fffffffu) : ~k;
    float f;
    memcpy(&f, &b, 4);
    return f;
}

static mc_status device_bbox(const float* d_coords, int dim, long long nv, hipStream_t s, float lo[3], float hi[3])
{
    unsigned init[6] = {~0u, 0u, ~0u, 0u, ~0u, 0u};
    TempAllocs ta;
    hipError_t e;
    unsigned* keys = ta.get<unsigned>(6, e);
    if (!keys) return mc_fail(MC_ERR_NOMEM, "bbox keys: %s", hipGetErrorString(e));
    if ((e = hipMemcpyAsync(keys, init, sizeof init, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = mck::bbox(d_coords, dim, nv, keys, s)) != hipSuccess ||
        (e = hipMemcpyAsync(init, keys, sizeof init, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return mc_fail(MC_ERR_DEVICE, "bbox: %s", hipGetErrorString(e));
    for (int d = 0; d < 3; ++d) {
        lo[d] = d < dim ? fkey_inv(init[2 * d]) : 0.f;
        hi[d] = d < dim ? fkey_inv(init[2 * d + 1]) : 0.f;
    }
    return MC_OK;
}

static mc_status check_mesh_args(const float* d_coords, int32_t dim, int64_t nv)
{
    if (!d_coords) return mc_fail(MC_ERR_ARG, "coordinates pointer is NULL");
    if (dim != 2 && dim != 3) return mc_fail(MC_ERR_ARG, "dim must be 2 or 3 (got %d)", dim);
    if (nv <= 0 || nv >= (1ll << 31)) return mc_fail(MC_ERR_ARG, "n_vertices must be in [1, 2^31) (got %lld)", (long long)nv);
    return MC_OK;
}

extern "C" mc_status mc_grid_from_dims(const float* d_coords, int32_t dim, int64_t n_vertices, const int64_t dims[3],
                                       hipStream_t stream, mc_grid* out)
{
    mc_status st = check_mesh_args(d_coords, dim, n_vertices);
    if (st != MC_OK) return st;
    if (!dims || !out) return mc_fail(MC_ERR_ARG, "dims/out pointer is NULL");
    for (int d = 0; d < dim; ++d)
        if (dims[d] < 2) return mc_fail(MC_ERR_ARG, "grid dims must be >= 2 on every axis");
    float lo[3], hi[3];
    if ((st = device_bbox(d_coords, dim, n_vertices, stream, lo, hi)) != MC_OK) return st;
    memset(out, 0, sizeof *out);
    out->dim = dim;
    for (int d = 0; d < 3; ++d) {
        if (d < dim) {
            if (!(hi[d] > lo[d])) return mc_fail(MC_ERR_ARG, "mesh has zero extent along axis %d", d);
            out->dims[d] = dims[d];
            out->origin[d] = (double)lo[d];
            out->spacing[d] = ((double)hi[d] - (double)lo[d]) / (double)(dims[d] - 1);
        } else {
            out->dims[d] = 1;
            out->origin[d] = 0.0;
            out->spacing[d] = 1.0;
        }
    }
    return MC_OK;
}

extern "C" mc_status mc_grid_from_spacing(const float* d_coords, int32_t dim, int64_t n_vertices,
                                          const double spacing[3], hipStream_t stream, mc_grid* out)
{
    mc_status st = check_mesh_args(d_coords, dim, n_vertices);
    if (st != MC_OK) return st;
    if (!spacing || !out) return mc_fail(MC_ERR_ARG, "spacing/out pointer is NULL");
    for (int d = 0; d < dim; ++d)
        if (!(spacing[d] > 0.0) || !std::isfinite(spacing[d])) return mc_fail(MC_ERR_ARG, "spacing must be > 0");
    float lo[3], hi[3];
    if ((st = device_bbox(d_coords, dim, n_vertices, stream, lo, hi)) != MC_OK) return st;
    memset(out, 0, sizeof *out);
    out->dim = dim;
    for (int d = 0; d < 3; ++d) {
        if (d < dim) {
            double n = std::ceil(((double)hi[d] - (double)lo[d]) / spacing[d]) + 1.0;
            if (n < 2.0) n = 2.0;
            if (n > 2147483647.0) return mc_fail(MC_ERR_ARG, "grid too large");
            out->dims[d] = (int64_t)n;
            out->origin[d] = (double)lo[d];
            out->spacing[d] = spacing[d];
        } else {
            out->dims[d] = 1;
            out->origin[d] = 0.0;
            out->spacing[d] = 1.0;
        }
    }
    return MC_OK;
}

// Exact k-th smallest (1-based rank r) FP32 edge extent along one axis by a
// three-pass radix select; hist0 holds the first pass's histogram.
static mc_status edge_select(const float* d_coords, const int32_t* d_cells, int dim, long long nv, long long nc,
                             int axis, const std::vector<unsigned long long>& hist0, unsigned long long r,
                             unsigned long long* d_hist, unsigned* d_bad, hipStream_t s, float* out)
{
    static const unsigned shifts[3] = {21u, 10u, 0u}, nbits[3] = {11u, 11u, 10u};
    unsigned prefix = 0u, pmask = 0u;
    std::vector<unsigned long long> h(2048);
    for (int pass = 0; pass < 3; ++pass) {
        const unsigned nb = 1u << nbits[pass];
        if (pass == 0) {
            h = hist0;
        } else {
            hipError_t e;
            if ((e = hipMemsetAsync(d_hist, 0, sizeof(unsigned long long) * nb, s)) != hipSuccess ||
                (e = mck::edge_hist(d_coords, d_cells, dim, nv, nc, axis, shifts[pass], nbits[pass], pmask, prefix,
                                    d_hist, d_bad, s)) != hipSuccess ||
                (e = hipMemcpyAsync(h.data(), d_hist, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost, s)) !=
                    hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return mc_fail(MC_ERR_DEVICE, "edge histogram: %s", hipGetErrorString(e));
        }
        unsigned long long cum = 0;
        unsigned b = 0;
        for (; b < nb; ++b) {
            if (cum + h[b] >= r) break;
            cum += h[b];
        }
        if (b == nb) return mc_fail(MC_ERR_DEVICE, "edge histogram lost counts");
        r -= cum;
        prefix |= b << shifts[pass];
        pmask |= (nb - 1u) << shifts[pass];
    }
    memcpy(out, &prefix, sizeof(float));
    return MC_OK;
}

extern "C" mc_status mc_grid_from_percentile(const float* d_coords, const int32_t* d_cells, int32_t dim,
                                             int64_t n_vertices, int64_t n_cells, double k_percent, int64_t g_max,
                                             hipStream_t stream, mc_grid* out, double k_used[3])
{
    mc_status st = check_mesh_args(d_coords, dim, n_vertices);
    if (st != MC_OK) return st;
    if (!d_cells || !out) return mc_fail(MC_ERR_ARG, "cells/out pointer is NULL");
    if (n_cells <= 0 || n_cells >= (1ll << 31)) return mc_fail(MC_ERR_ARG, "n_cells must be in [1, 2^31)");
    if (!(k_percent >= 0.0) || !(k_percent <= 100.0)) return mc_fail(MC_ERR_ARG, "k_percent must be in [0, 100]");
    if (g_max < 2) return mc_fail(MC_ERR_ARG, "g_max must be >= 2");
    float lo[3], hi[3];
    if ((st = device_bbox(d_coords, dim, n_vertices, stream, lo, hi)) != MC_OK) return st;
    const unsigned long long N = (unsigned long long)n_cells * (dim == 2 ? 3u : 6u);
    TempAllocs ta;
    hipError_t e = hipSuccess;
    unsigned long long* d_hist = ta.get<unsigned long long>(2048, e);
    if (e != hipSuccess) return mc_fail(MC_ERR_NOMEM, "histogram: %s", hipGetErrorString(e));
    unsigned* d_bad = ta.get<unsigned>(1, e);
    if (e != hipSuccess) return mc_fail(MC_ERR_NOMEM, "flag: %s", hipGetErrorString(e));
    if ((e = hipMemsetAsync(d_bad, 0, sizeof(unsigned), stream)) != hipSuccess)
        return mc_fail(MC_ERR_DEVICE, "memset: %s", hipGetErrorString(e));
    mc_grid g{};
    g.dim = dim;
    for (int d = 0; d < 3; ++d) {
        g.dims[d] = 1;
        g.origin[d] = 0.0;
        g.spacing[d] = 1.0;
        if (k_used) k_used[d] = 0.0;
    }
    for (int d = 0; d < dim; ++d) {
        std::vector<unsigned long long> hist0(2048);
        unsigned bad = 0;
        if ((e = hipMemsetAsync(d_hist, 0, sizeof(unsigned long long) * 2048, stream)) != hipSuccess ||
            (e = mck::edge_hist(d_coords, d_cells, dim, n_vertices, n_cells, d, 21u, 11u, 0u, 0u, d_hist, d_bad,
                                stream)) != hipSuccess ||
            (e = hipMemcpyAsync(hist0.data(), d_hist, sizeof(unsigned long long) * 2048, hipMemcpyDeviceToHost,
                                stream)) != hipSuccess ||
            (e = hipMemcpyAsync(&bad, d_bad, sizeof bad, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return mc_fail(MC_ERR_DEVICE, "edge histogram: %s", hipGetErrorString(e));
        if (bad) return mc_fail(MC_ERR_ARG, "cells reference a vertex id outside [0, n_vertices)");
        const double extent = (double)hi[d] - (double)lo[d];
        double k = k_percent, gs = 0.0;
        for (;;) {
            double r = std::ceil((k * (double)N) / 100.0);
            if (r < 1.0) r = 1.0;
            if (r > (double)N) r = (double)N;
            float v;
            if ((st = edge_select(d_coords, d_cells, dim, n_vertices, n_cells, d, hist0, (unsigned long long)r,
                                  d_hist, d_bad, stream, &v)) != MC_OK)
                return st;
            gs = (double)v;
            if (extent / gs < (double)g_max) break;          // also false when gs = 0
            if (k >= 100.0) return mc_fail(MC_ERR_ARG, "axis %d: even the largest edge extent gives >= g_max nodes", d);
            k = k + 1.0 > 100.0 ? 100.0 : k + 1.0;
        }
        double nd = std::ceil(extent / gs) + 1.0;
        if (nd < 2.0) nd = 2.0;
        g.dims[d] = (int64_t)nd;
        g.origin[d] = (double)lo[d];
        g.spacing[d] = gs;
        if (k_used) k_used[d] = k;
    }
    *out = g;
    return MC_OK;
}

mc_status mc_check_grid(const mc_grid* g, int32_t dim)
{
    if (!g) return mc_fail(MC_ERR_ARG, "grid pointer is NULL");
    if (g->dim != dim) return mc_fail(MC_ERR_ARG, "grid dim %d does not match mesh dim %d", g->dim, dim);
    long long ng = 1;
    for (int d = 0; d < 3; ++d) {
        if (d < dim) {
            if (g->dims[d] < 2) return mc_fail(MC_ERR_ARG, "grid dims must be >= 2 on axis %d", d);
            if (!(g->spacing[d] > 0.0) || !std::isfinite(g->spacing[d]) || !std::isfinite(g->origin[d]))
                return mc_fail(MC_ERR_ARG, "grid spacing/origin invalid on axis %d", d);
        } else if (g->dims[d] != 1) {
            return mc_fail(MC_ERR_ARG, "unused grid axis %d must have dims 1", d);
        }
        ng *= g->dims[d];
        if (ng >= (1ll << 31)) return mc_fail(MC_ERR_ARG, "grid has 2^31 or more nodes");
    }
    if (g->dims[0] > 8192) return mc_fail(MC_ERR_UNSUPPORTED, "grid dims[0] > 8192 is not supported");
    return MC_OK;
}

GridGeom mc_geom(const mc_grid& g)
{
    GridGeom gg;
    gg.dim = g.dim;
    gg.n0 = (int)g.dims[0];
    gg.n1 = (int)g.dims[1];
    gg.n2 = (int)g.dims[2];
    for (int d = 0; d < 3; ++d) {
        gg.of[d] = (float)g.origin[d];
        gg.hf[d] = (float)g.spacing[d];
        gg.ihf[d] = (float)(1.0 / g.spacing[d]);
    }
    return gg;
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
#define PCHK(expr)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            mc_plan_destroy(p);                                                            \
            return mc_fail(e_ == hipErrorOutOfMemory ? MC_ERR_NOMEM : MC_ERR_DEVICE, "%s: %s", \
                           #expr, hipGetErrorString(e_));                                  \
        }                                                                                  \
    } while (0)

static void decode_ws_shape(mc_plan p)
{
    const long long n0 = p->grid.dims[0], n1 = p->grid.dims[1], n2 = p->grid.dims[2];
    p->dws.fast3 = p->dim == 3 && n0 <= 1024;
    p->dws.pitch = (int)(p->dws.fast3 ? (n0 + 3) / 4 * 4 : n0);
    if (p->dws.fast3) {
        p->dws.rows = MC_DY_ROWS;
        p->dws.nyc = (int)((n1 + MC_DY_ROWS - 1) / MC_DY_ROWS);
        p->dws.ntiles_xy = (long long)p->dws.nyc * n2;
        p->dws.zplanes = MC_DZ_PLANES;
        p->dws.nzc = (int)((n2 + MC_DZ_PLANES - 1) / MC_DZ_PLANES);
        return;
    }
    long long rows;
    if (p->dim == 2) {
        rows = MC_D2_R;                     // rows per chunk of the row-segment decoder
    } else {
        long long cx = 1;                     // columns per thread of the z pass, as instantiated
        while (cx * 256 < n0) cx *= 2;
        rows = 32 / cx;                       // registers of the z pass: rows * cx <= 32
        if (rows > 16) rows = 16;
    }
    if (rows > n1) rows = n1;
    if (rows < 1) rows = 1;
    p->dws.rows = (int)rows;
    p->dws.nyc = (int)((n1 + rows - 1) / rows);
    p->dws.ntiles_xy = (long long)p->dws.nyc * n2;
    p->dws.zplanes = 1;
    p->dws.nzc = 0;
    if (p->dim == 3) {
        long long nzc = (1024 + p->dws.nyc - 1) / p->dws.nyc;    // about 1024 workgroup tiles
        if (nzc > n2) nzc = n2;
        const long long zp = (n2 + nzc - 1) / nzc;
        p->dws.zplanes = (int)zp;
        p->dws.nzc = (int)((n2 + zp - 1) / zp);
    }
}

// Nearest node of every vertex and each node's vertex list in ascending id
// order (the cluster-mean f sums in that order).
static mc_status build_cluster_map(mc_plan p, hipStream_t s)
{
    const long long nv = p->nv;
    long long ng = p->ng;
    hipError_t e = hipSuccess;
#define CCHK(expr)                                                                                   \
    do {                                                                                             \
        if ((e = (expr)) != hipSuccess)                                                              \
            return mc_fail(e == hipErrorOutOfMemory ? MC_ERR_NOMEM : MC_ERR_DEVICE, "%s: %s", #expr, \
                           hipGetErrorString(e));                                                    \
    } while (0)
    CCHK(plan_alloc(p, &p->m, (size_t)nv));
    CCHK(plan_alloc(p, &p->vlist, (size_t)nv));
    CCHK(plan_alloc(p, &p->noff, (size_t)ng + 1));
    CCHK(plan_alloc(p, &p->x1, (size_t)ng));
    TempAllocs ta;
    unsigned* cnt = ta.get<unsigned>((size_t)ng, e);
    CCHK(e);
    unsigned* ctr = ta.get<unsigned>(16, e);
    CCHK(e);
    const long long nscan_tiles = (ng + MC_TILE - 1) / MC_TILE + 1;
    unsigned long long* sst = ta.get<unsigned long long>((size_t)nscan_tiles, e);
    CCHK(e);
    uint32_t* keys = ta.get<uint32_t>((size_t)nv, e);
    CCHK(e);
    CCHK(hipMemsetAsync(cnt, 0, sizeof(unsigned) * ng, s));
    CCHK(hipMemsetAsync(ctr, 0, sizeof(unsigned) * 16, s));
    CCHK(hipMemsetAsync(sst, 0, sizeof(unsigned long long) * nscan_tiles, s));
    mck::NodeGeom geo;
    for (int d = 0; d < 3; ++d) {
        geo.o[d] = p->grid.origin[d];
        geo.h[d] = p->grid.spacing[d];
        geo.n[d] = p->grid.dims[d];
    }
    CCHK(mck::nearest_nodes(p->coords, p->dim, nv, geo, p->m, cnt, s));
    if (p->coarsen) {
        // Grid_Coarsen (Alg. 2): drop the planes no node lies in, renumber
        // the nodes on the coarsened grid and count them again
        const int n0 = (int)p->grid.dims[0], n1 = (int)p->grid.dims[1], n2 = (int)p->grid.dims[2];
        const long long nf = (long long)n0 + n1 + n2;
        int* flags = ta.get<int>((size_t)nf, e);
        CCHK(e);
        CCHK(hipMemsetAsync(flags, 0, sizeof(int) * nf, s));
        CCHK(mck::mark_planes(p->m, nv, n0, n1, n2, flags, s));
        std::vector<int32_t> hf((size_t)nf);
        CCHK(hipMemcpyAsync(hf.data(), flags, sizeof(int) * nf, hipMemcpyDeviceToHost, s));
        CCHK(hipStreamSynchronize(s));
        const long long off[3] = {0, n0, (long long)n0 + n1};
        long long nn[3];
        for (int d = 0; d < 3; ++d) {
            const long long n = p->grid.dims[d];
            long long kept = 0;
            for (long long i = 0; i < n; ++i) kept += hf[off[d] + i];
            if (kept < 2 && n >= 2)                       // fewer than two planes: the axis stays whole
                for (long long i = 0; i < n; ++i) hf[off[d] + i] = 1;
            long long next = 0;
            for (long long i = 0; i < n; ++i) hf[off[d] + i] = hf[off[d] + i] ? (int32_t)next++ : -1;
            nn[d] = next;
        }
        ng = nn[0] * nn[1] * nn[2];
        CCHK(hipMemcpyAsync(flags, hf.data(), sizeof(int) * nf, hipMemcpyHostToDevice, s));
        CCHK(hipMemsetAsync(cnt, 0, sizeof(unsigned) * ng, s));
        CCHK(mck::remap_nodes(p->m, nv, n0, n1, flags, (int)nn[0], (int)nn[1], cnt, s));
        CCHK(hipStreamSynchronize(s));                    // hf is read by the copy above
        p->keep = std::move(hf);
        for (int d = 0; d < 3; ++d) p->grid.dims[d] = nn[d];
        p->ng = ng;
        p->gg = mc_geom(p->grid);
    }
    CCHK(mck::scan_u32(cnt, ng, p->noff, sst, ctr + 3, s));
    CCHK(mck::count_empty(cnt, ng, ctr + 1, s));
    size_t tb = 0;
    CCHK(mck::sort_by_node(p->m, nv, ng, keys, p->vlist, nullptr, &tb, s));
    void* tmp = ta.get<unsigned char>(tb, e);
    CCHK(e);
    CCHK(mck::sort_by_node(p->m, nv, ng, keys, p->vlist, tmp, &tb, s));
    unsigned hctr[16];
    CCHK(hipMemcpyAsync(hctr, ctr, sizeof hctr, hipMemcpyDeviceToHost, s));
    CCHK(hipStreamSynchronize(s));
    p->n_unresolved = hctr[1];
#undef CCHK
    return MC_OK;
}

extern "C" mc_status mc_plan_create(const float* d_coords, const int32_t* d_cells, int32_t dim, int64_t n_vertices,
                                    int64_t n_cells, const mc_grid* grid, const mc_plan_opts* opts,
                                    hipStream_t stream, mc_plan* out)
{
    if (!out) return mc_fail(MC_ERR_ARG, "out pointer is NULL");
    *out = nullptr;
    mc_status st = check_mesh_args(d_coords, dim, n_vertices);
    if (st != MC_OK) return st;
    const int ops = opts ? opts->operators : MC_OPS_LINEAR;
    if (ops != MC_OPS_LINEAR && ops != MC_OPS_CLUSTER) return mc_fail(MC_ERR_ARG, "unknown operator pair");
    const int coarsen = opts ? opts->coarsen : 0;
    if (coarsen != 0 && coarsen != 1) return mc_fail(MC_ERR_ARG, "coarsen must be 0 or 1");
    if (coarsen && ops != MC_OPS_CLUSTER)
        return mc_fail(MC_ERR_UNSUPPORTED, "Grid_Coarsen needs the nearest-node pair (MC_OPS_CLUSTER)");
    if (ops == MC_OPS_LINEAR) {
        if (!d_cells) return mc_fail(MC_ERR_ARG, "cells pointer is NULL");
        if (n_cells <= 0 || n_cells >= (1ll << 31)) return mc_fail(MC_ERR_ARG, "n_cells must be in [1, 2^31)");
    } else if (n_cells < 0 || n_cells >= (1ll << 31)) {
        return mc_fail(MC_ERR_ARG, "n_cells must be in [0, 2^31)");
    }
    if ((st = mc_check_grid(grid, dim)) != MC_OK) return st;
    mc_fill fill = opts ? opts->fill : MC_FILL_NEAREST;
    if (fill != MC_FILL_NEAREST && fill != MC_FILL_MIDRANGE) return mc_fail(MC_ERR_ARG, "unknown fill mode");
    int B = opts && opts->bin_nodes > 0 ? opts->bin_nodes : 1;
    if (B > 64) return mc_fail(MC_ERR_ARG, "bin_nodes must be <= 64");

    mc_plan p = new mc_plan_s();
    p->dim = dim;
    p->nv = n_vertices;
    p->nc = n_cells;
    p->grid = *grid;
    p->gg = mc_geom(*grid);
    p->ng = grid->dims[0] * grid->dims[1] * grid->dims[2];
    p->fill = fill;
    p->B = B;
    p->ops = ops;
    p->coarsen = coarsen;
    const long long ng = p->ng, nv = p->nv, nc = p->nc;
    hipStream_t s = stream;

    PCHK(plan_alloc(p, &p->coords, (size_t)dim * nv));
    PCHK(hipMemcpyAsync(p->coords, d_coords, sizeof(float) * dim * nv, hipMemcpyDeviceToDevice, s));
    if (ops == MC_OPS_CLUSTER) {
        mc_status cs = build_cluster_map(p, s);
        if (cs != MC_OK) {
            mc_plan_destroy(p);
            return cs;
        }
    } else {
        PCHK(plan_alloc(p, &p->vid, (size_t)(dim + 1) * ng));
        PCHK(plan_alloc(p, &p->w, (size_t)(dim + 1) * ng));
        PCHK(plan_alloc(p, &p->cell, (size_t)ng));

        {
            TempAllocs ta;
            hipError_t e = hipSuccess;
            const int nb0 = (int)((grid->dims[0] + B - 1) / B), nb1 = (int)((grid->dims[1] + B - 1) / B),
                      nb2 = (int)((grid->dims[2] + B - 1) / B);
            const long long nbins = (long long)nb0 * nb1 * nb2;
            unsigned* cnt = ta.get<unsigned>(nbins + 4, e);
            PCHK(e);
            unsigned* ctr = ta.get<unsigned>(16, e);     // [0] bad cells, [1] unresolved, [2] near-degenerate, [3] ticket
            PCHK(e);
            long long* start = ta.get<long long>(nbins + 1, e);
            PCHK(e);
            const long long nscan_tiles = (nbins + MC_TILE - 1) / MC_TILE + 1;
            unsigned long long* sst = ta.get<unsigned long long>(nscan_tiles, e);
            PCHK(e);
            PCHK(hipMemsetAsync(cnt, 0, sizeof(unsigned) * nbins, s));
            PCHK(hipMemsetAsync(ctr, 0, sizeof(unsigned) * 16, s));
            PCHK(hipMemsetAsync(sst, 0, sizeof(unsigned long long) * nscan_tiles, s));
            PCHK(mck::bins_count(p->coords, d_cells, dim, nv, nc, p->gg, grid->origin, grid->spacing, B, nb0, nb1, nb2,
                                 cnt, ctr + 0, s));
            PCHK(mck::scan_u32(cnt, nbins, start, sst, ctr + 3, s));
            long long total = 0;
            unsigned hctr[16];
            PCHK(hipMemcpyAsync(&total, start + nbins, sizeof total, hipMemcpyDeviceToHost, s));
            PCHK(hipMemcpyAsync(hctr, ctr, sizeof hctr, hipMemcpyDeviceToHost, s));
            PCHK(hipStreamSynchronize(s));
            if (hctr[0] != 0) {
                p->invalid_cells = (int)hctr[0];
                mc_plan_destroy(p);
                return mc_fail(MC_ERR_ARG, "%u cells reference a vertex id outside [0, n_vertices)", hctr[0]);
            }
            p->n_pairs = total;
            int32_t* list = ta.get<int32_t>((size_t)total + 1, e);
            PCHK(e);
            PCHK(hipMemsetAsync(cnt, 0, sizeof(unsigned) * nbins, s));
            PCHK(mck::bins_fill(p->coords, d_cells, dim, nv, nc, p->gg, grid->origin, grid->spacing, B, nb0, nb1, nb2,
                                start, cnt, list, s));
            int32_t* unres = ta.get<int32_t>((size_t)ng, e);
            PCHK(e);
            PCHK(mck::locate(p->coords, d_cells, dim, nv, nc, p->gg, B, nb0, nb1, start, list, p->vid, p->w, p->cell,
                             unres, ctr + 1, ctr + 2, s));
            PCHK(hipMemcpyAsync(hctr, ctr, sizeof hctr, hipMemcpyDeviceToHost, s));
            PCHK(hipStreamSynchronize(s));
            p->n_unresolved = hctr[1];
            p->n_near_degenerate = hctr[2];
            if (p->n_unresolved > 0) {
                if (fill == MC_FILL_MIDRANGE) {
                    PCHK(mck::fill_midrange(dim, unres, p->n_unresolved, p->vid, p->w, ng, s));
                } else {
                    const int VB = dim == 2 ? 4 : 2;
                    const int vb0 = (int)((grid->dims[0] + VB - 1) / VB), vb1 = (int)((grid->dims[1] + VB - 1) / VB),
                              vb2 = dim == 3 ? (int)((grid->dims[2] + VB - 1) / VB) : 1;
                    const long long nvb = (long long)vb0 * vb1 * vb2;
                    unsigned* vcnt = ta.get<unsigned>(nvb + 4, e);
                    PCHK(e);
                    long long* vstart = ta.get<long long>(nvb + 1, e);
                    PCHK(e);
                    const long long vtiles = (nvb + MC_TILE - 1) / MC_TILE + 1;
                    unsigned long long* vst = ta.get<unsigned long long>(vtiles, e);
                    PCHK(e);
                    int32_t* vlist = ta.get<int32_t>((size_t)nv, e);
                    PCHK(e);
                    PCHK(hipMemsetAsync(vcnt, 0, sizeof(unsigned) * nvb, s));
                    PCHK(hipMemsetAsync(vst, 0, sizeof(unsigned long long) * vtiles, s));
                    PCHK(hipMemsetAsync(ctr + 4, 0, sizeof(unsigned), s));
                    PCHK(mck::vbins_count(p->coords, dim, nv, grid->origin, grid->spacing, VB, vb0, vb1, vb2, vcnt, s));
                    PCHK(mck::scan_u32(vcnt, nvb, vstart, vst, ctr + 4, s));
                    PCHK(hipMemsetAsync(vcnt, 0, sizeof(unsigned) * nvb, s));
                    PCHK(mck::vbins_fill(p->coords, dim, nv, grid->origin, grid->spacing, VB, vb0, vb1, vb2, vstart, vcnt,
                                         vlist, s));
                    PCHK(mck::fill_nearest(p->coords, dim, nv, p->gg, grid->origin, grid->spacing, VB, vb0, vb1, vb2,
                                           vstart, vlist, unres, p->n_unresolved, p->vid, p->w, ng, s));
                }
            }
            PCHK(hipStreamSynchronize(s));
        }
    }

    // compress / decompress workspace (on the coarsened grid when coarsened)
    const long long ngw = p->ng;
    p->ntg = (ngw + MC_TILE - 1) / MC_TILE;
    p->ntv = (nv + MC_TILE - 1) / MC_TILE;
    p->nblk = (nv + MC_LBLOCK - 1) / MC_LBLOCK;
    PCHK(plan_alloc(p, &p->p, (size_t)ngw));
    PCHK(plan_alloc(p, &p->ctl, 64));
    p->rbuf = (RangeOut*)p->ctl;                       // 2 slots of 3 words
    p->bound = (DevBound*)(p->ctl + 16);               // 11 words at word 16
    {
        RangeOut init[2];
        for (int k = 0; k < 2; ++k) { init[k].kmin = ~0ull; init[k].kmax = 0ull; init[k].flags = 0u; init[k].pad = 0u; }
        PCHK(hipMemsetAsync(p->ctl, 0, 64 * sizeof(unsigned long long), s));
        PCHK(hipMemcpyAsync(p->rbuf, init, sizeof init, hipMemcpyHostToDevice, s));
    }
    // per-call state cleared by k_range: error bits, outlier totals per group
    // of MC_SC_TILES tiles
    const long long ngg = (p->ntg + MC_SC_TILES - 1) / MC_SC_TILES, ngv = (p->ntv + MC_SC_TILES - 1) / MC_SC_TILES;
    p->nsmall = 16 + ngg + ngv;
    PCHK(plan_alloc(p, &p->small, (size_t)p->nsmall));
    PCHK(hipMemsetAsync(p->small, 0, (size_t)p->nsmall * 4, s));
    p->err = p->small + 2;
    p->gsum = p->small + 16;
    p->vsum = p->gsum + ngg;
    PCHK(plan_alloc(p, &p->counts, (size_t)(p->ntg + p->ntv)));
    PCHK(plan_alloc(p, &p->dagg, (size_t)p->ntv));
    PCHK(plan_alloc(p, &p->dcarry, (size_t)p->ntv));
    p->gcount = p->counts;
    p->vcount = p->counts + p->ntg;
    decode_ws_shape(p);
    PCHK(plan_alloc(p, &p->dws.agg_xy, (size_t)p->dws.ntiles_xy * p->dws.pitch));
    if (dim == 3) PCHK(plan_alloc(p, &p->dws.agg_z, (size_t)p->dws.nzc * p->dws.pitch * p->grid.dims[1]));
    if (p->dws.fast3) PCHK(plan_alloc(p, &p->dws.agg_t, (size_t)p->dws.nyc * p->dws.nzc * p->dws.pitch));
    if (dim == 2) PCHK(plan_alloc(p, &p->dws.segsum, (size_t)p->grid.dims[1] * ((p->grid.dims[0] + 255) / 256)));
    PCHK(plan_alloc(p, &p->xh, (size_t)ngw));
    PCHK(plan_alloc(p, &p->range_partial, (size_t)3 * MC_RANGE_BLOCKS));
    PCHK(hipStreamSynchronize(s));
    *out = p;
    return MC_OK;
}

// Times the point-location index build (cell counts per bin, their scan,
// the bin lists) and the location kernel for each candidate bin edge, on
// scratch buffers.  The mapping does not depend on the bin edge (bins only
// narrow the candidate cells of the lowest-id rule), so only time is
// compared.
extern "C" mc_status mc_plan_tune_bins(const float* d_coords, const int32_t* d_cells, int32_t dim, int64_t nv,
                                       int64_t nc, const mc_grid* grid, const int32_t* h_candidates,
                                       int32_t n_candidates, hipStream_t s, int32_t* best_bin_nodes,
                                       double* h_ms)
{
    mc_status st = check_mesh_args(d_coords, dim, nv);
    if (st != MC_OK) return st;
    if (!d_cells) return mc_fail(MC_ERR_ARG, "cells pointer is NULL");
    if (nc <= 0 || nc >= (1ll << 31)) return mc_fail(MC_ERR_ARG, "n_cells must be in [1, 2^31)");
    if ((st = mc_check_grid(grid, dim)) != MC_OK) return st;
    if (!h_candidates || n_candidates < 1 || n_candidates > 16) return mc_fail(MC_ERR_ARG, "1 to 16 candidates");
    for (int k = 0; k < n_candidates; ++k)
        if (h_candidates[k] < 1 || h_candidates[k] > 64) return mc_fail(MC_ERR_ARG, "bin edges must be in [1, 64]");
    if (!best_bin_nodes) return mc_fail(MC_ERR_ARG, "best_bin_nodes is NULL");
    const GridGeom gg = mc_geom(*grid);
    const long long ng = grid->dims[0] * grid->dims[1] * grid->dims[2];
    TempAllocs keep;
    hipError_t e = hipSuccess;
#define TCHK(x) do { if ((e = (x)) != hipSuccess) return mc_fail(MC_ERR_DEVICE, "%s: %s", #x, hipGetErrorString(e)); } while (0)
    float* coords = keep.get<float>((size_t)dim * nv, e);
    TCHK(e);
    TCHK(hipMemcpyAsync(coords, d_coords, sizeof(float) * dim * nv, hipMemcpyDeviceToDevice, s));
    int32_t* vid = keep.get<int32_t>((size_t)(dim + 1) * ng, e);
    TCHK(e);
    float* w = keep.get<float>((size_t)(dim + 1) * ng, e);
    TCHK(e);
    int32_t* cell = keep.get<int32_t>((size_t)ng, e);
    TCHK(e);
    int32_t* unres = keep.get<int32_t>((size_t)ng, e);
    TCHK(e);
    unsigned* ctr = keep.get<unsigned>(16, e);
    TCHK(e);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < 4; ++k) TCHK(hipEventCreateWithFlags(&ev[k], hipEventDisableSystemFence));
    struct EvFree {
        hipEvent_t* ev;
        ~EvFree() { for (int k = 0; k < 4; ++k) if (ev[k]) (void)hipEventDestroy(ev[k]); }
    } evfree{ev};
    double best_ms = 0.0;
    for (int k = 0; k < n_candidates; ++k) {
        const int B = h_candidates[k];
        TempAllocs ta;
        const int nb0 = (int)((grid->dims[0] + B - 1) / B), nb1 = (int)((grid->dims[1] + B - 1) / B),
                  nb2 = (int)((grid->dims[2] + B - 1) / B);
        const long long nbins = (long long)nb0 * nb1 * nb2;
        unsigned* cnt = ta.get<unsigned>(nbins + 4, e);
        TCHK(e);
        long long* start = ta.get<long long>(nbins + 1, e);
        TCHK(e);
        const long long nscan_tiles = (nbins + MC_TILE - 1) / MC_TILE + 1;
        unsigned long long* sst = ta.get<unsigned long long>(nscan_tiles, e);
        TCHK(e);
        TCHK(hipMemsetAsync(cnt, 0, sizeof(unsigned) * nbins, s));
        TCHK(hipMemsetAsync(ctr, 0, sizeof(unsigned) * 16, s));
        TCHK(hipMemsetAsync(sst, 0, sizeof(unsigned long long) * nscan_tiles, s));
        TCHK(hipEventRecord(ev[0], s));
        TCHK(mck::bins_count(coords, d_cells, dim, nv, nc, gg, grid->origin, grid->spacing, B, nb0, nb1, nb2, cnt,
                             ctr + 0, s));
        TCHK(mck::scan_u32(cnt, nbins, start, sst, ctr + 3, s));
        TCHK(hipEventRecord(ev[1], s));
        long long total = 0;
        unsigned bad = 0;
        TCHK(hipMemcpyAsync(&total, start + nbins, sizeof total, hipMemcpyDeviceToHost, s));
        TCHK(hipMemcpyAsync(&bad, ctr, sizeof bad, hipMemcpyDeviceToHost, s));
        TCHK(hipStreamSynchronize(s));
        if (bad != 0) return mc_fail(MC_ERR_ARG, "%u cells reference a vertex id outside [0, n_vertices)", bad);
        int32_t* list = ta.get<int32_t>((size_t)total + 1, e);
        TCHK(e);
        TCHK(hipMemsetAsync(cnt, 0, sizeof(unsigned) * nbins, s));
        TCHK(hipEventRecord(ev[2], s));
        TCHK(mck::bins_fill(coords, d_cells, dim, nv, nc, gg, grid->origin, grid->spacing, B, nb0, nb1, nb2, start,
                            cnt, list, s));
        TCHK(mck::locate(coords, d_cells, dim, nv, nc, gg, B, nb0, nb1, start, list, vid, w, cell, unres, ctr + 1,
                         ctr + 2, s));
        TCHK(hipEventRecord(ev[3], s));
        TCHK(hipEventSynchronize(ev[3]));
        float t01 = 0.f, t23 = 0.f;
        TCHK(hipEventElapsedTime(&t01, ev[0], ev[1]));
        TCHK(hipEventElapsedTime(&t23, ev[2], ev[3]));
        const double ms = (double)t01 + (double)t23;
        if (h_ms) h_ms[k] = ms;
        if (k == 0 || ms < best_ms) {
            best_ms = ms;
            *best_bin_nodes = B;
        }
    }
#undef TCHK
    return MC_OK;
}

extern "C" mc_status mc_plan_get_info(mc_plan p, mc_plan_info* out)
{
    if (!p || !out) return mc_fail(MC_ERR_ARG, "plan/out is NULL");
    out->n_grid = p->ng;
    out->n_vertices = p->nv;
    out->n_cells = p->nc;
    out->n_unresolved = p->n_unresolved;
    out->n_near_degenerate = p->n_near_degenerate;
    out->n_pairs = p->n_pairs;
    out->bin_nodes = p->B;
    out->device_bytes = (int64_t)p->bytes;
    out->invalid_cells = p->invalid_cells;
    return MC_OK;
}

extern "C" mc_status mc_plan_get_grid(mc_plan p, mc_grid* out)
{
    if (!p || !out) return mc_fail(MC_ERR_ARG, "plan/out is NULL");
    *out = p->grid;
    return MC_OK;
}

extern "C" mc_status mc_plan_mapping(mc_plan p, int32_t* d_vid, float* d_w, int32_t* d_cell, hipStream_t s)
{
    if (!p) return mc_fail(MC_ERR_ARG, "plan is NULL");
    if (p->ops != MC_OPS_LINEAR) return mc_fail(MC_ERR_UNSUPPORTED, "the plan has no cell mapping (MC_OPS_CLUSTER)");
    const size_t k = (size_t)(p->dim + 1) * p->ng;
    hipError_t e = hipSuccess;
    if (d_vid && e == hipSuccess) e = hipMemcpyAsync(d_vid, p->vid, k * 4, hipMemcpyDeviceToDevice, s);
    if (d_w && e == hipSuccess) e = hipMemcpyAsync(d_w, p->w, k * 4, hipMemcpyDeviceToDevice, s);
    if (d_cell && e == hipSuccess) e = hipMemcpyAsync(d_cell, p->cell, (size_t)p->ng * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "mapping copy: %s", hipGetErrorString(e));
    return MC_OK;
}

extern "C" mc_status mc_plan_kept_planes(mc_plan p, int32_t* h_keep, int64_t cap)
{
    if (!p || !h_keep) return mc_fail(MC_ERR_ARG, "plan/output pointer is NULL");
    if (!p->coarsen) return mc_fail(MC_ERR_UNSUPPORTED, "the plan was made without Grid_Coarsen");
    if (cap < (int64_t)p->keep.size()) return mc_fail(MC_ERR_CAPACITY, "h_keep needs %zu entries", p->keep.size());
    memcpy(h_keep, p->keep.data(), p->keep.size() * sizeof(int32_t));
    return MC_OK;
}

extern "C" mc_status mc_plan_nodes(mc_plan p, int32_t* d_m, hipStream_t s)
{
    if (!p) return mc_fail(MC_ERR_ARG, "plan is NULL");
    if (!d_m) return mc_fail(MC_ERR_ARG, "output pointer is NULL");
    if (p->ops != MC_OPS_CLUSTER) return mc_fail(MC_ERR_UNSUPPORTED, "the plan has no node map (MC_OPS_LINEAR)");
    hipError_t e = hipMemcpyAsync(d_m, p->m, (size_t)p->nv * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "node map copy: %s", hipGetErrorString(e));
    return MC_OK;
}

extern "C" mc_status mc_plan_node_lists(mc_plan p, int64_t* d_noff, int32_t* d_vlist, hipStream_t s)
{
    if (!p) return mc_fail(MC_ERR_ARG, "plan is NULL");
    if (p->ops != MC_OPS_CLUSTER) return mc_fail(MC_ERR_UNSUPPORTED, "the plan has no node lists (MC_OPS_LINEAR)");
    hipError_t e = hipSuccess;
    if (d_noff) e = hipMemcpyAsync(d_noff, p->noff, (size_t)(p->ng + 1) * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && d_vlist)
        e = hipMemcpyAsync(d_vlist, p->vlist, (size_t)p->nv * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "node list copy: %s", hipGetErrorString(e));
    return MC_OK;
}

extern "C" mc_status mc_plan_destroy(mc_plan p)
{
    if (!p) return MC_OK;
    mc_batch_forget(p);
    for (void* q : p->allocs) (void)hipFree(q);
    delete p;
    return MC_OK;
}

// ---------------------------------------------------------------------------
// compress / decompress
// ---------------------------------------------------------------------------
static mc_status check_codes(mc_plan p, const mc_codes* c, bool need_flags)
{
    if (!c) return mc_fail(MC_ERR_ARG, "codes pointer is NULL");
    if (c->residual_predictor != MC_RESPRED_NONE && c->residual_predictor != MC_RESPRED_DELTA)
        return mc_fail(MC_ERR_ARG, "unknown residual predictor");
    if (c->grid_predictor != MC_GRIDPRED_LORENZO && c->grid_predictor != MC_GRIDPRED_INTERP_LINEAR &&
        c->grid_predictor != MC_GRIDPRED_INTERP_CUBIC && c->grid_predictor != MC_GRIDPRED_TEMPORAL)
        return mc_fail(MC_ERR_ARG, "unknown grid predictor");
    if (c->grid_predictor == MC_GRIDPRED_TEMPORAL && !c->grid_ref)
        return mc_fail(MC_ERR_ARG, "the time-axis grid predictor needs grid_ref");
    if (c->residual_predictor == MC_RESPRED_DELTA && need_flags)
        return mc_fail(MC_ERR_UNSUPPORTED, "the delta residual predictor takes no learned model");
    if (!c->grid_codes || !c->vert_codes || !c->result) return mc_fail(MC_ERR_ARG, "codes buffers are NULL");
    if (c->g_out_cap < 0 || c->v_out_cap < 0) return mc_fail(MC_ERR_ARG, "negative outlier capacity");
    if (c->g_out_cap > 0 && (!c->g_out_idx || !c->g_out_delta)) return mc_fail(MC_ERR_ARG, "grid outlier buffers are NULL");
    if (c->v_out_cap > 0 && (!c->v_out_idx || !c->v_out_val)) return mc_fail(MC_ERR_ARG, "vertex outlier buffers are NULL");
    if (need_flags && !c->block_flags) return mc_fail(MC_ERR_ARG, "block_flags is required with a model");
    (void)p;
    return MC_OK;
}

// Grid codes of the prequantised grid p->p under the chosen grid predictor.
static hipError_t grid_codes(mc_plan p, const mc_codes* codes, hipStream_t s)
{
    const int n0 = (int)p->grid.dims[0], n1 = (int)p->grid.dims[1], n2 = (int)p->grid.dims[2];
    if (codes->grid_predictor == MC_GRIDPRED_LORENZO)
        return mck::lorenzo(p->p, p->dim, n0, n1, n2, p->ng, codes->grid_codes, p->gcount, p->gsum, p->knobs, s);
    if (codes->grid_predictor == MC_GRIDPRED_TEMPORAL)
        return mck::temporal_codes(p->p, codes->grid_ref, p->bound, p->ng, codes->grid_codes, p->gcount, p->gsum, s);
    return mck::interp_codes(p->p, n0, n1, n2, p->ng, codes->grid_predictor == MC_GRIDPRED_INTERP_CUBIC,
                             codes->grid_codes, p->gcount, p->gsum, s);
}

mc_status mc_compress_enqueue(mc_plan p, const void* d_field, mc_dtype dtype, const mc_params* prm,
                              const mc_codes* codes, hipStream_t s)
{
    const long long nbf = (p->nblk + 31) / 32;
    BoundParams bp;
    bp.eb = prm->eb;
    bp.split = prm->grid_share;
    bp.relative = prm->eb_mode == MC_EB_REL;
    bp.mode = prm->split_mode;
    hipError_t e;
#define ECHK(x) do { if ((e = (x)) != hipSuccess) return mc_fail(MC_ERR_DEVICE, "%s: %s", #x, hipGetErrorString(e)); } while (0)
    RangeOut* cur = p->rbuf;
    ECHK(mck::range(d_field, dtype, p->nv, p->range_partial, cur, bp, p->bound, p->small, p->nsmall, p->knobs, s));
    if (p->ops == MC_OPS_CLUSTER) {
        double* x1 = prm->residual == MC_RESIDUAL_OPEN ? p->x1 : nullptr;
        ECHK(mck::cluster_mean(p->noff, p->vlist, p->ng, d_field, dtype, p->bound, p->p, p->xh, x1,
                               codes->dbg_resampled, p->err, codes->result, p->gcount, p->ntg, s));
        p->xh_valid = true;
        ECHK(grid_codes(p, codes, s));
        if (codes->residual_predictor == MC_RESPRED_DELTA) {
            ECHK(mck::residual_delta(p->coords, p->nv, p->gg, p->xh, p->m, d_field, dtype, p->bound,
                                     codes->vert_codes, codes->dbg_vertex_g, p->vcount, p->vsum, p->err, s));
        } else {
            ECHK(mck::residual_nearest(p->m, p->nv, d_field, dtype, x1, p->xh, p->bound, codes->vert_codes,
                                       codes->dbg_vertex_g, p->vcount, p->vsum, s));
        }
        ECHK(mck::compact(p->p, p->dim, (int)p->grid.dims[0], (int)p->grid.dims[1], p->ng, codes->grid_predictor,
                          codes->grid_ref, codes->grid_codes, p->gcount, p->gsum, codes->g_out_idx,
                          codes->g_out_delta, codes->g_out_cap, d_field, dtype, p->nv, codes->vert_codes, p->vcount,
                          p->vsum, codes->v_out_idx, codes->v_out_val, codes->v_out_cap, p->err, codes->result, s));
        if (codes->dbg_grid_p)
            ECHK(hipMemcpyAsync(codes->dbg_grid_p, p->p, (size_t)p->ng * 4, hipMemcpyDeviceToDevice, s));
        if (codes->xhat_out)
            ECHK(hipMemcpyAsync(codes->xhat_out, p->xh, (size_t)p->ng * 4, hipMemcpyDeviceToDevice, s));
        return MC_OK;
    }
    // plain value-by-value residual codes read the cell corners from p (x1' is
    // then never written); the learned and delta coders and xhat_out read x1'
    const bool from_p = !prm->model && codes->residual_predictor == MC_RESPRED_NONE && !codes->xhat_out;
    ECHK(mck::resample(p->vid, p->w, p->dim, p->ng, d_field, dtype, p->bound, p->p, from_p ? nullptr : p->xh,
                       codes->dbg_resampled, codes->block_flags, codes->block_flags ? nbf : 0, p->err, codes->result,
                       p->gcount, p->ntg, p->knobs, s));
    p->xh_valid = !from_p;
    if (from_p && codes->grid_predictor == MC_GRIDPRED_LORENZO) {
        // grid and vertex codes in one launch
        ECHK(mck::codes(p->p, p->dim, (int)p->grid.dims[0], (int)p->grid.dims[1], (int)p->grid.dims[2],
                        codes->grid_codes, p->gcount, p->gsum, p->coords, p->nv, p->gg, p->xh, p->p, d_field, dtype,
                        p->bound, codes->vert_codes, codes->dbg_vertex_g, p->vcount, p->vsum, p->knobs, s));
        ECHK(mck::compact(p->p, p->dim, (int)p->grid.dims[0], (int)p->grid.dims[1], p->ng, codes->grid_predictor,
                          codes->grid_ref, codes->grid_codes, p->gcount, p->gsum, codes->g_out_idx,
                          codes->g_out_delta, codes->g_out_cap, d_field, dtype, p->nv, codes->vert_codes, p->vcount,
                          p->vsum, codes->v_out_idx, codes->v_out_val, codes->v_out_cap, p->err, codes->result, s));
        if (codes->dbg_grid_p)
            ECHK(hipMemcpyAsync(codes->dbg_grid_p, p->p, (size_t)p->ng * 4, hipMemcpyDeviceToDevice, s));
        return MC_OK;
    }
    ECHK(grid_codes(p, codes, s));
    if (codes->residual_predictor == MC_RESPRED_DELTA) {         // no model with this predictor
        ECHK(mck::residual_delta(p->coords, p->nv, p->gg, p->xh, nullptr, d_field, dtype, p->bound,
                                 codes->vert_codes, codes->dbg_vertex_g, p->vcount, p->vsum, p->err, s));
    } else if (prm->model) {
        // network shifts, block choice and vertex codes in one pass
        ECHK(mck::mlp_residual(prm->model->md, p->coords, p->nv, p->gg, p->xh, d_field, dtype, p->bound,
                               codes->vert_codes, codes->block_flags, codes->dbg_vertex_g, codes->rho_q, p->vcount,
                               p->vsum, s));
    } else {
        ECHK(mck::residual(p->coords, p->nv, p->gg, p->xh, from_p ? p->p : nullptr, d_field, dtype, p->bound,
                           codes->vert_codes, codes->dbg_vertex_g, p->vcount, p->vsum, p->knobs, s));
    }
    ECHK(mck::compact(p->p, p->dim, (int)p->grid.dims[0], (int)p->grid.dims[1], p->ng, codes->grid_predictor,
                      codes->grid_ref, codes->grid_codes, p->gcount, p->gsum, codes->g_out_idx, codes->g_out_delta,
                      codes->g_out_cap, d_field, dtype, p->nv, codes->vert_codes, p->vcount, p->vsum,
                      codes->v_out_idx, codes->v_out_val, codes->v_out_cap, p->err, codes->result, s));
    if (codes->dbg_grid_p) ECHK(hipMemcpyAsync(codes->dbg_grid_p, p->p, (size_t)p->ng * 4, hipMemcpyDeviceToDevice, s));
    if (codes->xhat_out) ECHK(hipMemcpyAsync(codes->xhat_out, p->xh, (size_t)p->ng * 4, hipMemcpyDeviceToDevice, s));
#undef ECHK
    return MC_OK;
}

mc_status mc_plan_ensure_xh(mc_plan p, hipStream_t s)
{
    if (p->xh_valid) return MC_OK;
    hipError_t e = mck::xhat_from_p(p->p, p->ng, p->bound, p->xh, s);
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "xhat_from_p: %s", hipGetErrorString(e));
    p->xh_valid = true;
    return MC_OK;
}

mc_status mc_check_params(mc_plan p, const void* d_field, mc_dtype dtype, const mc_params* prm, const mc_codes* codes)
{
    if (!p) return mc_fail(MC_ERR_ARG, "plan is NULL");
    if (!d_field) return mc_fail(MC_ERR_ARG, "field pointer is NULL");
    if (dtype != MC_F32 && dtype != MC_F64) return mc_fail(MC_ERR_ARG, "dtype must be MC_F32 or MC_F64");
    if (!prm) return mc_fail(MC_ERR_ARG, "params pointer is NULL");
    if (!(prm->eb > 0.0) || !std::isfinite(prm->eb)) return mc_fail(MC_ERR_ARG, "eb must be finite and > 0");
    if (prm->eb_mode != MC_EB_ABS && prm->eb_mode != MC_EB_REL) return mc_fail(MC_ERR_ARG, "unknown eb_mode");
    if (prm->split_mode != MC_SPLIT_SUM && prm->split_mode != MC_SPLIT_FULL) return mc_fail(MC_ERR_ARG, "unknown split_mode");
    if (prm->split_mode == MC_SPLIT_SUM && (!(prm->grid_share > 0.0) || !(prm->grid_share < 1.0)))
        return mc_fail(MC_ERR_ARG, "grid_share must be in (0, 1)");
    if (prm->split_mode == MC_SPLIT_FULL && (!(prm->grid_share > 0.0) || !(prm->grid_share <= 16.0)))
        return mc_fail(MC_ERR_ARG, "grid_share must be in (0, 16] with MC_SPLIT_FULL");
    if (prm->model && mc_model_dim(prm->model) != p->dim) return mc_fail(MC_ERR_ARG, "model dim does not match the plan");
    if (prm->residual != MC_RESIDUAL_CLOSED && prm->residual != MC_RESIDUAL_OPEN)
        return mc_fail(MC_ERR_ARG, "unknown residual reference");
    if (prm->residual == MC_RESIDUAL_OPEN && (p->ops != MC_OPS_CLUSTER || prm->split_mode != MC_SPLIT_SUM))
        return mc_fail(MC_ERR_UNSUPPORTED, "the open-loop residual needs an MC_OPS_CLUSTER plan and MC_SPLIT_SUM");
    if (prm->model && p->ops != MC_OPS_LINEAR)
        return mc_fail(MC_ERR_UNSUPPORTED, "the learned predictor needs an MC_OPS_LINEAR plan");
    if (codes && codes->residual_predictor == MC_RESPRED_DELTA && prm->residual == MC_RESIDUAL_OPEN)
        return mc_fail(MC_ERR_UNSUPPORTED, "the delta residual predictor needs the closed loop");
    return check_codes(p, codes, prm->model != nullptr);
}

extern "C" mc_status mc_compress(mc_plan p, const void* d_field, mc_dtype dtype, const mc_params* prm,
                                 const mc_codes* codes, hipStream_t s)
{
    mc_status st = mc_check_params(p, d_field, dtype, prm, codes);
    if (st != MC_OK) return st;
    return mc_compress_enqueue(p, d_field, dtype, prm, codes, s);
}

mc_status mc_check_decompress(mc_plan p, const mc_codes* codes, mc_model model, const void* d_out, mc_dtype dtype)
{
    if (!p) return mc_fail(MC_ERR_ARG, "plan is NULL");
    if (!d_out) return mc_fail(MC_ERR_ARG, "output pointer is NULL");
    if (dtype != MC_F32 && dtype != MC_F64) return mc_fail(MC_ERR_ARG, "dtype must be MC_F32 or MC_F64");
    if (model && mc_model_dim(model) != p->dim) return mc_fail(MC_ERR_ARG, "model dim does not match the plan");
    if (model && p->ops != MC_OPS_LINEAR)
        return mc_fail(MC_ERR_UNSUPPORTED, "the learned predictor needs an MC_OPS_LINEAR plan");
    return check_codes(p, codes, model != nullptr);
}

mc_status mc_grid_decode_enqueue(mc_plan p, const mc_codes* codes, float* xh, hipStream_t s)
{
    hipError_t e;
#define ECHK(x) do { if ((e = (x)) != hipSuccess) return mc_fail(MC_ERR_DEVICE, "%s: %s", #x, hipGetErrorString(e)); } while (0)
    if (codes->grid_predictor == MC_GRIDPRED_LORENZO)
        ECHK(mck::grid_decode(codes->grid_codes, codes->g_out_idx, codes->g_out_delta, codes->g_out_cap,
                              codes->result, p->dim, (int)p->grid.dims[0], (int)p->grid.dims[1],
                              (int)p->grid.dims[2], p->p, xh, p->dws, p->knobs, s));
    else if (codes->grid_predictor == MC_GRIDPRED_TEMPORAL)
        ECHK(mck::temporal_decode(codes->grid_codes, codes->g_out_idx, codes->g_out_delta, codes->g_out_cap,
                                  codes->result, codes->grid_ref, p->ng, p->p, xh, s));
    else
        ECHK(mck::interp_decode(codes->grid_codes, codes->g_out_idx, codes->g_out_delta, codes->g_out_cap,
                                codes->result, p->dim, (int)p->grid.dims[0], (int)p->grid.dims[1],
                                (int)p->grid.dims[2], codes->grid_predictor == MC_GRIDPRED_INTERP_CUBIC, p->p,
                                xh, s));
    if (xh == p->xh) p->xh_valid = true;
    if (codes->xhat_out)
        ECHK(hipMemcpyAsync(codes->xhat_out, xh, (size_t)p->ng * 4, hipMemcpyDeviceToDevice, s));
#undef ECHK
    return MC_OK;
}

mc_status mc_decompress_enqueue(mc_plan p, const mc_codes* codes, mc_model model, void* d_out, mc_dtype dtype,
                                hipStream_t s)
{
    hipError_t e;
    mc_status gst = mc_grid_decode_enqueue(p, codes, p->xh, s);
    if (gst != MC_OK) return gst;
#define ECHK(x) do { if ((e = (x)) != hipSuccess) return mc_fail(MC_ERR_DEVICE, "%s: %s", #x, hipGetErrorString(e)); } while (0)
    if (p->ops == MC_OPS_CLUSTER && codes->residual_predictor == MC_RESPRED_DELTA) {
        ECHK(mck::vertex_decode_delta(p->coords, p->nv, p->gg, p->xh, p->m, codes->vert_codes, codes->v_out_idx,
                                      codes->v_out_val, codes->v_out_cap, codes->result, p->dagg, p->dcarry, d_out,
                                      dtype, s));
        return MC_OK;
    }
    if (p->ops == MC_OPS_CLUSTER) {
        ECHK(mck::vertex_decode_nearest(p->m, p->nv, p->xh, codes->vert_codes, codes->v_out_idx, codes->v_out_val,
                                        codes->v_out_cap, codes->result, d_out, dtype, s));
        return MC_OK;
    }
    if (model && codes->residual_predictor != MC_RESPRED_DELTA) {
        // network shifts and vertex decode in one pass
        ECHK(mck::mlp_vdecode(model->md, p->coords, p->nv, p->gg, p->xh, codes->block_flags, codes->vert_codes,
                              codes->v_out_idx, codes->v_out_val, codes->result, codes->v_out_cap, d_out, dtype, s));
        return MC_OK;
    }
    if (codes->residual_predictor == MC_RESPRED_DELTA) {
        ECHK(mck::vertex_decode_delta(p->coords, p->nv, p->gg, p->xh, nullptr, codes->vert_codes, codes->v_out_idx,
                                      codes->v_out_val, codes->v_out_cap, codes->result, p->dagg, p->dcarry, d_out,
                                      dtype, s));
        return MC_OK;
    }
    ECHK(mck::vertex_decode(p->coords, p->nv, p->gg, p->xh, codes->vert_codes, codes->v_out_idx, codes->v_out_val,
                            codes->v_out_cap, codes->result, d_out, dtype, p->knobs, s));
#undef ECHK
    return MC_OK;
}

extern "C" mc_status mc_decompress(mc_plan p, const mc_codes* codes, mc_model model, void* d_out, mc_dtype dtype,
                                   hipStream_t s)
{
    mc_status st = mc_check_decompress(p, codes, model, d_out, dtype);
    if (st != MC_OK) return st;
    return mc_decompress_enqueue(p, codes, model, d_out, dtype, s);
}

// ---------------------------------------------------------------------------
// autotuning of the launch-order knobs
// ---------------------------------------------------------------------------
extern "C" mc_status mc_plan_get_tuning(mc_plan p, mc_tuning* out)
{
    if (!p || !out) return mc_fail(MC_ERR_ARG, "plan or output is NULL");
    *out = mc_tuning{};
    out->remap_mask = p->knobs;
    return MC_OK;
}

extern "C" mc_status mc_plan_set_tuning(mc_plan p, const mc_tuning* t)
{
    if (!p || !t) return mc_fail(MC_ERR_ARG, "plan or tuning is NULL");
    if (t->remap_mask & ~(unsigned)mck::MC_KNOB_ALL) return mc_fail(MC_ERR_ARG, "unknown bits in remap_mask");
    p->knobs = t->remap_mask;
    return MC_OK;
}

extern "C" mc_status mc_plan_tune(mc_plan p, const void* d_field, mc_dtype dtype, const mc_params* prm,
                                  const mc_codes* codes, void* d_out, int32_t reps, hipStream_t s, mc_tuning* chosen)
{
    mc_status st = mc_check_params(p, d_field, dtype, prm, codes);
    if (st != MC_OK) return st;
    if ((st = mc_check_decompress(p, codes, prm->model, d_out, dtype)) != MC_OK) return st;
    if (reps < 1 || reps > 1000) return mc_fail(MC_ERR_ARG, "reps must be in [1, 1000]");
    // device milliseconds of `reps` whole compress + decompress passes with
    // the given knobs (HIP events on the stream around the passes, after one
    // untimed pass; the per-launch profiler stays off while timing, since its
    // events would add to every launch)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return mc_fail(MC_ERR_DEVICE, "hipEventCreate failed");
    }
    auto measure = [&](unsigned knobs, double* ms) -> mc_status {
        p->knobs = knobs;
        mc_status r = mc_compress_enqueue(p, d_field, dtype, prm, codes, s);
        if (r == MC_OK) r = mc_decompress_enqueue(p, codes, prm->model, d_out, dtype, s);
        if (r != MC_OK) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return mc_fail(MC_ERR_DEVICE, "hipEventRecord failed");
        for (int i = 0; i < reps && r == MC_OK; ++i) {
            r = mc_compress_enqueue(p, d_field, dtype, prm, codes, s);
            if (r == MC_OK) r = mc_decompress_enqueue(p, codes, prm->model, d_out, dtype, s);
        }
        if (r != MC_OK) return r;
        float t = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            return mc_fail(MC_ERR_DEVICE, "timing events failed");
        *ms = t;
        return MC_OK;
    };
    const bool was_on = g_prof_on;
    mc_profile_enable(0);
    // coordinate descent from the default mask, two sweeps over the bits; a
    // flip is kept only when it is faster by more than half a percent, so
    // timing noise does not walk the mask away from the default
    unsigned best = mck::MC_KNOB_DEFAULT;
    double best_ms = 0.0;
    st = measure(best, &best_ms);
    for (int sweep = 0; sweep < 2 && st == MC_OK; ++sweep) {
        bool changed = false;
        for (unsigned bit = 1; (bit & mck::MC_KNOB_ALL) && st == MC_OK; bit <<= 1) {
            double ms = 0.0;
            if ((st = measure(best ^ bit, &ms)) != MC_OK) break;
            if (ms < 0.995 * best_ms) {
                best ^= bit;
                best_ms = ms;
                changed = true;
            }
        }
        if (!changed) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MC_OK) {
        mc_profile_enable(was_on ? 1 : 0);
        return st;
    }
    p->knobs = best;
    mc_profile_enable(was_on ? 1 : 0);
    if (chosen) {
        *chosen = mc_tuning{};
        chosen->remap_mask = best;
    }
    return MC_OK;
}

extern "C" mc_status mc_compress_mesh(const float* d_coords, const int32_t* d_cells, int32_t dim, int64_t nv, int64_t nc,
                                      const void* d_field, mc_dtype dtype, const double spacing[3], double eb,
                                      int32_t eb_mode, double grid_share, const mc_codes* codes, mc_grid* grid_out,
                                      hipStream_t s)
{
    mc_grid g;
    mc_status st = mc_grid_from_spacing(d_coords, dim, nv, spacing, s, &g);
    if (st != MC_OK) return st;
    mc_plan p = nullptr;
    if ((st = mc_plan_create(d_coords, d_cells, dim, nv, nc, &g, nullptr, s, &p)) != MC_OK) return st;
    mc_params prm{};
    prm.eb = eb;
    prm.eb_mode = eb_mode;
    prm.grid_share = grid_share;
    prm.model = nullptr;
    st = mc_compress(p, d_field, dtype, &prm, codes, s);
    if (st == MC_OK && hipStreamSynchronize(s) != hipSuccess) st = mc_fail(MC_ERR_DEVICE, "synchronize failed");
    mc_plan_destroy(p);
    if (st == MC_OK && grid_out) *grid_out = g;
    return st;
}
