// mc_batch.hip -- batched compression and decompression of many fields on
// many plans.
//
// The first call with a given item list captures the whole batch into one
// HIP graph and later calls replay it (a single graph launch per batch).
//
// Fields on the plain Lorenzo path (linear operator pair, no model, the
// value-by-value residual coder, no diagnostics) go through work-list stage
// launches: each stage of the method is one launch over the tiles of every
// such field (range, range fold, resample, grid + vertex codes, outlier
// lists; vertex decode), its blocks mapped to (field, tile) by prefix tables
// and the fields' value types and dimensions dispatched inside the kernel.
// Each field has its own workspace (range partials, control block,
// counters, p; decoded grid), owned by the graph, so fields on one mesh run
// in the same launch.  Stage boundaries are the launch boundaries: a single
// resident kernel would need a device-scope release and acquire between
// stages, and on this chip such a fence writes back or invalidates each
// XCD's L2 (2,048 fenced atomics cost 79 us in the range kernel).
//
// The other fields keep one chain of ordinary launches per distinct plan
// (fields on one mesh in order: they share the plan's workspace; chains of
// different meshes concurrent), forked from and joined back to the graph's
// origin.  In a decompress, the grid decode of every field runs on its
// plan's chain (writing the field's own decoded grid) and the batched
// vertex decode follows the join.  Every kernel is capturable: per-call
// state is cleared by a kernel, never by a memset node.
#include <string.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <vector>

#include "mc_internal.h"

namespace {

struct BatchGraph {
    int kind = 0;                       // 0 compress, 1 decompress
    std::vector<unsigned char> key;     // the item list the graph was captured from
    std::vector<const void*> refs;      // plans and models the graph uses
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<void*> dev;             // per-field workspaces, descriptors and prefix tables
    int n_batched = 0;                  // fields on the work-list stage launches
};

std::mutex g_bm;
std::vector<BatchGraph*> g_graphs;
const size_t kMaxGraphs = 16;

void destroy_graph(BatchGraph* g)
{
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
    for (hipStream_t s : g->streams) (void)hipStreamDestroy(s);
    for (void* q : g->dev) (void)hipFree(q);
    delete g;
}

// Replays the cached graph of (kind, key) if there is one.  Caller holds g_bm.
bool replay(int kind, const std::vector<unsigned char>& key, hipStream_t stream, mc_status* st)
{
    for (BatchGraph* g : g_graphs)
        if (g->kind == kind && g->key == key) {
            hipError_t e = hipGraphLaunch(g->exec, stream);
            *st = e == hipSuccess ? MC_OK : mc_fail(MC_ERR_DEVICE, "graph launch: %s", hipGetErrorString(e));
            return true;
        }
    return false;
}

// Captures the batch: `concurrent(origin)` on the origin stream while
// enqueue(i, s) runs every listed item i on one chain per distinct plan,
// then `after(origin)` once the chains have joined; instantiates the graph,
// launches it on `stream` and caches it (taking ownership of bg).  Caller
// holds g_bm.
mc_status capture(BatchGraph* bg, const std::vector<mc_plan>& item_plan, const std::vector<int>& chained,
                  const std::function<mc_status(int, hipStream_t)>& enqueue,
                  const std::function<mc_status(hipStream_t)>& concurrent,
                  const std::function<mc_status(hipStream_t)>& after, hipStream_t stream)
{
    std::vector<mc_plan> plans;
    for (int i : chained)
        if (std::find(plans.begin(), plans.end(), item_plan[i]) == plans.end()) plans.push_back(item_plan[i]);
    std::stable_sort(plans.begin(), plans.end(), [](mc_plan a, mc_plan b) { return a->nv + a->ng > b->nv + b->ng; });

    // Capture happens on a private origin stream (the caller's stream may be
    // the null stream, which cannot be captured); chain c runs on stream c + 1.
    const size_t nc = plans.size();
    hipError_t e = hipSuccess;
    for (size_t c = 0; c <= nc && e == hipSuccess; ++c) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) bg->streams.push_back(s);
    }
    for (size_t c = 0; c <= nc && e == hipSuccess; ++c) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) bg->events.push_back(ev);
    }
    if (e != hipSuccess) {
        destroy_graph(bg);
        return mc_fail(MC_ERR_DEVICE, "batch streams: %s", hipGetErrorString(e));
    }
    hipStream_t origin = bg->streams[0];
    mc_status st = MC_OK;
    mc_capturing = true;
    e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess && nc > 0) e = hipEventRecord(bg->events[0], origin);      // fork
    for (size_t c = 1; c <= nc && e == hipSuccess; ++c)
        e = hipStreamWaitEvent(bg->streams[c], bg->events[0], 0);
    if (e == hipSuccess) st = concurrent(origin);
    for (size_t c = 0; c < nc && e == hipSuccess && st == MC_OK; ++c)
        for (int i : chained)
            if (st == MC_OK && item_plan[i] == plans[c]) st = enqueue(i, bg->streams[c + 1]);
    for (size_t c = 1; c <= nc && e == hipSuccess; ++c) {                          // join
        e = hipEventRecord(bg->events[c], bg->streams[c]);
        if (e == hipSuccess) e = hipStreamWaitEvent(origin, bg->events[c], 0);
    }
    if (e == hipSuccess && st == MC_OK) st = after(origin);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(origin, &graph);
    mc_capturing = false;
    if (e == hipSuccess) e = e2;
    bg->graph = graph;
    if (st != MC_OK || e != hipSuccess) {
        destroy_graph(bg);
        return st != MC_OK ? st : mc_fail(MC_ERR_DEVICE, "batch capture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&bg->exec, bg->graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(bg->exec, stream);
    if (e != hipSuccess) {
        destroy_graph(bg);
        return mc_fail(MC_ERR_DEVICE, "batch graph: %s", hipGetErrorString(e));
    }
    if (g_graphs.size() >= kMaxGraphs) {
        // the oldest graph may still be executing: wait for it before freeing
        (void)hipDeviceSynchronize();
        destroy_graph(g_graphs.front());
        g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back(bg);
    return MC_OK;
}

// Device allocation owned by the graph, zero-filled (outside any capture).
template <typename T>
hipError_t gdev(BatchGraph* bg, T** out, size_t n)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n * sizeof(T) > 0 ? n * sizeof(T) : 16);
    if (e != hipSuccess) return e;
    bg->dev.push_back(q);
    e = hipMemset(q, 0, n * sizeof(T) > 0 ? n * sizeof(T) : 16);
    *out = (T*)q;
    return e;
}

// Uploads a host vector into a graph-owned device array.
template <typename T>
hipError_t gupload(BatchGraph* bg, T** out, const std::vector<T>& h)
{
    hipError_t e = gdev(bg, out, h.size());
    if (e == hipSuccess) e = hipMemcpy(*out, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

// Prefix table of per-field block counts.
std::vector<unsigned> bases(const std::vector<long long>& counts, unsigned* total)
{
    std::vector<unsigned> b(counts.size() + 1, 0u);
    for (size_t i = 0; i < counts.size(); ++i) b[i + 1] = b[i] + (unsigned)counts[i];
    *total = b.back();
    return b;
}

// The plain Lorenzo path that the work-list stage launches take.
bool batched_compress(const mc_batch_item& it)
{
    const mc_codes& c = it.codes;
    return it.plan->ops == MC_OPS_LINEAR && !it.params.model && c.residual_predictor == MC_RESPRED_NONE &&
           c.grid_predictor == MC_GRIDPRED_LORENZO && !c.xhat_out && !c.dbg_resampled && !c.dbg_grid_p &&
           !c.dbg_vertex_g && !c.rho_q;
}

bool batched_decompress(const mc_batch_ditem& it)
{
    return it.plan->ops == MC_OPS_LINEAR && !it.model && it.codes.residual_predictor == MC_RESPRED_NONE;
}

template <class T>
std::vector<unsigned char> key_of(const T* items, int32_t n)
{
    return std::vector<unsigned char>((const unsigned char*)items, (const unsigned char*)(items + n));
}

}  // namespace

// Profiler events are not recorded while a batch is being captured.
thread_local bool mc_capturing = false;

extern "C" mc_status mc_batch_compress(const mc_batch_item* items, int32_t n, hipStream_t stream)
{
    if (!items || n <= 0) return mc_fail(MC_ERR_ARG, "invalid batch (items NULL or n <= 0)");
    for (int32_t i = 0; i < n; ++i) {
        mc_status st = mc_check_params(items[i].plan, items[i].d_field, items[i].dtype, &items[i].params,
                                       &items[i].codes);
        if (st != MC_OK) return mc_fail(st, "batch item %d: %s", i, mc_last_error());
    }
    std::vector<unsigned char> key = key_of(items, n);
    std::lock_guard<std::mutex> lk(g_bm);
    mc_status st;
    if (replay(0, key, stream, &st)) return st;
    BatchGraph* bg = new BatchGraph();
    bg->kind = 0;
    bg->key = std::move(key);
    std::vector<mc_plan> ip(n);
    std::vector<int> chained, batched;
    for (int32_t i = 0; i < n; ++i) {
        ip[i] = items[i].plan;
        bg->refs.push_back(items[i].plan);
        if (items[i].params.model) bg->refs.push_back(items[i].params.model);
        (batched_compress(items[i]) ? batched : chained).push_back(i);
    }
    // descriptors and workspaces of the batched fields
    const int nb = (int)batched.size();
    std::vector<mck::BItemC> d(nb);
    std::vector<long long> c_range(nb), c_res(nb), c_codes(nb), c_scat(nb);
    hipError_t e = hipSuccess;
    for (int k = 0; k < nb && e == hipSuccess; ++k) {
        const mc_batch_item& it = items[batched[k]];
        const mc_plan p = it.plan;
        mck::BItemC& b = d[k];
        b = mck::BItemC{};
        b.cls = 2 * (it.dtype == MC_F64 ? 1 : 0) + (p->dim == 3 ? 1 : 0);
        b.vec = ((uintptr_t)it.d_field & 15u) == 0;
        b.n0 = (int)p->grid.dims[0];
        b.n1 = (int)p->grid.dims[1];
        b.n2 = (int)p->grid.dims[2];
        mck::lorenzo_units(p->dim, b.n0, b.n1, b.n2, &b.nxs, &b.nyb, &b.nunits);
        b.nbl = (b.nunits + 3) / 4;
        b.ng = p->ng;
        b.nv = p->nv;
        b.ntg = (p->ng + MC_TILE - 1) / MC_TILE;
        b.ntv = (p->nv + MC_TILE - 1) / MC_TILE;
        const long long ngg = (b.ntg + MC_SC_TILES - 1) / MC_SC_TILES, ngv = (b.ntv + MC_SC_TILES - 1) / MC_SC_TILES;
        b.nsmall = 16 + ngg + ngv;
        // about 32 values per thread in the range pass
        long long np = (p->nv + 256 * 32 - 1) / (256 * 32);
        b.nparts = (unsigned)(np < 1 ? 1 : (np > MC_RANGE_BLOCKS ? MC_RANGE_BLOCKS : np));
        b.knobs = p->knobs;
        b.gg = p->gg;
        b.bp.eb = it.params.eb;
        b.bp.split = it.params.grid_share;
        b.bp.relative = it.params.eb_mode == MC_EB_REL;
        b.bp.mode = it.params.split_mode;
        b.vid = p->vid;
        b.w = p->w;
        b.coords = p->coords;
        b.x = it.d_field;
        b.gcodes = it.codes.grid_codes;
        b.gidx = it.codes.g_out_idx;
        b.gdelta = it.codes.g_out_delta;
        b.gcap = it.codes.g_out_cap;
        b.vcodes = it.codes.vert_codes;
        b.vidx = it.codes.v_out_idx;
        b.vval = it.codes.v_out_val;
        b.vcap = it.codes.v_out_cap;
        b.res = it.codes.result;
        b.bflags = it.codes.block_flags;
        b.nbflags = it.codes.block_flags ? ((p->nv + MC_LBLOCK - 1) / MC_LBLOCK + 31) / 32 : 0;
        unsigned long long* ctl = nullptr;
        if (e == hipSuccess) e = gdev(bg, &b.partial, (size_t)3 * b.nparts);
        if (e == hipSuccess) e = gdev(bg, &ctl, 64);
        if (e == hipSuccess) e = gdev(bg, &b.small, (size_t)b.nsmall);
        if (e == hipSuccess) e = gdev(bg, &b.gcount, (size_t)b.ntg);
        if (e == hipSuccess) e = gdev(bg, &b.vcount, (size_t)b.ntv);
        if (e == hipSuccess) e = gdev(bg, &b.p, (size_t)b.ng);
        b.cur = (RangeOut*)ctl;
        b.bnd = (DevBound*)(ctl + 16);
        c_range[k] = b.nparts;
        c_res[k] = ((b.ng > b.nbflags ? b.ng : b.nbflags) + 255) / 256;
        c_codes[k] = (long long)b.nbl + b.ntv;
        c_scat[k] = ngg + ngv;
    }
    unsigned t_range = 0, t_res = 0, t_codes = 0, t_scat = 0;
    const std::vector<unsigned> b_range = bases(c_range, &t_range), b_res = bases(c_res, &t_res),
                                b_codes = bases(c_codes, &t_codes), b_scat = bases(c_scat, &t_scat);
    mck::BItemC* dd = nullptr;
    unsigned *db_range = nullptr, *db_res = nullptr, *db_codes = nullptr, *db_scat = nullptr;
    if (nb > 0) {
        if (e == hipSuccess) e = gupload(bg, &dd, d);
        if (e == hipSuccess) e = gupload(bg, &db_range, b_range);
        if (e == hipSuccess) e = gupload(bg, &db_res, b_res);
        if (e == hipSuccess) e = gupload(bg, &db_codes, b_codes);
        if (e == hipSuccess) e = gupload(bg, &db_scat, b_scat);
    }
    if (e != hipSuccess) {
        destroy_graph(bg);
        return mc_fail(MC_ERR_NOMEM, "batch workspace: %s", hipGetErrorString(e));
    }
    bg->n_batched = nb;
    return capture(bg, ip, chained, [&](int i, hipStream_t s) {
        return mc_compress_enqueue(items[i].plan, items[i].d_field, items[i].dtype, &items[i].params,
                                   &items[i].codes, s);
    }, [&](hipStream_t s) -> mc_status {
        if (nb == 0) return MC_OK;
        hipError_t e2;
#define BCHK(x) do { if ((e2 = (x)) != hipSuccess) return mc_fail(MC_ERR_DEVICE, "%s: %s", #x, hipGetErrorString(e2)); } while (0)
        BCHK(mck::batch_range(dd, db_range, nb, t_range, s));
        BCHK(mck::batch_range_final(dd, nb, s));
        BCHK(mck::batch_resample(dd, db_res, nb, t_res, s));
        BCHK(mck::batch_codes(dd, db_codes, nb, t_codes, s));
        BCHK(mck::batch_scatter(dd, db_scat, nb, t_scat, s));
#undef BCHK
        return MC_OK;
    }, [](hipStream_t) { return MC_OK; }, stream);
}

extern "C" mc_status mc_batch_decompress(const mc_batch_ditem* items, int32_t n, hipStream_t stream)
{
    if (!items || n <= 0) return mc_fail(MC_ERR_ARG, "invalid batch (items NULL or n <= 0)");
    for (int32_t i = 0; i < n; ++i) {
        mc_status st = mc_check_decompress(items[i].plan, &items[i].codes, items[i].model, items[i].d_out,
                                           items[i].dtype);
        if (st != MC_OK) return mc_fail(st, "batch item %d: %s", i, mc_last_error());
    }
    std::vector<unsigned char> key = key_of(items, n);
    std::lock_guard<std::mutex> lk(g_bm);
    mc_status st;
    if (replay(1, key, stream, &st)) return st;
    BatchGraph* bg = new BatchGraph();
    bg->kind = 1;
    bg->key = std::move(key);
    std::vector<mc_plan> ip(n);
    std::vector<int> all(n);
    std::vector<float*> xh(n, nullptr);                 // decoded grid of each batched field
    std::vector<mck::BItemD> d;
    std::vector<long long> cnt;
    hipError_t e = hipSuccess;
    for (int32_t i = 0; i < n; ++i) {
        ip[i] = items[i].plan;
        all[i] = i;
        bg->refs.push_back(items[i].plan);
        if (items[i].model) bg->refs.push_back(items[i].model);
        if (!batched_decompress(items[i]) || e != hipSuccess) continue;
        const mc_plan p = items[i].plan;
        e = gdev(bg, &xh[i], (size_t)p->ng);
        mck::BItemD b{};
        b.cls = 2 * (items[i].dtype == MC_F64 ? 1 : 0) + (p->dim == 3 ? 1 : 0);
        b.knobs = p->knobs;
        b.nv = p->nv;
        b.vcap = items[i].codes.v_out_cap;
        b.gg = p->gg;
        b.coords = p->coords;
        b.xh = xh[i];
        b.vcodes = items[i].codes.vert_codes;
        b.vidx = items[i].codes.v_out_idx;
        b.vval = items[i].codes.v_out_val;
        b.res = items[i].codes.result;
        b.xout = items[i].d_out;
        d.push_back(b);
        cnt.push_back((p->nv + MC_TILE - 1) / MC_TILE);
    }
    const int nb = (int)d.size();
    unsigned total = 0;
    const std::vector<unsigned> base = bases(cnt, &total);
    mck::BItemD* dd = nullptr;
    unsigned* db = nullptr;
    if (nb > 0 && e == hipSuccess) e = gupload(bg, &dd, d);
    if (nb > 0 && e == hipSuccess) e = gupload(bg, &db, base);
    if (e != hipSuccess) {
        destroy_graph(bg);
        return mc_fail(MC_ERR_NOMEM, "batch workspace: %s", hipGetErrorString(e));
    }
    bg->n_batched = nb;
    return capture(bg, ip, all, [&](int i, hipStream_t s) -> mc_status {
        if (!xh[i])
            return mc_decompress_enqueue(items[i].plan, &items[i].codes, items[i].model, items[i].d_out,
                                         items[i].dtype, s);
        return mc_grid_decode_enqueue(items[i].plan, &items[i].codes, xh[i], s);     // the vertex decode is batched
    }, [](hipStream_t) { return MC_OK; }, [&](hipStream_t s) -> mc_status {
        if (nb == 0) return MC_OK;
        hipError_t e2 = mck::batch_vdecode(dd, db, nb, total, s);
        return e2 == hipSuccess ? MC_OK : mc_fail(MC_ERR_DEVICE, "batch_vdecode: %s", hipGetErrorString(e2));
    }, stream);
}

// Drops the cached graphs that use a plan or model about to be destroyed
// (a later object at the same address must not replay a stale graph).
void mc_batch_forget(const void* obj)
{
    std::lock_guard<std::mutex> lk(g_bm);
    bool synced = false;
    for (size_t i = 0; i < g_graphs.size();) {
        const std::vector<const void*>& r = g_graphs[i]->refs;
        if (std::find(r.begin(), r.end(), obj) == r.end()) { ++i; continue; }
        if (!synced) (void)hipDeviceSynchronize();
        synced = true;
        destroy_graph(g_graphs[i]);
        g_graphs.erase(g_graphs.begin() + i);
    }
}

extern "C" mc_status mc_batch_graph_info(int32_t kind, const void* items, int32_t n, int32_t* n_batched,
                                         int64_t* n_nodes)
{
    if (!items || n <= 0 || (kind != 0 && kind != 1)) return mc_fail(MC_ERR_ARG, "invalid batch query");
    const size_t isz = kind == 0 ? sizeof(mc_batch_item) : sizeof(mc_batch_ditem);
    std::vector<unsigned char> key((const unsigned char*)items, (const unsigned char*)items + isz * (size_t)n);
    std::lock_guard<std::mutex> lk(g_bm);
    for (BatchGraph* g : g_graphs)
        if (g->kind == kind && g->key == key) {
            if (n_batched) *n_batched = g->n_batched;
            if (n_nodes) {
                size_t nn = 0;
                hipError_t e = hipGraphGetNodes(g->graph, nullptr, &nn);
                if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "hipGraphGetNodes: %s", hipGetErrorString(e));
                *n_nodes = (int64_t)nn;
            }
            return MC_OK;
        }
    return mc_fail(MC_ERR_ARG, "no cached graph for this item list");
}

extern "C" mc_status mc_batch_release(void)
{
    std::lock_guard<std::mutex> lk(g_bm);
    (void)hipDeviceSynchronize();
    for (BatchGraph* g : g_graphs) destroy_graph(g);
    g_graphs.clear();
    return MC_OK;
}
