// mc_batch.hip -- batched compression and decompression of many fields on
// many plans.
//
// The first call with a given item list captures the whole batch into one
// HIP graph and later calls replay it (a single graph launch per batch).
// The capture forks one chain per distinct plan: fields on the same mesh
// run in order on their chain (they share the plan's workspace), chains of
// different meshes run concurrently, and the chains join before the graph
// ends; the graph is launched on the caller's stream.  Chains are ordered
// largest plan first, so the longest chain starts first.  Every kernel of
// the compress and decompress sequences is capturable: the per-call state is
// cleared by a kernel, never by a memset node.
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

// Captures enqueue(i, s) for every item i on one chain per distinct plan,
// instantiates the graph, launches it on `stream` and caches it.  Caller
// holds g_bm.
mc_status capture(int kind, std::vector<unsigned char> key, const std::vector<mc_plan>& item_plan,
                  std::vector<const void*> refs, const std::function<mc_status(int, hipStream_t)>& enqueue,
                  hipStream_t stream)
{
    const int n = (int)item_plan.size();
    std::vector<mc_plan> plans;
    for (mc_plan p : item_plan)
        if (std::find(plans.begin(), plans.end(), p) == plans.end()) plans.push_back(p);
    std::stable_sort(plans.begin(), plans.end(), [](mc_plan a, mc_plan b) { return a->nv + a->ng > b->nv + b->ng; });

    // Capture happens on a private origin stream (the caller's stream may be
    // the null stream, which cannot be captured).  Chain 0 runs on it.
    BatchGraph* bg = new BatchGraph();
    bg->kind = kind;
    bg->key = std::move(key);
    bg->refs = std::move(refs);
    const size_t nc = plans.size();
    hipError_t e = hipSuccess;
    for (size_t c = 0; c < nc && e == hipSuccess; ++c) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) bg->streams.push_back(s);
    }
    for (size_t c = 0; c < nc && e == hipSuccess; ++c) {
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
    if (e == hipSuccess && nc > 1) e = hipEventRecord(bg->events[0], origin);      // fork
    for (size_t c = 1; c < nc && e == hipSuccess; ++c)
        e = hipStreamWaitEvent(bg->streams[c], bg->events[0], 0);
    for (size_t c = 0; c < nc && e == hipSuccess && st == MC_OK; ++c)
        for (int i = 0; i < n && st == MC_OK; ++i)
            if (item_plan[i] == plans[c]) st = enqueue(i, bg->streams[c]);
    for (size_t c = 1; c < nc && e == hipSuccess; ++c) {                           // join
        e = hipEventRecord(bg->events[c], bg->streams[c]);
        if (e == hipSuccess) e = hipStreamWaitEvent(origin, bg->events[c], 0);
    }
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
    std::vector<mc_plan> ip(n);
    std::vector<const void*> refs;
    for (int32_t i = 0; i < n; ++i) {
        ip[i] = items[i].plan;
        refs.push_back(items[i].plan);
        if (items[i].params.model) refs.push_back(items[i].params.model);
    }
    return capture(0, std::move(key), ip, std::move(refs), [&](int i, hipStream_t s) {
        return mc_compress_enqueue(items[i].plan, items[i].d_field, items[i].dtype, &items[i].params,
                                   &items[i].codes, s);
    }, stream);
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
    std::vector<mc_plan> ip(n);
    std::vector<const void*> refs;
    for (int32_t i = 0; i < n; ++i) {
        ip[i] = items[i].plan;
        refs.push_back(items[i].plan);
        if (items[i].model) refs.push_back(items[i].model);
    }
    return capture(1, std::move(key), ip, std::move(refs), [&](int i, hipStream_t s) {
        return mc_decompress_enqueue(items[i].plan, &items[i].codes, items[i].model, items[i].d_out,
                                     items[i].dtype, s);
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

extern "C" mc_status mc_batch_release(void)
{
    std::lock_guard<std::mutex> lk(g_bm);
    (void)hipDeviceSynchronize();
    for (BatchGraph* g : g_graphs) destroy_graph(g);
    g_graphs.clear();
    return MC_OK;
}
