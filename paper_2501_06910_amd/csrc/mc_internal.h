// mc_internal.h -- host-side objects behind the opaque handles of mc.h.
#pragma once
#include <vector>

#include "mc_kernels.h"

struct mc_plan_s {
    int dim = 0;
    long long nv = 0, nc = 0, ng = 0;
    mc_grid grid{};
    GridGeom gg{};
    int fill = 0;
    int B = 1;
    int ops = MC_OPS_LINEAR;       // operator pair (mc_plan_opts.operators)
    int coarsen = 0;               // Grid_Coarsen applied (mc_plan_opts.coarsen)
    std::vector<int32_t> keep;     // per original plane: coarsened index or -1 (coarsen only)
    // nearest-node / cluster-mean pair (device)
    int32_t* m = nullptr;          // nearest node of every vertex [nv]
    int32_t* vlist = nullptr;      // vertices sorted by node, ascending ids within a node [nv]
    long long* noff = nullptr;     // node j's vertices: vlist[noff[j] .. noff[j+1]) [ng + 1]
    double* x1 = nullptr;          // cluster means of the current call [ng] (open loop)
    int2* dagg = nullptr;          // residual delta decode: tile aggregates [ntv]
    int* dcarry = nullptr;         // and their exclusive scan [ntv]
    // mapping (device)
    float* coords = nullptr;       // [dim][nv] copy
    int32_t* vid = nullptr;        // [dim+1][ng]
    float* w = nullptr;            // [dim+1][ng]
    int32_t* cell = nullptr;       // [ng]
    // workspace (device)
    int32_t* p = nullptr;          // prequantised grid [ng]
    float* xh = nullptr;           // reconstructed grid x1' [ng]
    bool xh_valid = false;         // xh holds the x1' of the last enqueued call (a plain
                                   // compression writes only p: mc_plan_ensure_xh converts)
    unsigned long long* range_partial = nullptr;   // [3 * MC_RANGE_BLOCKS]
    unsigned long long* ctl = nullptr;   // 64 words: the two range slots
    RangeOut* rbuf = nullptr;            // field range of the current call
    DevBound* bound = nullptr;           // error split of the current call (in ctl)
    unsigned* small = nullptr;           // per-call state cleared by k_range (u32 words)
    long long nsmall = 0;
    unsigned* err = nullptr;             // small[2]
    unsigned* counts = nullptr;          // per-tile outlier counts and offsets
    unsigned* gcount = nullptr;
    unsigned* vcount = nullptr;
    unsigned* gsum = nullptr;            // outliers per group of tiles (in small)
    unsigned* vsum = nullptr;
    long long ntg = 0, ntv = 0, nblk = 0;
    mck::DecodeWs dws{};
    unsigned knobs = mck::MC_KNOB_DEFAULT;  // launch knobs (mc_plan_tune)
    // statistics
    long long n_unresolved = 0, n_near_degenerate = 0, n_pairs = 0;
    int invalid_cells = 0;
    size_t bytes = 0;
    std::vector<void*> allocs;
};

struct mc_model_s {
    int dim = 0, kin = 0, kpad = 0;
    float kappa = 1.0f;
    std::vector<float> params;     // host FP32 master copy
    void* dev = nullptr;           // packed device weights (bf16 + fp32 biases)
    mck::MlpDev md{};
};

mc_status mc_fail(mc_status s, const char* fmt, ...);
mc_status mc_check_grid(const mc_grid* g, int32_t dim);
GridGeom mc_geom(const mc_grid& g);
// Drops cached batch graphs that reference a plan or model (mc_batch.hip).
void mc_batch_forget(const void* obj);

mc_status mc_check_decompress(mc_plan p, const mc_codes* codes, mc_model model, const void* d_out, mc_dtype dtype);
mc_status mc_decompress_enqueue(mc_plan p, const mc_codes* codes, mc_model model, void* d_out, mc_dtype dtype,
                                hipStream_t s);
// The grid part of a decompress (Alg. 4: x1' = D(mu1)) into xh (the plan's
// x1' or a caller buffer of n_grid floats); the plan's p and decode
// workspace are used, so calls on one plan must be ordered.
mc_status mc_grid_decode_enqueue(mc_plan p, const mc_codes* codes, float* xh, hipStream_t s);
mc_status mc_check_params(mc_plan p, const void* d_field, mc_dtype dtype, const mc_params* prm,
                          const mc_codes* codes);
mc_status mc_compress_enqueue(mc_plan p, const void* d_field, mc_dtype dtype, const mc_params* prm,
                              const mc_codes* codes, hipStream_t s);
int mc_model_dim(mc_model m);
// Makes p->xh the x1' of the last enqueued compression (converting p when
// that call wrote only p).  Stream-ordered.
mc_status mc_plan_ensure_xh(mc_plan p, hipStream_t s);
