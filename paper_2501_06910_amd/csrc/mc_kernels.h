// mc_kernels.h -- internal interface between the host API (mc_api.hip) and
// the kernel files.  Launchers enqueue on the given stream and return the
// HIP error of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mc.h"
#include "mc_dev.h"

// True while the calling thread captures a batch graph (mc_batch.hip).
extern thread_local bool mc_capturing;

namespace mck {

// ---- profiling hook (mc_api.hip) -------------------------------------------
// Records a pair of events around one launch when profiling is on and the
// calling thread is not capturing a graph.
struct ProfScope {
    const char* name;
    hipStream_t stream;
    int idx;
    ProfScope(const char* n, hipStream_t s);
    ~ProfScope();
};

// ---- plan construction (k_plan.hip) ---------------------------------------
hipError_t bbox(const float* coords, int dim, long long nv, unsigned int* keys /*[6]*/, hipStream_t s);
hipError_t bins_count(const float* coords, const int32_t* cells, int dim, long long nv, long long nc,
                      GridGeom gg, const double* o, const double* h, int B, int nb0, int nb1, int nb2,
                      unsigned int* bin_count, unsigned int* bad_cells, hipStream_t s);
hipError_t bins_fill(const float* coords, const int32_t* cells, int dim, long long nv, long long nc,
                     GridGeom gg, const double* o, const double* h, int B, int nb0, int nb1, int nb2,
                     const long long* bin_start, unsigned int* cursor, int32_t* list, hipStream_t s);
hipError_t scan_u32(const unsigned int* in, long long n, long long* out /*[n+1]*/, unsigned long long* st,
                    unsigned int* ticket, hipStream_t s);
hipError_t locate(const float* coords, const int32_t* cells, int dim, long long nv, long long nc, GridGeom gg,
                  int B, int nb0, int nb1, const long long* bin_start, const int32_t* list,
                  int32_t* vid, float* w, int32_t* cell, int32_t* unres, unsigned int* n_unres,
                  unsigned int* n_neardeg, hipStream_t s);
hipError_t vbins_count(const float* coords, int dim, long long nv, const double* o, const double* h, int VB,
                       int nb0, int nb1, int nb2, unsigned int* cnt, hipStream_t s);
hipError_t vbins_fill(const float* coords, int dim, long long nv, const double* o, const double* h, int VB,
                      int nb0, int nb1, int nb2, const long long* start, unsigned int* cursor, int32_t* list,
                      hipStream_t s);
hipError_t fill_nearest(const float* coords, int dim, long long nv, GridGeom gg, const double* o,
                        const double* h, int VB, int nb0, int nb1, int nb2, const long long* vstart,
                        const int32_t* vlist, const int32_t* unres, long long n_unres, int32_t* vid, float* w,
                        long long ng, hipStream_t s);
hipError_t fill_midrange(int dim, const int32_t* unres, long long n_unres, int32_t* vid, float* w, long long ng,
                         hipStream_t s);

// ---- compression (k_compress.hip) -----------------------------------------
// Field range and error split (k_range, then one workgroup folds the partials).
// knobs: the partial-block count (partial holds 3 * MC_RANGE_BLOCKS words)
hipError_t range(const void* x, int dtype, long long n, unsigned long long* partial, RangeOut* cur, BoundParams bp,
                 DevBound* bnd, unsigned int* zero, long long nzero, unsigned knobs, hipStream_t s);
// xh may be NULL (x1' not written)
hipError_t resample(const int32_t* vid, const float* w, int dim, long long ng, const void* x, int dtype,
                    const DevBound* bnd, int32_t* p, float* xh, float* dbg_v, uint32_t* bflags,
                    long long nbflags, unsigned int* err, mc_result* res, unsigned int* gcount, long long ntg,
                    unsigned remap, hipStream_t s);
hipError_t lorenzo(const int32_t* p, int dim, int n0, int n1, int n2, long long ng, uint16_t* codes,
                   unsigned int* count, unsigned int* gsum, unsigned remap, hipStream_t s);
// Lorenzo grid codes and plain vertex residual codes in one launch (see
// lorenzo and residual; pq as for residual).
hipError_t codes(const int32_t* p, int dim, int n0, int n1, int n2, uint16_t* gcodes, unsigned int* gcount,
                 unsigned int* gsum, const float* coords, long long nv, GridGeom gg, const float* xh,
                 const int32_t* pq, const void* x, int dtype, const DevBound* bnd, uint16_t* vcodes, float* dbg_g,
                 unsigned int* vcount, unsigned int* vsum, unsigned remap, hipStream_t s);
// pq non-NULL (plain codes only): the cell corners are read from the
// prequantised grid and converted as x1' = (float)(c + p * 2 tau1); else
// from x1' (xh).
hipError_t residual(const float* coords, long long nv, GridGeom gg, const float* xh, const int32_t* pq,
                    const void* x, int dtype, const DevBound* bnd, uint16_t* codes, float* dbg_g,
                    unsigned int* count, unsigned int* vsum, unsigned remap, hipStream_t s);
// x1' = (float)(c + p * 2 tau1) over the whole grid (bound from bnd).
hipError_t xhat_from_p(const int32_t* p, long long ng, const DevBound* bnd, float* xh, hipStream_t s);
// gpred: the mc_grid_predictor whose errors the grid outliers carry (gref:
// the time-axis predictor's reference grid)
hipError_t compact(const int32_t* p, int dim, int n0, int n1, long long ng, int gpred, const float* gref,
                   const uint16_t* gcodes,
                   unsigned int* gcount, unsigned int* gsum, int32_t* gidx, int32_t* gdelta, long long gcap,
                   const void* x, int dtype,
                   long long nv, const uint16_t* vcodes, unsigned int* vcount, unsigned int* vsum, int32_t* vidx,
                   void* vval, long long vcap, unsigned int* err, mc_result* res, hipStream_t s);

// ---- batched stages (work lists over many fields) --------------------------
// One field of a batched compress, as the stage kernels read it (a device
// array of these, built by the batch layer).  The field's own workspace
// (range partials, control block, per-call counters, per-tile counts, p)
// belongs to the batch, so fields on one plan may run in the same launch.
struct BItemC {
    int cls;                          // 2 * (dtype == MC_F64) + (dim == 3)
    int vec;                          // field 16-byte aligned (range loads)
    int n0, n1, n2;
    int nxs, nyb;                     // Lorenzo units: 63-column runs, row blocks (3-D)
    unsigned nunits, nbl;             // Lorenzo units and their blocks (4 units per block)
    unsigned nparts;                  // range blocks (partials)
    unsigned knobs;                   // the plan's launch knobs (cache policy; tile order is launch order)
    long long ng, nv, ntg, ntv, nsmall, nbflags, gcap, vcap;
    GridGeom gg;
    BoundParams bp;
    const int32_t* vid;
    const float* w;
    const float* coords;
    const void* x;
    unsigned long long* partial;      // [3 * nparts]
    RangeOut* cur;
    DevBound* bnd;
    unsigned* small;                  // err at 2, grid group sums from 16, vertex group sums after them
    unsigned* gcount;                 // [ntg]
    unsigned* vcount;                 // [ntv]
    int32_t* p;                       // [ng]
    uint16_t* gcodes;
    int32_t* gidx;
    int32_t* gdelta;
    uint16_t* vcodes;
    int32_t* vidx;
    void* vval;
    mc_result* res;
    uint32_t* bflags;
};
// Lorenzo work units of a grid (63-column runs x row blocks x plane chunks in
// 3-D, x row chunks in 2-D), as k_lorenzo3 / k_lorenzo and k_codes take them.
void lorenzo_units(int dim, int n0, int n1, int n2, int* nxs, int* nyb, unsigned* nunits);
// Stage launches of a batched compress: block ranges per field are given by
// base tables (base[i] = first block of field i, base[n] = total blocks).
hipError_t batch_range(const BItemC* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s);
hipError_t batch_range_final(const BItemC* items, int n, hipStream_t s);
hipError_t batch_resample(const BItemC* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s);
hipError_t batch_codes(const BItemC* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s);
hipError_t batch_scatter(const BItemC* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s);

// One field of a batched vertex decode.
struct BItemD {
    int cls;                          // 2 * (dtype == MC_F64) + (dim == 3)
    unsigned knobs;
    long long nv, vcap;
    GridGeom gg;
    const float* coords;
    const float* xh;                  // the field's decoded grid
    const uint16_t* vcodes;
    const int32_t* vidx;
    const void* vval;
    const mc_result* res;
    void* xout;
};
hipError_t batch_vdecode(const BItemD* items, const unsigned* base, int n, unsigned nblocks, hipStream_t s);

// ---- decompression (k_decode.hip) -----------------------------------------
// Launch knobs (results do not depend on them): bit k set = kernel k takes
// its tiles in XCD-contiguous order (xcd_tile), clear = in launch order;
// bits 7 and 8 the cache policy of streamed arrays; bits 9-10 and 11-12
// launch shapes.  Chosen per plan by mc_plan_tune.
enum {
    MC_KNOB_RESAMPLE = 1u << 0,
    MC_KNOB_LORENZO = 1u << 1,
    MC_KNOB_RESIDUAL = 1u << 2,
    MC_KNOB_VDECODE = 1u << 3,
    MC_KNOB_DZTOT = 1u << 4,        // 3-D decode on x quads: tile sums
    MC_KNOB_DZAPPLY = 1u << 5,      // 3-D decode on x quads: apply
    MC_KNOB_DXYAPPLY = 1u << 6,     // no kernel reads it (kept so the mask keeps its meaning)
    MC_KNOB_NT_MAP = 1u << 7,       // resample: the mapping streamed with the non-temporal policy
    MC_KNOB_NT_VERT = 1u << 8,      // residual codes and vertex decode: coordinates, field, codes and
                                    // decoded values streamed with the non-temporal policy
    MC_KNOB_VPT = 3u << 9,          // vertex decode, vertices per thread: 0 -> 4, 1 -> 2, 2 -> 8, 3 -> 4
    MC_KNOB_RANGE = 3u << 11,       // field range, partial blocks: 0 -> 2048, 1 -> 1024, 2 -> 512, 3 -> 2048
    MC_KNOB_ALL = 0x1fffu,          // every valid bit
    MC_KNOB_DEFAULT = 0x1ecu        // a new plan: on the 16M-vertex tet mesh launch order for resample and
                                    // Lorenzo, XCD order for the vertex kernels (same time as launch order,
                                    // each grid line fetched once per pass instead of 1.4x) and for the
                                    // 3-D decode, non-temporal streams, 4 vertices per thread, 2048 range
                                    // blocks
};

// Launch shapes of a knob word.
inline int knob_vpt(unsigned k)
{
    const unsigned f = (k & MC_KNOB_VPT) >> 9;
    return f == 1u ? 2 : (f == 2u ? 8 : 4);
}
inline int knob_range_blocks(unsigned k)
{
    const unsigned f = (k & MC_KNOB_RANGE) >> 11;
    return f == 1u ? MC_RANGE_BLOCKS / 2 : (f == 2u ? MC_RANGE_BLOCKS / 4 : MC_RANGE_BLOCKS);
}

#define MC_D2_R 8                  // 2-D decode: rows per chunk (rows of DecodeWs in 2-D)
struct DecodeWs {
    bool fast3;                    // 3-D with n0 <= 1024: the quad kernels
    int pitch;                     // row pitch of the workspace arrays: n0, rounded up to 4 on the quad path
    int rows, nyc;                 // rows per tile, row chunks per plane
    long long ntiles_xy;           // nyc * n2
    int* agg_xy;                   // [ntiles_xy][pitch] column totals, then carries
    int zplanes, nzc;              // 3-D: planes per chunk, plane chunks
    int* agg_z;                    // [nzc][pitch*n1] chunk totals, then carries
    int* agg_t;                    // 3-D quads: [nyc][nzc][pitch] tile totals, then their 2-D exclusive prefix
    int* segsum;                   // 2-D: [n1][ceil(n0 / 256)] row-segment sums
};
// ---- multilevel interpolation grid predictor (k_interp.hip) ---------------
// Codes of the prequantised grid p (outliers counted per tile, as lorenzo).
hipError_t interp_codes(const int32_t* p, int n0, int n1, int n2, long long ng, bool cubic, uint16_t* codes,
                        unsigned int* count, unsigned int* gsum, hipStream_t s);
// p and x1' from the codes and outliers (all nodes written).
hipError_t interp_decode(const uint16_t* codes, const int32_t* oidx, const int32_t* odelta, long long gcap,
                         const mc_result* res, int dim, int n0, int n1, int n2, bool cubic, int32_t* p, float* xh,
                         hipStream_t s);

// Time-axis predictor from the reference grid ref (k_interp.hip).
hipError_t temporal_codes(const int32_t* p, const float* ref, const DevBound* bnd, long long ng, uint16_t* codes,
                          unsigned int* count, unsigned int* gsum, hipStream_t s);
hipError_t temporal_decode(const uint16_t* codes, const int32_t* oidx, const int32_t* odelta, long long gcap,
                           const mc_result* res, const float* ref, long long ng, int32_t* p, float* xh, hipStream_t s);

hipError_t grid_decode(const uint16_t* codes, const int32_t* oidx, const int32_t* odelta, long long gcap,
                       const mc_result* res, int dim, int n0, int n1, int n2, int32_t* pz, float* xh, DecodeWs& ws,
                       unsigned remap, hipStream_t s);
hipError_t vertex_decode(const float* coords, long long nv, GridGeom gg, const float* xh, const uint16_t* codes,
                         const int32_t* oidx, const void* oval, long long vcap, const mc_result* res, void* xout,
                         int dtype, unsigned remap, hipStream_t s);

// ---- 1-D serialisation baseline (k_serial.hip) ----------------------------
hipError_t serial_codes(const void* x, int dtype, long long n, const DevBound* bnd, uint16_t* codes, unsigned* count,
                        unsigned* vsum, unsigned* err, mc_result* res, hipStream_t s);
// agg: int2[], carry: int[], at least ceil(n / MC_TILE) entries each
hipError_t serial_decode(const uint16_t* codes, const int32_t* oidx, const void* oval, long long vcap,
                         const mc_result* res, long long n, int dtype, int2* agg, int* carry, void* out, hipStream_t s);

// ---- residual codes with the 1-D Lorenzo predictor (k_resdelta.hip) -------
// m == NULL: g by multilinear back-interpolation; else g = xh[m[v]] (nearest node)
hipError_t residual_delta(const float* coords, long long nv, GridGeom gg, const float* xh, const int32_t* m,
                          const void* x, int dtype, const DevBound* bnd, uint16_t* codes, float* dbg_g,
                          unsigned* count, unsigned* vsum, unsigned* err, hipStream_t s);
// agg: int2[ceil(nv / MC_TILE)], carry: int[ceil(nv / MC_TILE)]
hipError_t vertex_decode_delta(const float* coords, long long nv, GridGeom gg, const float* xh, const int32_t* m,
                               const uint16_t* codes,
                               const int32_t* oidx, const void* oval, long long vcap, const mc_result* res,
                               int2* agg, int* carry, void* xout, int dtype, hipStream_t s);
// exclusive segmented scan of tile aggregates from a restart at 0 (k_serial.hip)
hipError_t seg_carry(const int2* agg, long long ntiles, int* carry, hipStream_t s);

// ---- grid initialisation (k_grid_init.hip) --------------------------------
// Histogram (hist: 2^nbits u64 bins, zeroed by the caller) of bits
// [shift, shift + nbits) of the FP32 edge extents along `axis` whose bits
// under pmask equal pval; *bad |= 1 for a cell with an invalid vertex id.
hipError_t edge_hist(const float* coords, const int32_t* cells, int dim, long long nv, long long nc, int axis,
                     unsigned shift, unsigned nbits, unsigned pmask, unsigned pval, unsigned long long* hist,
                     unsigned* bad, hipStream_t s);

// ---- nearest-node g and cluster-mean f (k_cluster.hip) --------------------
struct NodeGeom {
    double o[3], h[3];
    long long n[3];
};
hipError_t nearest_nodes(const float* coords, int dim, long long nv, NodeGeom g, int32_t* m, unsigned* count,
                         hipStream_t s);
// Grid_Coarsen: mark the planes holding a node (flags int[n0 + n1 + n2],
// zeroed by the caller); remap the nodes to the coarsened grid through keep
// (new index per plane) and count the vertices per coarsened node.
hipError_t mark_planes(const int32_t* m, long long nv, int n0, int n1, int n2, int* flags, hipStream_t s);
hipError_t remap_nodes(int32_t* m, long long nv, int n0, int n1, const int* keep, int c0, int c1, unsigned* count,
                       hipStream_t s);
hipError_t count_empty(const unsigned* count, long long ng, unsigned* out, hipStream_t s);
// Stable sort of the vertices by node (temp == NULL: *temp_bytes receives the size).
hipError_t sort_by_node(const int32_t* m, long long nv, long long ng, uint32_t* keys_out, int32_t* vlist,
                        void* temp, size_t* temp_bytes, hipStream_t s);
hipError_t cluster_mean(const long long* noff, const int32_t* vlist, long long ng, const void* x, int dtype,
                        const DevBound* bnd, int32_t* p, float* xh, double* x1, float* dbg_v, unsigned* err,
                        mc_result* res, unsigned* gcount, long long ntg, hipStream_t s);
// x1 == NULL: closed loop (against the reconstructed grid xhat), else open loop (against x1)
hipError_t residual_nearest(const int32_t* m, long long nv, const void* x, int dtype, const double* x1,
                            const float* xhat, const DevBound* bnd, uint16_t* codes, float* dbg_g, unsigned* count,
                            unsigned* vsum, hipStream_t s);
hipError_t vertex_decode_nearest(const int32_t* m, long long nv, const float* xhat, const uint16_t* codes,
                                 const int32_t* oidx, const void* oval, long long vcap, const mc_result* res,
                                 void* xout, int dtype, hipStream_t s);

// ---- learned predictor (k_mlp.hip) ----------------------------------------
struct MlpDev {
    int dim, kin, kpad;
    float kappa;
    const uint16_t* w1;   // bf16 [64][kpad] (output-major, zero padded)
    const uint16_t* w2;   // bf16 [64][64]
    const uint16_t* w3;   // bf16 [64][64]
    const uint16_t* w4;   // bf16 [64]
    const float* b1; const float* b2; const float* b3; const float* b4;
    void* img;            // the weights as MFMA A fragments (k_mlp.hip), mlp_image_bytes(dim)
};
hipError_t mlp_pack(const float* params, int dim, uint16_t* w1, uint16_t* w2, uint16_t* w3, uint16_t* w4,
                    float* b1, float* b2, float* b3, float* b4, hipStream_t s);
// Learned vertex codes (network, block choice, codes, tile counts) in one
// launch; rho_out optional.
hipError_t mlp_residual(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh,
                        const void* x, int dtype, const DevBound* bnd, uint16_t* codes, uint32_t* bflags,
                        float* dbg_g, int32_t* rho_out, unsigned int* count, unsigned int* vsum, hipStream_t s);
// Learned decompress of every vertex (network shifts in learned blocks).
hipError_t mlp_vdecode(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh,
                       const uint32_t* bflags, const uint16_t* codes, const int32_t* oidx, const void* oval,
                       const mc_result* res, long long vcap, void* xout, int dtype, hipStream_t s);
hipError_t mlp_features(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh, long long v0,
                        long long count, float* z, hipStream_t s);
hipError_t mlp_forward_z(const MlpDev& m, const float* z, long long batch, float* rho, hipStream_t s);
hipError_t mlp_feature_sumsq(const float* coords, long long nv, GridGeom gg, const float* xh, int dim,
                             double* partial, int nblocks, hipStream_t s);
size_t mlp_image_bytes(int dim);
// Builds m.img from the row-major weights and biases of m.
hipError_t mlp_image(const MlpDev& m, hipStream_t s);
// training: samples of steps [t0, t0 + nsteps) as input fragments
// (train_sample_bytes per step) and targets [nsteps][batch]
size_t train_sample_bytes(int dim, long long batch);
hipError_t train_sample(const MlpDev& m, const float* coords, long long nv, GridGeom gg, const float* xh,
                        const mc_result* res, const void* x, int dtype, long long batch, unsigned long long seed,
                        long long t0, long long nsteps, void* zfr, float* y, hipStream_t s);
// given inputs [batch][kpad] and targets -> the same layout (ypad: whole 64-sample parts)
hipError_t train_zfrag(int dim, const float* z, const float* y, long long batch, void* zfr, float* ypad,
                       hipStream_t s);
// one workgroup per 64 samples writes its gradient to grad_part[part]
hipError_t train_grad(const MlpDev& m, const void* zfr, const float* y, long long batch, float* grad_part,
                      float* loss_part, hipStream_t s);
// fixed-order sum of the parts; with apply, Adam on params and the new
// weights into m's row-major arrays and image
hipError_t train_adam(const MlpDev& m, int nparts, const float* grad_part, const float* loss_part, float* grad,
                      float* loss_out, float* params, float* mom, float* vel, long long t, float lr, int apply,
                      long long batch, hipStream_t s);

}  // namespace mck
