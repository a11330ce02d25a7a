/*
 * mc.h -- C ABI of the MI355X (gfx950) multi-component error-bounded
 * compressor for values on unstructured triangle / tetrahedral meshes
 * (Gong et al., "A General Framework for Error-controlled Unstructured
 * Scientific Data Compression").
 *
 * The method (paper Sec. III, Sec. IV-B..IV-E, Algorithms 3 and 4):
 * vertex values x are resampled onto a rectilinear grid (x1 = f(x)), the
 * grid is compressed with bound tau1, the reconstructed grid x1' is
 * interpolated back to the vertices (g, non-negative weights summing to one)
 * and the residuals x - g(x1') are compressed with bound tau2, so every
 * reconstructed vertex x' = g(x1') + x2' satisfies |x - x'| <= tau2 <= tau
 * (Sec. III).  f is barycentric interpolation in the lowest-numbered cell
 * containing the node (the "linear interpolation" f of Sec. IV-D); g is
 * multilinear interpolation; the grid compressor is a Lorenzo predictor on
 * prequantised integers with linear quantisation (the SZ-family predictor
 * named in Sec. II); the residual compressor is linear quantisation with a
 * per-vertex bound check.  An optional learned predictor (a small MLP)
 * shifts residual codes per 4096-vertex block without changing the bound.
 *
 * Conventions
 *  - Pointers prefixed d_ are device (HBM) pointers, h_ are host pointers.
 *  - Layouts are structure-of-arrays: coordinates float[dim][n_vertices],
 *    cells int32[dim+1][n_cells] (0-based vertex ids), grid arrays with
 *    linear index i0 + n0*(i1 + n1*i2) (x fastest).
 *  - Calls marked (sync) block the host; all others only enqueue work on the
 *    given HIP stream and return.  Host-detectable argument errors return
 *    before any HIP call.  Errors found on the device (NaN/Inf in the field,
 *    integer range, outlier capacity) are written to mc_result.status and
 *    are visible once the stream has been synchronised.
 *  - The caller owns every buffer it passes; buffers must stay alive until
 *    the stream has finished using them.  Plans and models are owned by the
 *    library (mc_plan_destroy / mc_model_destroy).
 *  - Calls on one plan use that plan's device workspace: they must be
 *    ordered on one stream (overlapping calls on one plan race).
 *  - No C++ exception crosses this ABI; mc_last_error() gives the text of
 *    the last host-side failure of the calling thread.
 */
#ifndef MC_H
#define MC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MC_OK = 0,
    MC_ERR_ARG = 1,         /* invalid argument (host) or invalid field (device: NaN/Inf, tau <= 0) */
    MC_ERR_RANGE = 2,       /* |(v - c) / (2 tau1)| >= 2^27: error bound too small for the data range */
    MC_ERR_CAPACITY = 3,    /* more outliers than the caller's capacity; counts are still exact */
    MC_ERR_NOMEM = 4,       /* device allocation failed */
    MC_ERR_DEVICE = 5,      /* a HIP call failed */
    MC_ERR_FORMAT = 6,      /* malformed serialized model or stream */
    MC_ERR_UNSUPPORTED = 7  /* valid request outside what the library supports */
} mc_status;

typedef enum { MC_F32 = 0, MC_F64 = 1 } mc_dtype;
typedef enum { MC_EB_ABS = 0, MC_EB_REL = 1 } mc_eb_mode;   /* REL: tau = eb * (max x - min x) */
typedef enum { MC_FILL_NEAREST = 0, MC_FILL_MIDRANGE = 1 } mc_fill;

#define MC_RADIUS 32768      /* quantisation radius R: code = value + R, code 0 = outlier */
#define MC_BLOCK 4096        /* vertices per learned/plain decision block */

/* Rectilinear grid.  Node (i0,i1,i2) is at origin + i * spacing; its FP32
 * position is (float)origin + (float)i * (float)spacing.  dims >= 2 on every
 * used axis; 2-D grids have dims[2] = 1. */
typedef struct {
    int32_t dim;
    int64_t dims[3];
    double origin[3];
    double spacing[3];
} mc_grid;

typedef struct mc_plan_s* mc_plan;
typedef struct mc_model_s* mc_model;

/* Operator pair of a plan.
 * MC_OPS_LINEAR (default): f = barycentric interpolation in the lowest-id
 *   cell holding the node, g = multilinear interpolation on the vertex's
 *   grid cell; the residual is taken against the reconstructed grid.
 * MC_OPS_CLUSTER: the paper's own pair (Sec. IV-C, IV-D): g = the nearest
 *   grid node m_k (per axis rint((p - origin) / spacing), clamped), f = the
 *   mean of the vertices whose nearest node it is (FP64, summed in
 *   ascending vertex id; c for a node no vertex maps to).  Needs no
 *   connectivity (d_cells may be NULL and n_cells 0).  No learned model. */
typedef enum { MC_OPS_LINEAR = 0, MC_OPS_CLUSTER = 1 } mc_operators;

typedef struct {
    mc_fill fill;            /* nodes outside every cell: nearest vertex (default) or mid-range */
    int32_t bin_nodes;       /* point-location bin edge in grid nodes (0 = tuned default) */
    int32_t operators;       /* mc_operators (0 = MC_OPS_LINEAR) */
    int32_t coarsen;         /* 1: Grid_Coarsen (Alg. 2), MC_OPS_CLUSTER only (else MC_ERR_UNSUPPORTED):
                                a grid plane that no vertex's nearest node lies in is dropped, axis by axis
                                (an axis left with fewer than two planes keeps all of them); the plan then
                                works on the coarsened grid, whose dims mc_plan_get_grid returns and whose
                                planes mc_plan_kept_planes lists; 0: the grid as given */
} mc_plan_opts;

typedef struct {
    int64_t n_grid;          /* grid nodes */
    int64_t n_vertices;
    int64_t n_cells;
    int64_t n_unresolved;    /* grid nodes in no cell (filled per mc_plan_opts.fill); MC_OPS_CLUSTER: nodes no vertex maps to */
    int64_t n_near_degenerate;  /* cells whose weights were recomputed in FP64 */
    int64_t n_pairs;         /* (bin, cell) pairs of the point-location index */
    int64_t bin_nodes;
    int64_t device_bytes;    /* device memory held by the plan */
    int32_t invalid_cells;   /* cells with an out-of-range vertex id (plan creation fails) */
} mc_plan_info;

/* Error split.  MC_SPLIT_SUM: the grid receives tau1 = grid_share * tau and
 * the residuals tau2 = tau - tau1 (Sec. III: tau1 + tau2 <= tau); every
 * vertex ends within tau2.  MC_SPLIT_FULL: tau1 = grid_share * tau and
 * tau2 = tau.  The residuals are taken against the reconstructed grid and
 * checked per vertex, so a vertex's error is the residual's own
 * quantisation error: tau2 alone bounds it, and tau1 only sets the grid's
 * quantisation step (grid noise is absorbed by the residual). */
typedef enum { MC_SPLIT_SUM = 0, MC_SPLIT_FULL = 1 } mc_split;

/* Residual reference.  MC_RESIDUAL_CLOSED: x - g(x1'), the reconstructed
 * grid; every vertex within tau2.  MC_RESIDUAL_OPEN: x - g(x1), the grid
 * before its compression, as Alg. 3 writes it; every vertex within
 * tau1 + tau2 = tau (Sec. III; each vertex is checked, values that miss are
 * stored raw).  OPEN needs an MC_OPS_CLUSTER plan and MC_SPLIT_SUM. */
typedef enum { MC_RESIDUAL_CLOSED = 0, MC_RESIDUAL_OPEN = 1 } mc_residual;

/* Compression parameters (zero-initialise, then fill). */
typedef struct {
    double eb;               /* error bound, > 0 */
    int32_t eb_mode;         /* mc_eb_mode */
    double grid_share;       /* tau1 / tau: in (0, 1) for MC_SPLIT_SUM, (0, 16] for MC_SPLIT_FULL */
    mc_model model;          /* NULL: plain residual codes; else learned shift per block */
    int32_t split_mode;      /* mc_split (0 = MC_SPLIT_SUM) */
    int32_t residual;        /* mc_residual (0 = MC_RESIDUAL_CLOSED) */
} mc_params;

/* Device-side result header, written by mc_compress and read by
 * mc_decompress (it carries the quantisation steps). */
typedef struct {
    int32_t status;          /* mc_status of the device work */
    int32_t dtype;
    int64_t n_grid_outliers;
    int64_t n_vertex_outliers;
    int64_t n_learned_blocks;
    double tau, tau1, tau2, c, xmin, xmax;
    double kappa_unused;
} mc_result;

/* How vertex residual codes are formed.  MC_RESPRED_NONE: each vertex's
 * quantised residual q on its own (code q + R).  MC_RESPRED_DELTA: the
 * residuals serialised in vertex order through a 1-D Lorenzo predictor, as
 * the paper's underlying compressors treat the serialised residual array
 * (Sec. IV-B): code (q_i - q_{i-1}) + R with q_{-1} = 0; a vertex whose
 * difference exceeds R - 1 (or whose reconstruction misses tau2) is stored
 * raw and decoding restarts there from rint((raw - g) / (2 tau2)).
 * Either operator pair (g = multilinear or nearest node), closed-loop
 * residual, no learned model (else MC_ERR_UNSUPPORTED): the restart at a
 * raw value needs the decoder-side reference x1'.
 * Decoding needs one more pass over the codes (tile aggregates). */
typedef enum { MC_RESPRED_NONE = 0, MC_RESPRED_DELTA = 1 } mc_residual_predictor;

/* How grid codes are formed from the prequantised grid p (the grid
 * compressor C(x1) may be any error-controlled compressor, Sec. IV-D; the
 * SZ family's predictors, Sec. II, include Lorenzo and interpolation).
 * The bound tau1, p, x1' and the vertex codes do not depend on the choice.
 * MC_GRIDPRED_LORENZO: the Lorenzo predictor (zeros outside the grid).
 * MC_GRIDPRED_INTERP_LINEAR / _CUBIC: multilevel interpolation.  With L
 * the least integer such that 2^L >= n_d on every axis, strides
 * s = 2^(L-1) .. 1; the origin is predicted by 0; any other node is in
 * class (s, a): s = 2^t, t the fewest trailing zero bits among its
 * non-zero coordinates, a the highest axis whose coordinate is non-zero
 * with t trailing zeros.  Its prediction along a, from the nodes at -s,
 * +s (and -3s, +3s), all of earlier classes:
 *   +s outside the grid:          p[-s]
 *   CUBIC, -3s and +3s inside:    floor((-p[-3s] + 9 p[-s] + 9 p[+s] - p[+3s] + 8) / 16)
 *   otherwise:                    floor((p[-s] + p[+s]) / 2)
 * Decoding visits the origin, then the classes s = 2^(L-1) .. 1, and
 * a = 0 .. D-1 within a stride: one launch per fine class, the coarse
 * classes in one workgroup.
 * MC_GRIDPRED_TEMPORAL: the time axis (Sec. I: analyses read many
 * timesteps of one mesh).  Node j is predicted from a reference grid r that
 * compressor and decompressor both hold, normally the x1' of the previous
 * timestep (mc_codes.xhat_out of that call):
 *   P_j = rint(((double)r_j - c) / (2 tau1)) when below 2^27 in magnitude,
 *   else 0 (also for a non-finite r_j); error p_j - P_j.
 * mc_codes.grid_ref must then point to r (device, float[n_grid]), the
 * same array at compress and decompress.  Unknown values: MC_ERR_ARG. */
typedef enum {
    MC_GRIDPRED_LORENZO = 0,
    MC_GRIDPRED_INTERP_LINEAR = 1,
    MC_GRIDPRED_INTERP_CUBIC = 2,
    MC_GRIDPRED_TEMPORAL = 3
} mc_grid_predictor;

/* Compressed representation (caller-allocated device buffers).
 *   grid_codes  uint16[n_grid]      code d + R of the grid prediction error d, 0 = outlier
 *   g_out_idx   int32[g_out_cap]    grid outlier node ids, ascending
 *   g_out_delta int32[g_out_cap]    their prediction errors
 *   vert_codes  uint16[n_vertices]  residual code q + R (learned: q - rho_q + R), 0 = outlier
 *   v_out_idx   int32[v_out_cap]    vertex outlier ids, ascending
 *   v_out_val   T[v_out_cap]        their raw values (T = field dtype)
 *   block_flags uint32[ceil(ceil(n_v/4096)/32)]  bit b: block b learned (may be NULL for plain)
 *   result      mc_result (device)
 * Optional diagnostics, written when non-NULL:
 *   dbg_resampled float[n_grid] (f(x) on the grid), dbg_grid_p int32[n_grid]
 *   (prequantised grid), dbg_vertex_g float[n_vertices] (g(x1') at the
 *   vertices), rho_q int32[n_vertices] (learned shift, learned mode only). */
typedef struct {
    uint16_t* grid_codes;
    int32_t* g_out_idx;
    int32_t* g_out_delta;
    int64_t g_out_cap;
    uint16_t* vert_codes;
    int32_t* v_out_idx;
    void* v_out_val;
    int64_t v_out_cap;
    uint32_t* block_flags;
    mc_result* result;
    float* dbg_resampled;
    int32_t* dbg_grid_p;
    float* dbg_vertex_g;
    int32_t* rho_q;
    int32_t residual_predictor;  /* mc_residual_predictor of vert_codes; the same for compress and decompress */
    int32_t grid_predictor;      /* mc_grid_predictor of grid_codes; the same for compress and decompress */
    const float* grid_ref;       /* MC_GRIDPRED_TEMPORAL: reference grid [n_grid] (device); else ignored */
    float* xhat_out;             /* optional [n_grid] (device): x1' of this call, written by compress and
                                    decompress after every other use of grid_ref (so it may be grid_ref) */
} mc_codes;

const char* mc_status_string(mc_status s);
const char* mc_last_error(void);
int32_t mc_abi_version(void);

/* Grid spanning the bounding box of the vertices (Alg. 1 takes the grid
 * corners from the minimum and maximum vertex coordinates): origin = min,
 * spacing = (max - min) / (dims - 1).  (sync) */
mc_status mc_grid_from_dims(const float* d_coords, int32_t dim, int64_t n_vertices,
                            const int64_t dims[3], hipStream_t stream, mc_grid* out);
/* Grid with the given spacing h over the bounding box:
 * dims = ceil((max - min) / h) + 1.  (sync) */
mc_status mc_grid_from_spacing(const float* d_coords, int32_t dim, int64_t n_vertices,
                               const double spacing[3], hipStream_t stream, mc_grid* out);

/* Grid by the paper's initialisation (Alg. 1, Sec. IV-C): the spacing of
 * each axis is the k_percent-th percentile (nearest rank: the
 * ceil(k N / 100)-th smallest, at least the first) of the N extents
 * |p_a,d - p_b,d| (FP32) of every edge of every cell (3 per triangle, 6 per
 * tetrahedron; an edge counts once per cell holding it); while
 * (max_d - min_d) / spacing_d >= g_max, k rises by one point (at most to
 * 100, else MC_ERR_ARG).  The grid spans the vertex bounding box with that
 * spacing, dims = ceil((max - min) / spacing) + 1 (as
 * mc_grid_from_spacing).  k_used (may be NULL) receives the final k per
 * axis.  The percentile is an exact radix select on the GPU.  (sync) */
mc_status mc_grid_from_percentile(const float* d_coords, const int32_t* d_cells, int32_t dim,
                                  int64_t n_vertices, int64_t n_cells, double k_percent, int64_t g_max,
                                  hipStream_t stream, mc_grid* out, double k_used[3]);

/* Field-independent plan (the paper's reusable mesh-grid mapping, Sec.
 * IV-B/IV-C): a uniform bin index over the grid, the containing cell and
 * barycentric weights of every grid node, and the fill of nodes outside the
 * mesh.  The plan copies the coordinates; the caller may free the mesh once
 * this returns.  (sync) */
mc_status mc_plan_create(const float* d_coords, const int32_t* d_cells, int32_t dim,
                         int64_t n_vertices, int64_t n_cells, const mc_grid* grid,
                         const mc_plan_opts* opts, hipStream_t stream, mc_plan* out);
mc_status mc_plan_get_info(mc_plan plan, mc_plan_info* out);
/* Autotuning of the point-location bin edge (mc_plan_opts.bin_nodes) for a
 * mesh and grid: for each of the n_candidates (1..16) bin edges in
 * h_candidates (1..64 grid nodes), times the bin index build and the
 * location kernel on scratch buffers (HIP events) and writes the fastest
 * edge to *best_bin_nodes and each candidate's milliseconds to h_ms (may be
 * NULL).  The mapping a plan gets is the same for every bin edge.  (sync) */
mc_status mc_plan_tune_bins(const float* d_coords, const int32_t* d_cells, int32_t dim, int64_t n_vertices,
                            int64_t n_cells, const mc_grid* grid, const int32_t* h_candidates, int32_t n_candidates,
                            hipStream_t stream, int32_t* best_bin_nodes, double* h_ms);

/* Copies the mapping: d_vid int32[dim+1][n_grid] (-1 for mid-range-filled
 * nodes), d_w float[dim+1][n_grid], d_cell int32[n_grid] (-1 = unresolved);
 * any may be NULL (MC_OPS_LINEAR plans; MC_ERR_UNSUPPORTED otherwise). */
mc_status mc_plan_mapping(mc_plan plan, int32_t* d_vid, float* d_w, int32_t* d_cell,
                          hipStream_t stream);
mc_status mc_plan_get_grid(mc_plan plan, mc_grid* out);
/* Copies the nearest node of every vertex, d_m int32[n_vertices], on the
 * plan's (coarsened) grid (MC_OPS_CLUSTER plans; MC_ERR_UNSUPPORTED
 * otherwise). */
mc_status mc_plan_nodes(mc_plan plan, int32_t* d_m, hipStream_t stream);
/* Copies the vertex list of every node, the sets whose means are the
 * cluster resampling f (Sec. IV-D): node j's vertices, in ascending id
 * order, are d_vlist[d_noff[j] .. d_noff[j+1]); d_noff int64[n_grid + 1],
 * d_vlist int32[n_vertices], either may be NULL (MC_OPS_CLUSTER plans;
 * MC_ERR_UNSUPPORTED otherwise). */
mc_status mc_plan_node_lists(mc_plan plan, int64_t* d_noff, int32_t* d_vlist, hipStream_t stream);
/* Grid_Coarsen (Alg. 2) of a plan made with mc_plan_opts.coarsen = 1 (sync):
 * h_keep (host, int32[dims0 + dims1 + dims2] of the grid given at plan
 * creation, axis 0 first) receives each original plane's index on the
 * coarsened axis, or -1 where the plane was dropped.  MC_ERR_CAPACITY if
 * cap is smaller; MC_ERR_UNSUPPORTED for a plan without coarsening. */
mc_status mc_plan_kept_planes(mc_plan plan, int32_t* h_keep, int64_t cap);
mc_status mc_plan_destroy(mc_plan plan);

/* Compress one field (Alg. 3, residuals against the reconstructed grid). */
mc_status mc_compress(mc_plan plan, const void* d_field, mc_dtype dtype,
                      const mc_params* params, const mc_codes* codes, hipStream_t stream);
/* Decompress (Alg. 4) into d_field_out (dtype of the compressed field).
 * model must be the model the field was compressed with (NULL if plain). */
mc_status mc_decompress(mc_plan plan, const mc_codes* codes, mc_model model,
                        void* d_field_out, mc_dtype dtype, hipStream_t stream);

/* ---- autotuning -----------------------------------------------------------
 * Launch knobs of a plan.  Bits 0-6: bit k set = kernel k takes its tiles
 * in XCD-contiguous order (each of the 8 XCDs, with its own L2, gets one
 * contiguous run of tiles), clear = in launch order: 0 resample, 1 Lorenzo
 * codes, 2 residual codes (and the learned block costs), 3 vertex decode,
 * 4/5 the 3-D grid decode's tile sums and apply (grids with n0 at most
 * 1024); bit 6 has no effect.  Bits 7-8 pick the cache policy of data a
 * kernel streams once: set = non-temporal loads and stores, so the stream
 * does not evict lines that other threads read again; 7 the resample's
 * mapping, 8 the coordinates, field, codes and decoded values of the
 * residual codes and the vertex decode.  Bits 9-12 pick launch shapes:
 * bits 9-10 the vertex decode's vertices per thread (0: 4, 1: 2, 2: 8,
 * 3: 4), bits 11-12 the field range's partial blocks (0: 2048, 1: 1024,
 * 2: 512, 3: 2048).  Any other bit is rejected.
 * Codes and values never depend on the knobs.  Default: 0x1ec (on a
 * 16M-vertex tetrahedral mesh with a 256^3 grid: the fastest mask of a
 * sweep with XCD order for the two vertex kernels, which leaves their time
 * unchanged and fetches each grid line once per pass instead of 1.4x). */
typedef struct {
    uint32_t remap_mask;
    uint32_t reserved[3];
} mc_tuning;

mc_status mc_plan_get_tuning(mc_plan plan, mc_tuning* out);
mc_status mc_plan_set_tuning(mc_plan plan, const mc_tuning* tuning);
/* Coordinate descent over the knob bits from the default mask (two sweeps):
 * each candidate is timed as `reps` whole compress + decompress passes of
 * d_field (HIP events on the stream, after one untimed pass) and a bit is
 * flipped when that makes the passes faster by more than 0.5 %.  codes and d_out
 * (T[n_vertices]) receive the last pass's results.  The per-launch
 * profiler is paused while timing and left as it was.  Writes the choice
 * to *chosen if not NULL.  (sync) */
mc_status mc_plan_tune(mc_plan plan, const void* d_field, mc_dtype dtype, const mc_params* params,
                       const mc_codes* codes, void* d_out, int32_t reps, hipStream_t stream,
                       mc_tuning* chosen);

/* One-shot form: builds a plan for the mesh and a grid with the given
 * spacing, compresses, and releases the plan.  (sync) */
mc_status mc_compress_mesh(const float* d_coords, const int32_t* d_cells, int32_t dim,
                           int64_t n_vertices, int64_t n_cells, const void* d_field,
                           mc_dtype dtype, const double spacing[3], double eb,
                           int32_t eb_mode, double grid_share, const mc_codes* codes,
                           mc_grid* grid_out, hipStream_t stream);

/* ---- learned residual predictor ----------------------------------------
 * MLP in -> 64 -> 64 -> 64 -> 1 (ReLU).  Inputs per vertex: for the 4^dim
 * grid nodes around its grid cell (indices clamped), bf16((x1'[n] - g) *
 * kappa), then bf16(t_d - 0.5) per axis, zero-padded to 32 (2-D) or 96
 * (3-D).  Weights BF16, accumulation FP32, output in residual-code units.
 * Parameter vector (FP32, shared with the model file): W1[64][Kin]
 * (output-major), b1[64], W2[64][64], b2, W3[64][64], b3, W4[64], b4[1];
 * Kin = 4^dim + dim. */
typedef struct {
    int32_t steps;           /* Adam steps (default 2000) */
    int32_t batch;           /* minibatch (default 8192) */
    float lr;                /* default 1e-3 */
    uint64_t seed;           /* SplitMix64 seed for init and sampling */
    float* h_loss_out;       /* optional host float[steps]: loss per step */
    int32_t sample_steps;    /* steps whose samples one launch draws; 0: as many
                                as fit in 256 MB.  The trained model does not
                                depend on it. */
} mc_train_opts;

int64_t mc_model_param_count(int32_t dim);
/* Model from a host parameter vector and input scale kappa. */
mc_status mc_model_create(int32_t dim, const float* h_params, float kappa, mc_model* out);
/* Trains a model on the residuals of field_t0 (plain compression with
 * params), on the GPU.  (sync) */
mc_status mc_model_train(mc_plan plan, const void* d_field_t0, mc_dtype dtype,
                         const mc_params* params, const mc_train_opts* opts,
                         hipStream_t stream, mc_model* out);
mc_status mc_model_get_params(mc_model model, float* h_params, float* kappa);
mc_status mc_model_export(mc_model model, void* h_buf, size_t cap, size_t* written);
mc_status mc_model_import(const void* h_buf, size_t n, mc_model* out);
mc_status mc_model_destroy(mc_model model);
/* Forward pass on given inputs d_z float[batch][Kpad] (BF16-valued):
 * d_rho float[batch]. */
mc_status mc_model_forward(mc_model model, const float* d_z, int64_t batch, float* d_rho,
                           hipStream_t stream);
/* Mean-squared-error loss and gradient (d_grad float[param_count]) over a
 * batch, with the training kernels. */
mc_status mc_model_loss_grad(mc_model model, const float* d_z, const float* d_y,
                             int64_t batch, float* d_grad, float* d_loss,
                             hipStream_t stream);
/* Input features of vertices [v0, v0+count) for a compressed field: d_z
 * float[count][Kpad]; uses the plan's last reconstructed grid. */
mc_status mc_model_features(mc_model model, mc_plan plan, const mc_codes* codes, int64_t v0,
                            int64_t count, float* d_z, hipStream_t stream);

/* ---- batched compression ------------------------------------------------
 * Compresses many fields, on one or more plans, as one HIP graph.  The
 * first call with a given item list (compared byte for byte, so zero the
 * structs before filling them) captures the batch into a graph.  Fields on
 * the plain Lorenzo path (MC_OPS_LINEAR plan, no model, MC_RESPRED_NONE,
 * MC_GRIDPRED_LORENZO, no xhat_out or diagnostics) go through work-list
 * stage launches: one launch per stage (range, range fold, resample, grid
 * and vertex codes, outlier lists) over the tiles of all of them, each with
 * its own workspace held by the graph (about 4 bytes per grid node plus
 * 1 KB per 1,024 nodes and vertices).  The other fields run as one chain of
 * kernels per distinct plan, forked from and joined back to the graph's
 * origin; fields that share a plan run in list order on its chain, since
 * they share its workspace.  Later calls with the same list replay the graph
 * in one launch.  Each item follows mc_compress
 * exactly (same codes, outliers and result), including its error statuses,
 * which are written to that item's `codes.result` on the device.  Host-side
 * argument errors of any item fail the whole call before anything is
 * enqueued (MC_ERR_ARG, mc_last_error names the item).  Graph capture
 * records no memset nodes.  At most 16 graphs are cached (least recently
 * created dropped first); destroying a plan or model drops the graphs that
 * use it.  Async with respect to the host. */
typedef struct {
    mc_plan plan;
    const void* d_field;
    mc_dtype dtype;
    mc_params params;
    mc_codes codes;
} mc_batch_item;

mc_status mc_batch_compress(const mc_batch_item* items, int32_t n_items, hipStream_t stream);

/* The inverse (Alg. 4 for every item), captured and replayed the same way:
 * each item follows mc_decompress exactly, writing d_out (T[n_vertices] of
 * its plan, caller-owned).  `codes` are the buffers a compress filled.  The
 * grid decodes run on one chain per plan, each into the field's own decoded
 * grid held by the graph; the vertex decode of every field without a model
 * and with value-by-value residual codes is then one work-list launch. */
typedef struct {
    mc_plan plan;
    mc_codes codes;
    mc_model model;        /* the model the field was compressed with, or NULL */
    void* d_out;
    mc_dtype dtype;
} mc_batch_ditem;

mc_status mc_batch_decompress(const mc_batch_ditem* items, int32_t n_items, hipStream_t stream);
/* The cached graph of an item list (kind 0: mc_batch_item[n], 1:
 * mc_batch_ditem[n], compared byte for byte as in the calls): how many of
 * its fields run on the work-list stage launches and how many nodes the
 * graph has.  MC_ERR_ARG when no graph is cached for the list.  (host) */
mc_status mc_batch_graph_info(int32_t kind, const void* items, int32_t n_items, int32_t* n_batched,
                              int64_t* n_nodes);
/* Synchronises the device and frees every cached batch graph. */
mc_status mc_batch_release(void);

/* ---- 1-D serialisation baseline --------------------------------------------
 * The comparison the multi-component scheme is measured against (Sec. V-C,
 * the "default" compression: the underlying compressor applied to the
 * vertex values as a serialised 1-D array).  With the whole bound tau on
 * one component, c the mid-range and R = MC_RADIUS:
 *   p_i = rint((x_i - c) / (2 tau))      (FP64, |.| < 2^27 else MC_ERR_RANGE)
 *   d_i = p_i - p_{i-1}, p_{-1} = 0      (1-D Lorenzo)
 *   x'_i = (T)(c + p_i 2 tau)
 *   code_i = d_i + R if |d_i| <= R - 1 and |x_i - x'_i| <= tau, else 0 with
 *   x_i stored raw (vertex order).
 * Decoding rebuilds p_i as the running sum of the codes, restarting at each
 * raw value from rint((raw - c) / (2 tau)).  Every vertex satisfies
 * |x - x'| <= tau.
 * Only the vertex fields of mc_codes are used: vert_codes (uint16[n]),
 * v_out_idx / v_out_val / v_out_cap and result (tau1 = tau, tau2 = 0); the
 * grid fields, block_flags and diagnostics may be NULL.  A context holds the
 * device workspace for fields of up to n_max values; calls on one context
 * must be ordered on one stream. */
typedef struct mc_serial_s* mc_serial;

mc_status mc_serial_create(int64_t n_max, mc_serial* out);                  /* (sync) */
mc_status mc_serial_destroy(mc_serial ctx);
/* Compress d_field (T[n], 1 <= n <= n_max). */
mc_status mc_serial_compress(mc_serial ctx, const void* d_field, mc_dtype dtype, int64_t n, double eb,
                             int32_t eb_mode, const mc_codes* codes, hipStream_t stream);
/* Decompress into d_out (T[n]); n must be the compressed length. */
mc_status mc_serial_decompress(mc_serial ctx, const mc_codes* codes, int64_t n, void* d_out, mc_dtype dtype,
                               hipStream_t stream);

/* Compress without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): mc_serial_compress without a context.  Its scratch
 * (range partials, control block, outlier counters; about 1.2 MB) is one
 * fixed array in device memory per GPU, held from the first call on that
 * GPU until the process ends; n is limited to MC_SERIAL_NOALLOC_MAX
 * values (above it: MC_ERR_CAPACITY, nothing enqueued).  Codes, outliers
 * and result equal mc_serial_compress's for the same input.  Every call on
 * one GPU shares that array (each call re-initialises it on the stream
 * before use): calls that may overlap on one GPU -- different streams,
 * different host threads -- race and must be serialised by the caller.
 * Calls no hipMalloc, hipFree or allocating library routine. */
#define MC_SERIAL_NOALLOC_MAX (1LL << 28)
int64_t mc_serial_noalloc_max(void);
mc_status mc_serial_compress_noalloc(const void* d_field, mc_dtype dtype, int64_t n, double eb, int32_t eb_mode,
                                     const mc_codes* codes, hipStream_t stream);

/* ---- profiling -----------------------------------------------------------
 * When enabled, every kernel launch is bracketed by HIP events on the
 * launch stream; mc_profile_read returns per-kernel launch counts and
 * summed milliseconds (sync). */
mc_status mc_profile_enable(int32_t on);
/* Brackets only the launches of the named kernel (NULL or "": every kernel),
 * so that one kernel is timed without events around its neighbours. */
mc_status mc_profile_only(const char* name);
mc_status mc_profile_reset(void);
/* Writes up to cap entries: names (each a static string), counts, total ms. */
int32_t mc_profile_read(const char** names, int64_t* counts, double* total_ms, int32_t cap);

/* ---- CPU entropy stage (host, outside the hot path) ---------------------
 * Canonical Huffman (code lengths <= 24) over uint16 symbols plus the
 * outlier lists; gives the compressed size used for the compression ratio
 * S / (stream bytes) (the paper's ratio, Sec. IV-A, with original size S). */
/* Bytes of the Huffman-coded symbol stream including its code table. */
int64_t mc_huffman_size(const uint16_t* h_sym, int64_t n);
/* Encode into h_out (cap bytes); returns bytes written or -1. */
int64_t mc_huffman_encode(const uint16_t* h_sym, int64_t n, uint8_t* h_out, int64_t cap);
/* Decode n symbols; returns bytes consumed or -1 on a malformed stream. */
int64_t mc_huffman_decode(const uint8_t* h_in, int64_t n_in, uint16_t* h_sym, int64_t n);
/* Empirical Shannon entropy of the symbols, bits per symbol. */
double mc_entropy_bits(const uint16_t* h_sym, int64_t n);

/* ---- self-describing stream (host, outside the hot path) -----------------
 * The compressed bytes whose size gives the compression ratio (Sec. IV-A:
 * original size over compressed size; mesh, grid and mapping are reusable
 * state and not part of it): a header (dims, dtype, predictors, tau, tau1,
 * tau2, c), the canonical Huffman streams of the grid and vertex codes,
 * both outlier lists (LEB128 index gaps; grid errors zigzag-LEB128, vertex
 * values raw), the block flags in learned mode, optionally the model file,
 * and a checksum.  Host arrays throughout; sizes follow from the header
 * (n_grid = dims[0] * dims[1] * dims[2]). */
typedef struct {
    int32_t dim;                 /* 2 or 3; 1: a 1-D serialisation baseline stream (no grid sections,
                                    dims unused, tau1 = tau, tau2 = 0) */
    int32_t dtype;               /* mc_dtype of the field */
    int64_t dims[3];             /* grid nodes per axis; dims[2] = 1 in 2-D */
    int64_t n_vertices;
    int32_t grid_predictor;      /* mc_grid_predictor of the grid codes */
    int32_t residual_predictor;  /* mc_residual_predictor of the vertex codes */
    int32_t learned;             /* 1: vertex codes carry the learned shift; block flags present */
    int32_t reserved;
    double tau, tau1, tau2, c;   /* as in mc_result */
    int64_t n_grid_outliers, n_vertex_outliers;
} mc_stream_header;

typedef struct {
    uint16_t* grid_codes;        /* [n_grid] (unused for dim 1) */
    int32_t* g_out_idx;          /* [n_grid_outliers], ascending */
    int32_t* g_out_delta;        /* [n_grid_outliers] */
    uint16_t* vert_codes;        /* [n_vertices] */
    int32_t* v_out_idx;          /* [n_vertex_outliers], ascending */
    void* v_out_val;             /* [n_vertex_outliers] values of dtype */
    uint32_t* block_flags;       /* [ceil(ceil(n_vertices / 4096) / 32)], learned only */
} mc_stream_arrays;

/* Bytes of the stream (-1 on invalid input; mc_last_error says why).
 * model (model_bytes, 0 = none) is embedded when given, e.g. once per
 * timestep sequence.  section_bytes (may be NULL) receives 8 sizes: header,
 * grid codes, vertex codes, grid outliers, vertex outliers, block flags,
 * model, checksum. */
int64_t mc_stream_size(const mc_stream_header* hdr, const mc_stream_arrays* a, const void* model,
                       int64_t model_bytes, int64_t* section_bytes);
/* Writes the stream into h_out; returns its length, or -1 (invalid input or
 * cap too small: MC_ERR_CAPACITY in mc_last_error). */
int64_t mc_stream_write(const mc_stream_header* hdr, const mc_stream_arrays* a, const void* model,
                        int64_t model_bytes, uint8_t* h_out, int64_t cap, int64_t* section_bytes);
/* Header of a stream (checksum and ranges checked) and the size of its
 * embedded model (0 if none). */
mc_status mc_stream_read_header(const uint8_t* h_in, int64_t n, mc_stream_header* hdr, int64_t* model_bytes);
/* Arrays of a stream into caller buffers sized from its header; model
 * (model_cap bytes, may be NULL to skip) receives the embedded model.
 * MC_ERR_FORMAT for a malformed or truncated stream. */
mc_status mc_stream_read(const uint8_t* h_in, int64_t n, const mc_stream_arrays* a, void* model,
                         int64_t model_cap);

#ifdef __cplusplus
}
#endif
#endif
