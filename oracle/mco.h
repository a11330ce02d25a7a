/*
 * mco.h -- CPU oracle of the multi-component error-bounded compressor for
 * unstructured-mesh data (Gong et al., "A General Framework for
 * Error-controlled Unstructured Scientific Data Compression").
 *
 * TEST INFRASTRUCTURE.  This is the plain, slow, obviously-correct
 * definition the HIP library is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source with the HIP library and includes none of its headers.
 *
 * Every floating-point formula is evaluated exactly as parenthesised here:
 * each + - * / is one IEEE-754 round-to-nearest-even operation in the stated
 * type (the library is built with -ffp-contract=off, x86-64 SSE arithmetic,
 * no fused multiply-add).  rint() rounds half to even.
 *
 * Method (paper, Sec. III and Sec. IV-B..IV-E, Algorithms 3 and 4):
 *   x  = x2 + g(x1)                       decomposition (Sec. III)
 *   x1 = f(x) on grid nodes               resample (Sec. IV-D, "linear" f)
 *   mu1 = C(x1) with bound tau1           grid compressor (Sec. IV-B)
 *   x2 = x - g(x1')                       residual on vertices (Alg. 3)
 *   mu2 = C(x2) with bound tau2           residual compressor
 *   x' = g(x1') + x2'                     reconstruction (Alg. 4)
 * g has non-negative weights summing to one, so tau1 + tau2 <= tau keeps
 * every vertex within tau (Sec. III, the piece-wise linear special case).
 * The grid compressor is a Lorenzo predictor with linear quantisation (the
 * SZ-family predictor the paper names in Sec. II); f is barycentric
 * interpolation inside the lowest-numbered containing simplex; g is
 * multilinear interpolation on the grid cell that holds the vertex.
 */
#ifndef MCO_H
#define MCO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { MCO_OK = 0, MCO_ERR_ARG = 1, MCO_ERR_RANGE = 2, MCO_ERR_CAPACITY = 3 };
enum { MCO_F32 = 0, MCO_F64 = 1 };
#define MCO_RADIUS 32768          /* quantisation radius R; code 0 = outlier */
#define MCO_BLOCK 4096            /* vertices per learned/plain decision block */

/* Rectilinear grid: node (i0,i1,i2) sits at o + i*h (double description);
 * linear index i0 + n0*(i1 + n1*i2), x fastest.  2-D grids have n[2] = 1. */
typedef struct {
    int32_t dim;
    int64_t n[3];
    double o[3], h[3];
} mco_grid;

/* Error-bound split (Sec. III; Sec. IV-B splits tau into tau1 for the grid
 * and tau2 for the residuals). */
typedef struct {
    double tau, tau1, tau2, c, xmin, xmax, inv1, step1, inv2, step2;
} mco_bound;

/* ---- error bound ------------------------------------------------------ */
enum { MCO_SPLIT_SUM = 0, MCO_SPLIT_FULL = 1 };
int mco_bound_compute_mode(const void* x, int dtype, int64_t n, double eb, int relative,
                           double split, int mode, mco_bound* out);
int mco_bound_compute(const void* x, int dtype, int64_t n, double eb, int relative,
                      double split, mco_bound* out);

/* ---- geometry --------------------------------------------------------- */
void mco_bbox(const float* coords, int dim, int64_t nv, float lo[3], float hi[3]);
int mco_grid_from_dims(const float* coords, int dim, int64_t nv, const int64_t dims[3],
                       mco_grid* g);
void mco_grid_node(const mco_grid* g, int64_t j, float y[3]);
int mco_bary(int dim, const float* verts, const float* y, float* lam, int* near_degenerate);
int64_t mco_locate_brute(const float* coords, const int32_t* cells, int dim, int64_t nv,
                         int64_t nc, const mco_grid* g, int32_t* cell_of_node,
                         int32_t* vid, float* w);
int64_t mco_locate_raster(const float* coords, const int32_t* cells, int dim, int64_t nv,
                          int64_t nc, const mco_grid* g, int32_t* cell_of_node,
                          int32_t* vid, float* w);
void mco_fill_unresolved(const float* coords, int dim, int64_t nv, const mco_grid* g,
                         const int32_t* cell_of_node, int nearest, int32_t* vid, float* w);
void mco_fill_candidates(const float* coords, int dim, int64_t nv, const mco_grid* g, const int64_t* nodes,
                         int64_t nn, const int64_t* cand_ptr, const int32_t* cand, int32_t* vid, float* w);
void mco_locate_nodes(const float* coords, const int32_t* cells, int dim, int64_t nv, int64_t nc,
                      const mco_grid* g, const int64_t* nodes, int64_t nn, const int32_t* cand, int ncand,
                      int nearest, int32_t* cell_out, int32_t* vid_out, float* w_out);
void mco_resample(const int32_t* vid, const float* w, int dim, int64_t ng, const void* x,
                  int dtype, double c, float* v);
void mco_vertex_cell(const float* coords, int dim, int64_t nv, const mco_grid* g,
                     int64_t v, int32_t idx[3], float t[3]);
void mco_back_interp(const float* coords, int dim, int64_t nv, const mco_grid* g,
                     const float* xhat, float* gv);

/* ---- grid compressor --------------------------------------------------- */
int mco_grid_quantize(const float* v, const mco_grid* g, const mco_bound* b, int32_t* p,
                      uint16_t* codes, int32_t* out_idx, int32_t* out_delta, int64_t cap,
                      int64_t* n_out);
int mco_grid_quantize_f64(const double* v, const mco_grid* g, const mco_bound* b, int32_t* p,
                          uint16_t* codes, int32_t* out_idx, int32_t* out_delta, int64_t cap,
                          int64_t* n_out);
void mco_grid_recon(const int32_t* p, int64_t ng, const mco_bound* b, float* xhat);
int mco_grid_decode(const uint16_t* codes, const int32_t* out_idx, const int32_t* out_delta,
                    int64_t n_out, const mco_grid* g, int32_t* p);
void mco_lorenzo(const int32_t* p, const mco_grid* g, int64_t* delta);

/* Multilevel interpolation predictor on the prequantised grid
 * (mco_interp.c): cubic = 0 linear, 1 cubic; same code format. */
void mco_interp_delta(const int32_t* p, const mco_grid* g, int cubic, int64_t* delta);
int mco_interp_codes(const int32_t* p, const mco_grid* g, int cubic, uint16_t* codes, int32_t* out_idx,
                     int32_t* out_delta, int64_t cap, int64_t* n_out);
int mco_interp_decode(const uint16_t* codes, const int32_t* out_idx, const int32_t* out_delta, int64_t n_out,
                      const mco_grid* g, int cubic, int32_t* p);

/* Time-axis predictor from a reference grid (mco_temporal.c). */
int mco_temporal_codes(const int32_t* p, const float* ref, int64_t ng, const mco_bound* b, uint16_t* codes,
                       int32_t* out_idx, int32_t* out_delta, int64_t cap, int64_t* n_out);
int mco_temporal_decode(const uint16_t* codes, const int32_t* out_idx, const int32_t* out_delta, int64_t n_out,
                        const float* ref, int64_t ng, const mco_bound* b, int32_t* p);

/* ---- residual compressor ------------------------------------------------ */
int mco_residual_quantize(const void* x, int dtype, int64_t nv, const float* gv,
                          const mco_bound* b, uint16_t* codes, int32_t* out_idx,
                          void* out_val, int64_t cap, int64_t* n_out);
int mco_learned_codes(const void* x, int dtype, int64_t nv, const float* gv,
                      const mco_bound* b, const int32_t* rho_q, uint16_t* codes,
                      uint32_t* block_flags, int32_t* out_idx, void* out_val, int64_t cap,
                      int64_t* n_out);
void mco_vertex_decode(const uint16_t* codes, const int32_t* out_idx, const void* out_val,
                       int64_t n_out, const float* gv, const mco_bound* b, int dtype,
                       int64_t nv, const int32_t* rho_q, const uint32_t* block_flags,
                       void* xout);

/* ---- learned residual predictor ---------------------------------------- */
uint64_t mco_splitmix64(uint64_t seed, uint64_t counter);
float mco_bf16(float f);
int mco_mlp_kin(int dim);
int mco_mlp_kpad(int dim);
int64_t mco_mlp_nparams(int dim);
void mco_mlp_init(int dim, uint64_t seed, float* params);
void mco_mlp_features(const float* coords, int dim, int64_t nv, const mco_grid* g,
                      const float* xhat, const float* gv, float kappa, int64_t v0,
                      int64_t count, float* z);
double mco_mlp_feature_rms(const float* coords, int dim, int64_t nv, const mco_grid* g,
                           const float* xhat, const float* gv);
void mco_mlp_forward(int dim, const float* params, const float* z, int64_t batch,
                     float* h1, float* h2, float* h3, float* rho);
double mco_mlp_backward(int dim, const float* params, const float* z, int64_t batch,
                        const float* y, int round_bf16, float* grad);
double mco_mlp_loss_exact(int dim, const double* params, const double* z, int64_t batch,
                          const double* y, double* grad);
void mco_adam_step(int64_t n, float* params, float* m, float* v, const float* grad,
                   int64_t t, float lr, float beta1, float beta2, float eps);
int32_t mco_rho_quantize(float rho);
void mco_sample_indices(uint64_t seed, int64_t step, int64_t batch, int64_t n,
                        int64_t* idx);

/* The paper's own operator pair (mco_cluster.c): nearest-node g,
 * cluster-mean f, open- or closed-loop residual. */
void mco_nearest_nodes(const float* coords, int dim, int64_t nv, const mco_grid* g, int32_t* m);
void mco_cluster_mean(const void* x, int dtype, int64_t nv, const int32_t* m, int64_t ng, double c,
                      double* x1, int32_t* count);
int mco_residual_nearest(const void* x, int dtype, int64_t nv, const int32_t* m, const double* x1,
                         const float* xhat, const mco_bound* b, int open, uint16_t* codes, int32_t* out_idx,
                         void* out_val, int64_t cap, int64_t* n_out);
/* Grid_Coarsen (Alg. 2) for the nearest-node g (mco_cluster.c). */
void mco_grid_coarsen(const int32_t* m, int64_t nv, const mco_grid* g, int32_t* keep, int64_t new_n[3],
                      int32_t* m_out);
void mco_vertex_decode_nearest(const uint16_t* codes, const int32_t* out_idx, const void* out_val, int64_t n_out,
                               const int32_t* m, const float* xhat, const mco_bound* b, int dtype, int64_t nv,
                               void* xout);

/* Residuals with a 1-D Lorenzo predictor along the vertex order
 * (mco_resdelta.c). */
int mco_residual_delta(const void* x, int dtype, int64_t nv, const float* gv, const mco_bound* b, uint16_t* codes,
                       int32_t* out_idx, void* out_val, int64_t cap, int64_t* n_out);
void mco_vertex_decode_delta(const uint16_t* codes, const int32_t* out_idx, const void* out_val, int64_t n_out,
                             const float* gv, const mco_bound* b, int dtype, int64_t nv, void* xout);

/* Grid initialisation, Alg. 1 (mco_grid_init.c): per-axis spacing = the
 * k-th percentile (nearest rank) of the cells' edge extents along the axis,
 * k raised by one point while (max - min) / spacing >= g_max.  k_used may be
 * NULL. */
int mco_grid_init(const float* coords, const int32_t* cells, int dim, int64_t nv, int64_t nc, double k0,
                  int64_t g_max, mco_grid* g, double k_used[3]);

/* 1-D serialisation baseline (mco_serial.c). */
int mco_serial_compress(const void* x, int dtype, int64_t n, double eb, int relative, uint16_t* codes,
                        int32_t* out_idx, void* out_val, int64_t cap, int64_t* n_out, mco_bound* b);
void mco_serial_decompress(const uint16_t* codes, const int32_t* out_idx, const void* out_val, int64_t n_out,
                           int64_t n, const mco_bound* b, int dtype, void* out);

#ifdef __cplusplus
}
#endif
#endif
