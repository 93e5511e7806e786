/*
 * mdnp.h -- C ABI of the MI355X library for the neural-preconditioned flexible
 * GMRES solve of the coupled 3D-1D finite-element system.
 *
 * The problem (Section 2 of the paper): for a parameter mu, i.e. a 1D vessel
 * tree Lambda inside the unit cube, solve A^mu u = F^mu where
 *     A = [K00 0; 0 K11] + 2 pi eps [M00 M01; M10 M11]      (eq. "mainsys")
 * with K00 the 3D stiffness, K11 the 1D stiffness on the tree and M the
 * averaging/extension coupling.  The solver is right-preconditioned,
 * restarted flexible GMRES (Section 4), stopped on ||b - A x|| / ||b|| <= tol
 * (Section 5.1), with the block upper-triangular preconditioner of Section 2.2
 * (eq. "twosteps"): an exact 1D solve, then the 3D correction handed to the
 * neural operator P(v, d) (eq. "decoupled_3d_problem"), a U-net of Section 4.2
 * whose second input channel is the distance field d of the tree.
 *
 * Conventions for every call:
 *   - the return value is an mdnp_status; 0 means success; no C++ exception
 *     crosses this boundary; mdnp_last_error() gives a message;
 *   - "host" pointers are read (or written) during the call only and stay
 *     owned by the caller; "device" pointers are borrowed, must be valid
 *     device memory on the context's GPU, and are used in stream order on
 *     the given HIP stream (NULL = the context's stream);
 *   - one context per thread; calls on one context are not thread-safe;
 *   - non-convergence is not an error (see mdnp_inst_stats.converged).
 *
 * Vector layout of a system of n_inst instances: instances are concatenated;
 * instance i occupies [offset_i, offset_i + n3d + n1d_i), its 3D unknowns first
 * (grid node i + n j + n^2 k, n = n_cells + 1, x fastest), then its 1D
 * unknowns (tree vertices, then the interior nodes of segment s numbered
 * V + s (E - 1) + t from the parent end).
 */
#ifndef MDNP_H
#define MDNP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mdnp_ctx mdnp_ctx;
typedef struct mdnp_sys mdnp_sys;

typedef enum {
  MDNP_OK = 0,
  MDNP_E_ARG = -1,        /* invalid argument or size                       */
  MDNP_E_HIP = -2,        /* a HIP runtime call failed                      */
  MDNP_E_OOM = -3,        /* device allocation failed                       */
  MDNP_E_GEOM = -4,       /* invalid geometry (vertex outside, R <= 0, ...) */
  MDNP_E_NONFINITE = -5,  /* NaN/Inf in b, x0 or the weights                */
  MDNP_E_STATE = -6       /* call out of order (e.g. no preconditioner set) */
} mdnp_status;

typedef enum {
  MDNP_PREC_NONE = 0,         /* z = v                                                    */
  MDNP_PREC_JACOBI = 1,       /* z = diag(A)^-1 v  (Jacobi-preconditioned GMRES)           */
  MDNP_PREC_NEURAL = 2,       /* block preconditioner of eq. "twosteps", 3D block by the U-net */
  MDNP_PREC_BLOCK_JACOBI = 3  /* same block preconditioner with diag(A00)^-1 for the 3D block
                                 (the method without the network)                          */
} mdnp_prec_kind;

typedef enum { MDNP_F64 = 0, MDNP_F32 = 1, MDNP_BF16 = 2, MDNP_FP8E4M3 = 3, MDNP_FP8E4M3_ACT = 4 } mdnp_dtype;

/* Condition on the faces of the unit cube for the 3D unknowns. */
typedef enum {
  MDNP_BC_DIRICHLET = 0,  /* u = 0: boundary rows and columns eliminated symmetrically, unit rows kept */
  MDNP_BC_NEUMANN = 1     /* natural (homogeneous Neumann) condition, the setup of Section 5: all nodes free */
} mdnp_boundary;

/* Which linear system an instance stands for. */
typedef enum {
  MDNP_PROBLEM_COUPLED = 0,  /* the coupled 3D-1D system A u = F of eq. "mainsys"                      */
  MDNP_PROBLEM_BLOCK3D = 1   /* the 3D block alone, C u0 = b with C = K00 + 2 pi eps M00 (eq. "matrixC")
                                and b = -A01 A11^-1 f1 (eq. "setB"), the problem of Section 5; stored in
                                the coupled layout as [C 0; 0 I] [u0; u1] = [b; 0], so the 1D parts of
                                all vectors stay zero and every solver call solves C u0 = b */
} mdnp_problem;

/* One parameter instance mu (Section 2.1).  All arrays are host memory, copied
 * by mdnp_upload.  The segments must form a tree rooted at vertex 0 with
 * seg_vertices[2s] the parent end and seg_vertices[2s+1] the child end of
 * segment s; every vertex lies strictly inside the unit cube. */
typedef struct {
  int32_t n_cells;                 /* 3D cells per side; n = n_cells + 1 grid nodes per side   */
  double k_omega, sigma_omega;     /* 3D diffusion and reaction coefficients (eq. "aomega")    */
  int32_t n_vertices;
  const double* vertex_xyz;        /* [n_vertices * 3]                                         */
  int32_t n_segments;
  const int32_t* seg_vertices;     /* [n_segments * 2] (parent, child)                         */
  const double* seg_radius;        /* [n_segments] vessel radius R (eps of the paper)           */
  const double* seg_beta;          /* [n_segments] wall permeability; coupling c = 2 pi R beta  */
  int32_t elems_per_segment;       /* P1 elements per segment                                   */
  double k_lambda;                 /* 1D diffusion; the 1D operator carries the area pi R^2     */
  double f_lambda;                 /* line source on the tree; F = [0; int f phi]               */
  int32_t n_circle;                /* points of the cross-section average T_Lambda (>= 3)       */
  int32_t boundary;                /* mdnp_boundary; every instance of a system the same        */
  int32_t problem;                 /* mdnp_problem                                              */
} mdnp_instance_desc;

typedef struct {
  int32_t restart;            /* m, Arnoldi steps per cycle                                  */
  int32_t max_iters;          /* cap on Arnoldi steps per instance (all cycles)              */
  int32_t fallback_restart;   /* restart used once every active instance is on the fallback  */
  int32_t fallback_max_iters; /* extra steps allowed on the Jacobi fallback (0 = none)       */
  double tol;                 /* stop when ||b - A x|| <= tol ||b||                          */
  int32_t record_history;     /* keep rho_j / ||b|| per step for mdnp_history               */
  int32_t use_graph;          /* capture a restart cycle as HIP graphs of 5 Arnoldi steps and
                                 replay them (the next one only while an instance is active) */
} mdnp_solve_opts;

typedef struct {
  int32_t iters;            /* Arnoldi steps (= preconditioner applications) before fallback */
  int32_t fallback_iters;   /* Arnoldi steps taken on the Jacobi fallback                  */
  int32_t converged;        /* 1 when the true relative residual met tol                   */
  int32_t used_fallback;    /* 1 when the stall detector switched this instance to Jacobi  */
  double final_rel_res;     /* true ||b - A x|| / ||b|| recomputed in FP64 at the end      */
} mdnp_inst_stats;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `hip_device`; `hip_stream` (may be NULL) is the
 * default stream of all calls.  The caller keeps ownership of the stream. */
mdnp_status mdnp_create(mdnp_ctx** out, int hip_device, void* hip_stream);
mdnp_status mdnp_destroy(mdnp_ctx* ctx);
/* Message of the last failed call on this context (never NULL). */
const char* mdnp_last_error(const mdnp_ctx* ctx);

/* ---------------------------------------------------------------- systems */

/* Assemble A, F, the distance field d and the 1D factorisation for n_inst
 * instances (Section 2.1, eq. "mainsys"; distance channel of Section 2.1) and
 * copy them to the device.  All instances must share n_cells.  vec_dtype is
 * the storage type of the Krylov vectors and of the inner SpMV values:
 * MDNP_F64 (all FP64) or MDNP_F32 (FP32 vectors, FP64 orthogonalisation,
 * least squares, solution and true residual).  Errors: MDNP_E_ARG, MDNP_E_GEOM,
 * MDNP_E_OOM, MDNP_E_HIP.  *out is owned by the context; free with
 * mdnp_sys_free. */
mdnp_status mdnp_upload(mdnp_ctx* ctx, const mdnp_instance_desc* descs, int32_t n_inst,
                        mdnp_dtype vec_dtype, mdnp_sys** out);
mdnp_status mdnp_sys_free(mdnp_ctx* ctx, mdnp_sys* sys);

/* Sizes of instance `inst`: 3D and 1D unknowns, nonzeros of its CSR block and
 * its offset in the concatenated vectors. */
mdnp_status mdnp_sys_sizes(const mdnp_sys* sys, int32_t inst, int32_t* n3d, int32_t* n1d,
                           int64_t* nnz, int64_t* offset);

/* Sizes of the split operator of instance `inst` on the device, A = S + M
 * (Section 2.1: S the trilinear stiffness/mass stencil of the free 3D nodes,
 * identical at every interior node; M the coupling terms of eq. "mainsys"
 * and the 1D rows): entries stored for M and rows of M that hold any entry
 * (3D rows touched by the coupling plus every 1D row). */
mdnp_status mdnp_sys_split_sizes(const mdnp_sys* sys, int32_t inst, int64_t* m_nnz, int64_t* m_rows);

/* Sizes of the coupling of instance `inst` in the factored form the stencil-
 * sweep path applies, M = B^T W B + R (eq. "mainsys": each Gauss point q of the
 * 1D mesh contributes W_q (Pi_q u0 - Phi_q u1)(Pi_q v0 - Phi_q v1), Section
 * 2.1): Gauss points (rows of B), stored entries of W B, and stored entries of
 * the row-wise B^T | R the second pass reads (R: the 1D stiffness rows, or
 * unit 1D rows in the 3D-block layout, and the natural-boundary stencil
 * entries). */
mdnp_status mdnp_sys_coupling_sizes(const mdnp_sys* sys, int32_t inst, int64_t* n_gauss, int64_t* b_nnz,
                                    int64_t* s_nnz);

/* Host copy of the assembled matrix of one instance in CSR with local indices
 * (row_ptr [n+1], col [nnz], val [nnz], n = n3d + n1d): columns ascending,
 * duplicates merged, zero values kept where the pattern has them, Dirichlet
 * rows equal to the unit row.  Any output pointer may be NULL. */
mdnp_status mdnp_export_csr(const mdnp_sys* sys, int32_t inst, int32_t* row_ptr, int32_t* col,
                            double* val);

/* Host copy of the right-hand side F [n], the distance field d [n3d] and the
 * network normalisation alpha = RMS of diag(A00) over the free 3D nodes
 * (Section 5.1).  Any output pointer may be NULL. */
mdnp_status mdnp_export_rhs(const mdnp_sys* sys, int32_t inst, double* F, double* dist,
                            double* alpha);

/* ---------------------------------------------------------------- preconditioner */

/* Select the right preconditioner of the solve.  For MDNP_PREC_NEURAL, `weights`
 * (host, FP32, n_weights = 353713) holds the U-net parameters layer by layer,
 * each as [Cout][kz][ky][kx][Cin] then the bias, layers in the order
 * L0a L0b L1a L1b L2a L2b U1 D1 U0 D0 H; cnn_dtype is the arithmetic of the
 * network (MDNP_F32 or MDNP_BF16; FP32 accumulation).  MDNP_FP8E4M3 rounds
 * every layer's weights (not the biases) to the OCP 8-bit format E4M3 times
 * one power-of-two scale per output channel (the smallest 2^k with
 * max|w| / 2^k <= 448; round to nearest, ties to even) and runs the network
 * with them on the BF16 kernels, where those values are exact: E4M3 weights,
 * BF16 activations, FP32 accumulation.  MDNP_FP8E4M3_ACT rounds the weights
 * the same way and also stores every tensor a 3x3x3 layer reads (the input
 * and each 3x3x3 layer's output) as E4M3 codes of value / s, one power-of-two
 * scale s per tensor, on the FP8 matrix cores (E4M3 x E4M3 products, FP32
 * accumulation; the 1x1 head in FP32 on the E4M3 grid of D0's output); its
 * scales must be set (mdnp_fp8_calibrate, mdnp_set_fp8_scales) before a solve
 * or an application, else those return MDNP_E_STATE.  alpha <= 0 keeps each
 * instance's own alpha.  Requires n_cells divisible by 4.  Errors: MDNP_E_ARG,
 * MDNP_E_NONFINITE. */
mdnp_status mdnp_set_preconditioner(mdnp_ctx* ctx, mdnp_sys* sys, mdnp_prec_kind kind,
                                    const float* weights, int64_t n_weights, double alpha,
                                    mdnp_dtype cnn_dtype);

/* Activation scales of the MDNP_FP8E4M3_ACT network (an 8-bit variant of the
 * network of Section 4.2; the paper runs it in full precision): scales[11]
 * (host) for X, L0a, L0b, L1a, L1b, L2a, L2b, U1, D1, U0, D0, each a positive
 * power of two; the stacked pairs (L1b, U1) and (L0b, U0) need equal scales.
 * Captured cycle graphs are rebuilt.  Errors: MDNP_E_ARG (count != 11, a scale
 * not a power of two, a pair unequal), MDNP_E_STATE (no MDNP_FP8E4M3_ACT
 * network set). */
mdnp_status mdnp_set_fp8_scales(mdnp_ctx* ctx, mdnp_sys* sys, const float* scales, int32_t count);
/* The scales in use (0 where not set), scales[11] host. */
mdnp_status mdnp_get_fp8_scales(mdnp_ctx* ctx, const mdnp_sys* sys, float* scales, int32_t count);
/* Calibrate the scales on a sample: apply the preconditioner to the device
 * vector d_v (the system's vector type and length, e.g. a right-hand side)
 * with the network in FP32, take the largest magnitude of the network input
 * and of every 3x3x3 layer output over all instances (a stacked pair: over
 * both), and set each scale to the smallest power of two s with
 * 2 amax / s <= 448.  Synchronises the stream.  Errors: MDNP_E_ARG,
 * MDNP_E_STATE (as mdnp_set_fp8_scales), MDNP_E_NONFINITE (a non-finite
 * activation), MDNP_E_OOM. */
mdnp_status mdnp_fp8_calibrate(mdnp_ctx* ctx, mdnp_sys* sys, const void* d_v, void* hip_stream);

/* Jacobi pre- and post-smoothing of the network's 3D solve (Section 5, "Effect
 * of pre- and post-smoothing"): with sweeps > 0 the MDNP_PREC_NEURAL
 * preconditioner computes its 3D part as
 *   z0 = `sweeps` damped Jacobi steps z <- z + omega D^-1 (b0 - A00 z) from 0,
 *   z0 += N(b0 - A00 z0)   (the network with its own normalisation),
 *   z0 = `sweeps` more steps from z0,
 * D = diag(A00).  sweeps = 0 switches it off (the default).  Takes effect on
 * the next solve or preconditioner application; allocates three vectors of
 * the system's length and type, freed with the system or by sweeps = 0.
 * Errors: MDNP_E_ARG (sweeps outside [0, 16], omega outside (0, 2)),
 * MDNP_E_STATE (inner FGMRES steps are on, or the system has the natural
 * boundary condition). */
mdnp_status mdnp_set_smoothing(mdnp_ctx* ctx, mdnp_sys* sys, int32_t sweeps, double omega);

/* Inner Krylov 3D solve (Section 6): with steps > 0 the MDNP_PREC_NEURAL
 * preconditioner computes its 3D part z0 by `steps` FGMRES steps on
 * A00 z0 = b0 from z0 = 0, right-preconditioned by the network (Arnoldi by
 * modified Gram-Schmidt in FP64 dot products, stopped early on breakdown), in
 * place of one network application.  steps = 0 switches it off (the
 * default).  Allocates 2 steps + 1 vectors of the system's length and type,
 * freed with the system or by steps = 0.  Errors: MDNP_E_ARG (steps outside
 * [0, 8]), MDNP_E_STATE (smoothing is on, or the system has the natural
 * boundary condition). */
mdnp_status mdnp_set_inner_steps(mdnp_ctx* ctx, mdnp_sys* sys, int32_t steps);

/* Autotuner of the launch shapes, timed on this system's own batch and grid
 * with HIP events: the wave count that the stencil sweep of the SpMV splits
 * its z range for (from {1024 .. 6144}; best of three batches of 20 SpMVs),
 * and, with a BF16 (or FP8-weight) neural preconditioner set, the shape of
 * every convolution launch: the workgroup count of the z split of the sweep
 * layers (L0a, L0b, L1b, L2b, D1, D0; from {256 .. 2048}) and the 16-voxel
 * M blocks per wave of the stride-2 and transposed layers (L1a {2, 4, 8}, L2a
 * {1, 2, 4}, U1 {1, 2}, U0 {1, 2, 4}) and the output rows of the sweep
 * layers L1b {2, 3, 4, 6}, D1 {2, 3} (per workgroup), L0b {3, 4, 5, 6} (per
 * wave pair) and D0 (fused with the head; its three-plane z sweep with 4, 6
 * or 8 rows per workgroup, codes {12, 13, 14}), the workgroup count of U1 and U0
 * ({256 .. 4096}; each workgroup stages its weights in LDS and loops over
 * voxel blocks) and the 16-column x blocks per workgroup of L0a, L0b, D0
 * {1, 2, 4} and L1b, D1 {1, 2} (rows wider than that split over workgroups);
 * two rounds of coordinate descent, best of 5 whole network applications.
 * The choices only move output planes between waves and workgroups: results
 * are unchanged.  They are kept with the system; `chosen` (nullable, [23])
 * receives them: [0 .. 10] the z split or M blocks of the convolution layers
 * L0a = 0 .. H = 10 (0 = the built-in default, always for H), [11] the SpMV
 * sweep target (0 = default; also 0 where the grid has more than 65 nodes per
 * side and no sweep is used), [12 .. 15] the output rows of L1b, D1, L0b,
 * D0, [16], [17] the workgroups of U1, U0, [18 .. 22] the x blocks per
 * workgroup of L0a, L0b, L1b, D1, D0 (0 = as many as fit).  The library
 * allocates two vectors of the system's size for the timing and frees them
 * before returning.  Errors: MDNP_E_OOM if those buffers cannot be allocated
 * (the defaults are kept). */
mdnp_status mdnp_autotune(mdnp_ctx* ctx, mdnp_sys* sys, int32_t* chosen);

/* Sets the launch shapes directly, in the layout mdnp_autotune reports
 * (`chosen` [23], host; 0 = the built-in default): to restore a tuning
 * without timing it again, or to pick one shape.  Any code is safe (codes
 * outside the candidate sets select the default shape); every choice gives
 * the same results.  Errors: MDNP_E_ARG for a null pointer or a negative
 * code. */
mdnp_status mdnp_set_tuning(mdnp_ctx* ctx, mdnp_sys* sys, const int32_t* chosen);

/* Time the network as the solver applies it (Section 4.2 U-net inside the
 * 3D block of eq. "twosteps"), stage by stage, on this system's batch and
 * grid with the launch shapes currently chosen: after one application to a
 * fixed vector, each stage is launched `reps` times back to back on its own
 * inputs between two HIP events on the context's stream.
 * ms (host, [10]) receives the average duration in milliseconds of L0a, L0b,
 * L1a, L1b, L2a, L2b, U1, D1, U0 and D0 (which includes the 1x1 head and the
 * unscaling).  Allocates two vectors of the system's size for the duration of
 * the call.  Errors: MDNP_E_ARG, MDNP_E_STATE (no neural preconditioner),
 * MDNP_E_OOM. */
mdnp_status mdnp_cnn_layer_times(mdnp_ctx* ctx, mdnp_sys* sys, int32_t reps, float* ms);

/* ---------------------------------------------------------------- solve */

/* Restarted right-preconditioned FGMRES(m) on every instance at once (Section
 * 4; stopping rule of Section 5.1 with x0 as given): b and x are host arrays of
 * the concatenated length, x holds x0 on entry and the solution on return;
 * stats [n_inst] may be NULL.  An instance whose true relative residual falls
 * by less than 10% over a cycle, becomes non-finite, or reaches max_iters
 * unconverged is switched to Jacobi-preconditioned GMRES from its current x
 * for up to fallback_max_iters more steps.  Errors: MDNP_E_ARG,
 * MDNP_E_NONFINITE (b or x0), MDNP_E_STATE (no preconditioner set). */
mdnp_status mdnp_solve(mdnp_ctx* ctx, mdnp_sys* sys, const double* b, double* x,
                       const mdnp_solve_opts* opts, mdnp_inst_stats* stats);

/* Same with device buffers d_b, d_x (FP64, concatenated) on `hip_stream`. */
mdnp_status mdnp_solve_device(mdnp_ctx* ctx, mdnp_sys* sys, const double* d_b, double* d_x,
                              const mdnp_solve_opts* opts, mdnp_inst_stats* stats,
                              void* hip_stream);

/* Residual history of the last solve of instance `inst`: rho_j / ||b|| after
 * every Arnoldi step, and the true relative residual at the start of every
 * cycle stored negated.  Copies at most cap values to out (host); *n_out
 * receives the number available. */
mdnp_status mdnp_history(const mdnp_sys* sys, int32_t inst, double* out, int32_t cap,
                         int32_t* n_out);

/* Copy Arnoldi vector v_k (0 <= k <= restart) of the last cycle of the last
 * solve into d_out (device, vec_dtype, concatenated length): the
 * solver-generated residual samples used to train the network (Section 4.1,
 * Krylov augmentation).  Errors: MDNP_E_STATE before any solve, MDNP_E_ARG
 * for k outside [0, restart of that last cycle]. */
mdnp_status mdnp_export_basis(mdnp_ctx* ctx, const mdnp_sys* sys, int32_t k, void* d_out, void* hip_stream);

/* ---------------------------------------------------------------- path steps (device) */

/* y = A x (block 0) or y = A00 x on the 3D unknowns only (block 1, vectors of
 * length n_inst * n3d), for every instance.  dtype MDNP_F64 or MDNP_F32 selects
 * the value array and the vector type.  Block 0 applies the coupling through a
 * per-system intermediate (one value per Gauss point), as the solver does:
 * calls on one system, this one included, must not overlap in time (issue
 * them on one stream). */
mdnp_status mdnp_spmv(mdnp_ctx* ctx, mdnp_sys* sys, int32_t block, const void* d_x, void* d_y,
                      mdnp_dtype dtype, void* hip_stream);

/* The same y = A x (block 0) launched `reps` times back to back on the stream,
 * for timing the kernels without per-call host overhead between launches.
 * Errors: MDNP_E_ARG (reps < 1, null vectors, dtype not F32/F64). */
mdnp_status mdnp_spmv_repeat(mdnp_ctx* ctx, mdnp_sys* sys, const void* d_x, void* d_y, mdnp_dtype dtype,
                             int32_t reps, void* hip_stream);

/* z1 = A11^-1 v1 for every instance: the exact 1D solve of eq. "twosteps".
 * The tree matrix is factored without fill in chain-compressed form (each
 * segment's interior nodes as a tridiagonal block, then the Schur complement
 * on the tree vertices) when every segment has at most 32 interior nodes,
 * else as a leaves-first LDL^T of the whole tree.  d_v and d_z
 * are full concatenated vectors of the system's vec_dtype; only the 1D parts
 * are read and written. */
mdnp_status mdnp_tree_solve(mdnp_ctx* ctx, mdnp_sys* sys, const void* d_v, void* d_z,
                            void* hip_stream);

/* z = Q(v): one application of the selected preconditioner to one vector per
 * instance (vec_dtype, concatenated).  For the block kinds: the 1D solve, the
 * extension b0 = v0 - A01 z1 (eq. "decoupled_3d_problem"), then the 3D block
 * operator. */
mdnp_status mdnp_precond_apply(mdnp_ctx* ctx, mdnp_sys* sys, const void* d_v, void* d_z,
                               void* hip_stream);

/* U-net forward on a batch: d_x is [batch][n][n][n][2] FP32 (channel 0 the
 * normalised residual, channel 1 the distance), d_y is [batch][n][n][n] FP32.
 * d_w is the flat FP32 weight vector (device).  When d_saved is non-NULL the
 * layer activations needed by mdnp_cnn_backward are written there (size from
 * mdnp_cnn_saved_bytes).  dtype MDNP_F32 or MDNP_BF16. */
mdnp_status mdnp_cnn_forward(mdnp_ctx* ctx, const float* d_w, const float* d_x, float* d_y,
                             void* d_saved, int32_t batch, int32_t n, mdnp_dtype dtype,
                             void* hip_stream);
int64_t mdnp_cnn_saved_bytes(int32_t batch, int32_t n, mdnp_dtype dtype);

/* Adjoint of mdnp_cnn_forward: given dy [batch][n^3] FP32, accumulate nothing,
 * write the weight gradient d_dw [353713] (FP32, overwritten) and, when d_dx
 * is non-NULL, the input gradient [batch][n^3][2]. */
mdnp_status mdnp_cnn_backward(mdnp_ctx* ctx, const float* d_w, const void* d_saved,
                              const float* d_dy, float* d_dx, float* d_dw, int32_t batch,
                              int32_t n, mdnp_dtype dtype, void* hip_stream);

/* Training objective of Section 5.1 for a batch of unit samples: slot k uses
 * instance d_inst[k] of the system; r [n_slots][n3d] and the network output
 * u [n_slots][n3d] (FP32).  Writes loss[k] = || r_k - alpha_k^-1 C_k mask(u_k) ||^2
 * (C = A00, mask zeroes the Dirichlet entries) and its gradient du [n_slots][n3d]. */
mdnp_status mdnp_loss_grad(mdnp_ctx* ctx, mdnp_sys* sys, const int32_t* d_inst, int32_t n_slots,
                           const float* d_r, const float* d_u, float* d_du, double* d_loss,
                           void* hip_stream);

/* The same loss and gradient as mdnp_loss_grad without any device allocation,
 * for callers that cannot allocate: code under HIP graph capture, training
 * loops that must not call hipMalloc.  Its scratch (the masked outputs, C e
 * and the partial sums: n_slots * n3d * 8 + n_slots * 512 bytes) lives in a
 * fixed workspace of 32 MiB that the library holds on every GPU it runs on
 * until the process ends; larger requests fail with MDNP_E_ARG and change
 * nothing.  Results are bit-identical to mdnp_loss_grad's.  All calls on one
 * GPU share that workspace: calls that overlap in time on one GPU (other
 * streams, other contexts, other threads) race and must be serialised by the
 * caller.  No part of the workspace needs clearing between calls.  Errors:
 * MDNP_E_ARG, MDNP_E_STATE (workspace address not resolved), MDNP_E_HIP. */
mdnp_status mdnp_loss_grad_noalloc(mdnp_ctx* ctx, mdnp_sys* sys, const int32_t* d_inst, int32_t n_slots,
                                   const float* d_r, const float* d_u, float* d_du, double* d_loss,
                                   void* hip_stream);

/* Network input for training slots: X[k] = [r_k, d_{inst[k]}] as
 * [n_slots][n][n][n][2] FP32. */
mdnp_status mdnp_pack_input(mdnp_ctx* ctx, mdnp_sys* sys, const int32_t* d_inst, int32_t n_slots,
                            const float* d_r, float* d_x, void* hip_stream);

/* Adam (Kingma and Ba) on FP32 master weights, step counted from 1. */
mdnp_status mdnp_adam_step(mdnp_ctx* ctx, float* d_w, const float* d_g, float* d_m, float* d_v,
                           int64_t n, float lr, float beta1, float beta2, float eps, int32_t step,
                           void* hip_stream);

/* ---------------------------------------------------------------- host-only assembly */

/* Assemble one instance on the host without touching any GPU (the same code
 * mdnp_upload runs), for inspection and CPU-side checks.  Errors: MDNP_E_ARG,
 * MDNP_E_GEOM.  Free with mdnp_host_free. */
typedef struct mdnp_host_sys mdnp_host_sys;
mdnp_status mdnp_host_assemble(const mdnp_instance_desc* desc, mdnp_host_sys** out, char* err,
                               int32_t err_len);
mdnp_status mdnp_host_sizes(const mdnp_host_sys* hs, int32_t* n3d, int32_t* n1d, int64_t* nnz,
                            int32_t* n_levels);
/* CSR (local indices) as in mdnp_export_csr, F [n], dist [n3d], alpha; any may be NULL. */
mdnp_status mdnp_host_export(const mdnp_host_sys* hs, int32_t* row_ptr, int32_t* col, double* val,
                             double* F, float* dist, double* alpha);
/* The factored coupling of a host assembly, M = B^T W B + R (eq. "mainsys",
 * Section 2.1), local indices.  B: one row per Gauss point (b_ptr [n_gauss+1],
 * b_col / b_val [b_nnz]): the cross-section average Pi_q on the free 3D nodes,
 * columns ascending, then from b_split[q] the entries -Phi_q of the element's
 * two 1D nodes (none in the 3D-block layout); w [n_gauss] the weights
 * W_q = 2 pi R beta |e| / 2.  R: CSR over all n3d + n1d rows (r_ptr [n+1],
 * r_col / r_val [r_nnz]).  Sizes from mdnp_host_coupling_sizes; any pointer
 * may be NULL. */
mdnp_status mdnp_host_coupling_sizes(const mdnp_host_sys* hs, int32_t* n_gauss, int64_t* b_nnz, int64_t* r_nnz);
mdnp_status mdnp_host_coupling(const mdnp_host_sys* hs, int32_t* b_ptr, int32_t* b_split, int32_t* b_col,
                               double* b_val, double* w, int32_t* r_ptr, int32_t* r_col, double* r_val);
/* z1 = A11^-1 v1 on the host with the factorisation used by the GPU 1D solve
 * (v1, z1 of length n1d): the chain-compressed form (segment interiors as
 * tridiagonal blocks, then the vertex Schur complement) when every segment has
 * at most 32 interior nodes, else the leaves-first LDL^T of the whole tree. */
mdnp_status mdnp_host_tree_solve(const mdnp_host_sys* hs, const double* v1, double* z1);
void mdnp_host_free(mdnp_host_sys* hs);

#ifdef __cplusplus
}
#endif

#endif /* MDNP_H */
