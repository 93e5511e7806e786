// Host-side launchers of the HIP kernels (implemented in krylov.hip and conv.hip).
#pragma once

#include "internal.hpp"

namespace mdnp {

// ---------------------------------------------------------------- Krylov (krylov.hip)
// y = A x over the whole system (CSR, block diagonal over instances).  When
// `mask` is set, instances whose state is not active are skipped.
template <typename T>
void launch_spmv(mdnp_sys* s, const T* x, T* y, const InstState* st, bool mask, hipStream_t stream);
// y = A00 x on slots [n_slots][n3d] that map to instances `inst` (device).
void launch_spmv_a00_slots(mdnp_sys* s, const int32_t* inst, int n_slots, const float* x, float* y,
                           hipStream_t stream);
template <typename T>
void launch_spmv_a00_all(mdnp_sys* s, const T* x, T* y, hipStream_t stream);

// r = b - A x in FP64 with per-block partial sums of r^2 (instances not done).
void launch_residual(mdnp_sys* s, const double* b, const double* x, double* r, double* part, double* partm,
                     const InstState* st, hipStream_t stream);
// per-block partial sums of x^2 over whole vectors
void launch_norm2_partials(mdnp_sys* s, const double* x, double* part, hipStream_t stream);
void launch_init_state(mdnp_sys* s, InstState* st, const double* part, const double* partx, double tol,
                       int max_iters, hipStream_t stream);
void launch_cycle_start(mdnp_sys* s, InstState* st, const double* part, const double* partm, double* g,
                        double* hist, int hist_cap, int m, hipStream_t stream);
template <typename T>
void launch_scale_to(mdnp_sys* s, const double* r, T* v0, const InstState* st, hipStream_t stream);

// preconditioner pieces
template <typename T>
void launch_prec_copy(mdnp_sys* s, const T* v, T* z, const InstState* st, hipStream_t stream);
template <typename T>
void launch_prec_jacobi(mdnp_sys* s, const T* v, T* z, const InstState* st, int want_mode,
                        hipStream_t stream);
void tree_solve_setup(size_t shm_bytes);
// chain-compressed tree solve: largest supported number of interior nodes per segment
constexpr int kChainMaxM = 32;
void chain_solve_setup(size_t shm_bytes);
// LDS bytes of the chain-compressed solve's vertex kernel for V vertices and nlev levels
inline size_t chain_lds_bytes(int V, int S, int nlev) {
  (void)S;
  return sizeof(double) * 3 * (size_t)V + sizeof(int32_t) * (5 * (size_t)V + 2 + (size_t)nlev);
}
template <typename T>
void launch_tree_solve(mdnp_sys* s, const T* v, T* z, const InstState* st, int want_mode,
                       hipStream_t stream);
template <typename T>
void launch_extension(mdnp_sys* s, const T* v, T* z, double* part3, double* part3m, const InstState* st,
                      int want_mode, hipStream_t stream, bool smooth_first = false);
template <typename T>
void launch_block_jacobi3d(mdnp_sys* s, T* z, const InstState* st, int want_mode, hipStream_t stream);
void launch_inv_scale(mdnp_sys* s, const double* part3, const double* part3m, double* inv_s, InstState* st,
                      int want_mode, hipStream_t stream);
// Jacobi smoothing around the network (part3m of launch_inv_scale may be null)
template <typename T>
void launch_a00(mdnp_sys* s, const T* x, T* y, const InstState* st, hipStream_t stream, const T* x2 = nullptr);
template <typename T>
void launch_smooth_pre(mdnp_sys* s, T* z, const InstState* st, double* part3, hipStream_t stream);
template <typename T>
void launch_smooth_post(mdnp_sys* s, T* z, const InstState* st, hipStream_t stream);
// Inner FGMRES(K) with the network as preconditioner for the 3D block
template <typename T>
void launch_inner_fgmres(mdnp_sys* s, T* z, const InstState* st, double* pA, double* pB, double* pW,
                         hipStream_t stream);

// Arnoldi: modified Gram-Schmidt of V[j+1] in passes g = 0 .. mgs_passes(j) - 1,
// kMgsGroup basis vectors per pass; each pass keeps kMgsVals partial sums per
// block (ping-pong buffers of kMgsVals * blk.nblk doubles).
constexpr int kMgsGroup = 4;
constexpr int kMgsVals = kMgsGroup + kMgsGroup * (kMgsGroup - 1) / 2;
inline int mgs_passes(int j) { return (j + kMgsGroup) / kMgsGroup + 1; }
template <typename T>
void launch_mgs(mdnp_sys* s, T* V, int j, int g, const double* part_prev, double* part_cur,
                double* part_w0, double* H, int m, const InstState* st, hipStream_t stream);
template <typename T>
void launch_mgs_finish(mdnp_sys* s, T* V, int j, const double* part_last, const double* part_w0,
                       double* H, double* cs, double* sn, double* g, double* hist, int hist_cap,
                       int m, InstState* st, hipStream_t stream);
void launch_solve_y(mdnp_sys* s, const double* H, const double* g, double* y, int m, const InstState* st,
                    hipStream_t stream);
template <typename T>
void launch_update_x(mdnp_sys* s, const T* Z, const double* y, double* x, int m, const InstState* st,
                     hipStream_t stream);

// ---------------------------------------------------------------- network (conv.hip)
int64_t cnn_layer_count();
// Prepare weight copies for the given flat FP32 weights (device pointer).
void cnn_prepare_weights(CnnState& c, const float* d_w, hipStream_t stream);
// Whole U-net on a batch; `in` FP32 [batch][n^3][2]; `out` FP32 [batch][n^3];
// `saved` non-null: keep every activation for the backward pass.
void cnn_forward_batch(CnnState& c, const float* in, float* out, void* saved, int batch, int n,
                       mdnp_dtype dtype, hipStream_t stream);
int64_t cnn_saved_bytes(int batch, int n, mdnp_dtype dtype);
// Allocate the activation scratch of a batch; false when the allocation fails.
bool cnn_reserve(CnnState& c, int batch, int n, mdnp_dtype dtype);
void cnn_backward_batch(CnnState& c, const void* saved, const float* dy, float* dx, float* dw,
                        int batch, int n, mdnp_dtype dtype, hipStream_t stream);
// In-solver application on the 3D parts of the vectors (type T): reads
// zin0 * inv_s and the distance field, writes z0 = s / alpha * U on the free
// nodes of z (zin and z may be the same vector).  scales = [inv_s; s] per
// instance (null: the context's, set by launch_inv_scale).
// only_stage in [0, 10): launch only that stage of L0a, L0b, L1a, L1b, L2a,
// L2b, U1, D1, U0, D0 (with the head), reading the activations a previous
// whole application left (for timing); -1: the whole network.
template <typename T>
void cnn_apply_in_solver(mdnp_sys* s, const T* zin, T* z, const InstState* st, hipStream_t stream,
                         const double* scales = nullptr, int only_stage = -1);
// Average duration (ms) of each of those ten stages: `reps` launches of the
// stage back to back between two HIP events on `stream`, after one whole
// application to a fixed vector; false if its buffers or events could not
// be created.
// E4M3 network (conv_fp8.hip): weight packing from the (already quantised)
// master weights, the in-solver application, and the calibration helpers
bool fp8_prepare_weights(CnnState& c, hipStream_t stream);
int64_t fp8_act_bytes(int batch, int n);
template <typename Tv>
void cnn_apply_fp8(mdnp_sys* s, const Tv* zin, Tv* z, const InstState* st, hipStream_t stream, const double* isc);
void fp8_zero_amax(unsigned* d_amax, hipStream_t stream);
template <typename Tv>
void fp8_record_amax(mdnp_sys* s, const Tv* zin, const double* isc, void* const act[12], unsigned* d_amax,
                     hipStream_t stream);
// scales from the largest magnitudes (X, L0a, ..., D0): stacked pairs share
// one; each the smallest power of two with 2 amax / s <= 448
void fp8_scales_from_amax(const float amax[11], float out[11]);
bool cnn_layer_times(mdnp_sys* s, hipStream_t stream, int reps, float* ms);
// Per-layer z split of the BF16 sweep convolutions chosen by timing on the
// system's batch and grid (CnnState::sweep_blocks); false if its timing
// buffers or events could not be created (the defaults are then kept).
bool cnn_autotune(mdnp_sys* s, hipStream_t stream, int reps);
// Rounds the weights of every layer (not the biases) of the flat FP32 vector
// d_w in place to E4M3 codes times a power-of-two scale per output channel.
void cnn_quantize_e4m3(float* d_w, hipStream_t stream);
// Wave count of the stencil sweep's z split chosen by timing the batched SpMV
// (mdnp_sys::sweep_target); false if its buffers or events could not be made.
bool spmv_autotune(mdnp_sys* s, hipStream_t stream);
void cnn_release(CnnState& c);
void launch_loss_grad(mdnp_sys* s, const int32_t* inst, int n_slots, const float* r, const float* u,
                      float* du, double* loss, hipStream_t stream);
// Bytes of scratch one loss/gradient evaluation needs.
size_t loss_grad_scratch_bytes(int64_t n3d, int n_slots);
// The allocation-free variant's fixed per-device workspace: its size, the
// one-time resolution of its device address on `device` (which must be
// current), and the launch with that address.
constexpr size_t kLossScratchBytes = size_t(32) << 20;
bool loss_scratch_resolve(int device, void** out);
void launch_loss_grad_fixed(mdnp_sys* s, const int32_t* inst, int n_slots, const float* r, const float* u,
                            float* du, double* loss, void* scratch_ptr, hipStream_t stream);
void launch_pack_input(mdnp_sys* s, const int32_t* inst, int n_slots, const float* r, float* x,
                       hipStream_t stream);
void launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                 float eps, int step, hipStream_t stream);

}  // namespace mdnp
