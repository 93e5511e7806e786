// Internal structures shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "assembly.hpp"
#include "mdnp.h"

namespace mdnp {

typedef __hip_bfloat16 bf16;

// Doubles per instance in the stencil array: the four stencil values by the
// number of differing coordinates, then the diagonal of a boundary row of S.
constexpr int kStencilStride = 5;

// Per-instance solver state, kept in device memory and read by every kernel of
// an Arnoldi step (masking of converged or inactive instances).
struct InstState {
  int32_t active;      // takes part in the Arnoldi steps of the current cycle
  int32_t done;        // finished (converged or given up)
  int32_t converged;
  int32_t mode;        // 0 = configured preconditioner, 1 = Jacobi fallback
  int32_t jend;        // Arnoldi steps taken in the current cycle
  int32_t iters;       // steps before the fallback
  int32_t fb_iters;    // steps on the fallback
  int32_t stalled;     // set by the cycle-start kernel when the stall rule fires
  int32_t nhist;       // entries written to the history
  int32_t cycles;
  int32_t max_iters;   // step cap of the current mode
  int32_t bad_input;   // ||b|| or ||x0|| is not finite (the solve is refused)
  double bnorm;        // ||b||
  double beta;         // ||r|| at the start of the current cycle
  double rel;          // true relative residual at the start of the current cycle
  double prev_rel;     // same, one cycle earlier
  double tol;
  double scale3d;      // ||b0|| of the current preconditioner input (network normalisation)
};

// Reduction tiling: contiguous element chunks, each inside one instance.
struct Blocks {
  int nblk = 0;
  int chunk = 0;
  int32_t* inst = nullptr;     // [nblk]
  int64_t* start = nullptr;    // [nblk] element start (global)
  int64_t* end = nullptr;      // [nblk]
  int32_t* first = nullptr;    // [n_inst + 1] first block of each instance
  std::vector<int32_t> h_first;
};

struct CnnState {
  bool ready = false;
  mdnp_dtype dtype = MDNP_F32;
  bool fp8_weights = false;    // weights rounded to E4M3 x per-channel power-of-two scales (run as BF16)
  const float* w = nullptr;    // flat weights in use [353713] (owned copy or borrowed)
  float* w_own = nullptr;      // owned copy set by mdnp_set_preconditioner
  float* wt = nullptr;         // per-layer [taps][cin][cout] copies for the direct kernels
  bf16* wmf = nullptr;         // per-layer bf16 [cout][taps][cin] copies for the MFMA kernels
  std::vector<int64_t> w_off, wt_off, b_off;  // per-layer offsets
  int batch = 0, n = 0;
  void* act[12] = {};          // activation buffers
  size_t act_bytes = 0;
  double* inv_s = nullptr;     // [n_inst] 1 / ||b0||, followed by [n_inst] ||b0||
  void* bwd = nullptr;         // backward scratch
  size_t bwd_bytes = 0;
  void* loss = nullptr;        // loss scratch
  size_t loss_bytes = 0;
  // stand-alone BF16 forward: the packed input split into its two channels for
  // the MFMA first layer, with per-sample offsets and unit scales
  float* split = nullptr;      // [2][batch * n^3]
  size_t split_n = 0;
  int64_t* std_off = nullptr;  // [batch] b * n^3
  double* std_ones = nullptr;  // [batch] 1
  int std_batch = 0, std_n = 0;
  // launch shape of each BF16 layer set by the autotuner, by layer (L0a = 0 ..
  // D0 = 9; 0: built-in default): for the sweep layers the workgroups their z
  // split aims at, for L1a, L2a, U1, U0 the 16-voxel M blocks per wave
  int sweep_blocks[11] = {};
  // output rows per wave (pair) of the sweep layers L0b, L1b, D1, D0, and the
  // workgroup count of the transposed layers U1, U0 (0: default)
  int tile_mb[11] = {};
  // 16-column x blocks per workgroup of the sweep layers L0a, L0b, L1b, D1, D0
  // (0: as many as fit; fewer splits each row over more workgroups)
  int tile_xb[11] = {};
  // E4M3 weights and activations on the FP8 matrix cores (MDNP_FP8E4M3_ACT):
  // packed weight fragments and per-output-channel scales of the ten 3x3x3
  // layers, and the activation scales of X, L0a, L0b, L1a, L1b, L2a, L2b, U1,
  // D1, U0, D0 (0: not set)
  uint8_t* w8 = nullptr;
  std::vector<int64_t> w8_off;
  float* w8s = nullptr;
  std::vector<int64_t> w8s_off;
  float act8_scale[11] = {};
  // set while mdnp_fp8_calibrate runs the network in FP32 to record the
  // largest magnitude of every tensor into fp8_amax (device, 11 words)
  bool fp8_calibrating = false;
  unsigned* fp8_amax = nullptr;
};

// Jacobi pre/post-smoothing of the neural 3D solve (sweeps = 0: off) and its
// scratch vectors (full length, vector type).
struct SmoothState {
  int sweeps = 0;
  double omega = 0.0;
  void* sb = nullptr;          // b0
  void* sr = nullptr;          // network input b0 - A00 z
  void* t = nullptr;           // A00 z
};

// Inner FGMRES(steps) with the network as preconditioner for the 3D block
// (steps = 0: one network application).
struct InnerState {
  int steps = 0;
  void* IV = nullptr;          // (steps + 1) x ntot basis vectors (1D parts zero)
  void* IZ = nullptr;          // steps x ntot preconditioned directions
  double* IH = nullptr;        // n_inst x (steps + 1) x steps
  double* IH0 = nullptr;       // n_inst x steps: ||A00 z_j|| before orthogonalisation
  double* y = nullptr;         // n_inst x steps
  int* jend = nullptr;         // n_inst
  double* ones = nullptr;      // 2 n_inst ones: unit scaling of the network input/output
};

struct SolveWork {
  int m = 0;                   // restart the buffers were sized for
  int last_m = -1;             // restart of the last cycle run (-1: no solve yet)
  int hist_cap = 0;
  void* V = nullptr;           // (m+1) x ntot vectors
  void* Z = nullptr;           // m x ntot
  double* r = nullptr;         // ntot
  double* H = nullptr;         // n_inst x (m+1) x m
  double* cs = nullptr;
  double* sn = nullptr;
  double* g = nullptr;         // n_inst x (m+1)
  double* y = nullptr;         // n_inst x m
  double* part = nullptr;      // partial sums: 3 x blk, blk3, mblk, mblk3
  double* hist = nullptr;      // n_inst x hist_cap
  InstState* st = nullptr;     // n_inst
  double* xs = nullptr;        // ntot: x at the start of the last cycle (the last finite iterate)
  // one restart cycle as graphs of at most kCycleChunk Arnoldi steps each, so
  // the host can stop launching once no instance takes part any more
  std::vector<hipGraphExec_t> graphs;
  int graph_m = -1, graph_fb = -1;
  InstState* h_st = nullptr;   // pinned host copy of st, read between chunks
  std::vector<double> h_hist;
  std::vector<int32_t> h_nhist;
};

}  // namespace mdnp

struct mdnp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<mdnp_sys*> systems;
  mdnp::CnnState cnn;              // state of the stand-alone network calls
  void* loss_scratch = nullptr;    // this device's fixed loss workspace (mdnp_loss_grad_noalloc)
};

struct mdnp_sys {
  mdnp_ctx* ctx = nullptr;
  int n_inst = 0, n_cells = 0, n = 0, n3d = 0;
  mdnp_dtype vec_dtype = MDNP_F32;
  std::vector<mdnp::HostInstance> host;
  std::vector<int64_t> off;        // [n_inst + 1] vector offsets
  std::vector<int64_t> nnz_off;    // [n_inst + 1]
  int64_t ntot = 0, nnz_tot = 0, mnz_tot = 0;
  std::vector<int64_t> m_nnz, m_rows;  // per instance: entries and non-empty rows of M
  std::vector<int64_t> c_gauss, c_bnnz, c_snnz;  // per instance: Gauss points, entries of W B and of B^T | R
  int max_n1d = 0;
  // device arrays
  int64_t* d_off = nullptr;
  // operator A = S + M: S the constant 27-point stencil of the free 3D nodes
  // (unit rows on the Dirichlet nodes), M the coupling / 1D part in CSR
  double* d_stencil = nullptr;     // [n_inst * kStencilStride] stencil value by differing coordinates,
                                   // then the value of a boundary row of S (1 Dirichlet, 0 Neumann)
  bool neumann = false;            // natural boundary on the cube faces (every instance)
  int sweep_target = 0;            // workgroups aimed at by the stencil sweep's z split (0: 2048)
  int32_t* d_mptr = nullptr;       // [ntot + 1], global entry offsets
  uint8_t* d_mfree = nullptr;      // [ntot] 1 where the row has no M entry
  int32_t* d_mcol = nullptr;       // global column indices
  double* d_mval64 = nullptr;
  float* d_mval32 = nullptr;
  int32_t* d_ma01 = nullptr;       // [n_inst * n3d] first M entry of each 3D row with a 1D column
  int32_t* d_mrows = nullptr;      // global ids of the rows with M entries (per instance: 3D rows, then 1D rows)
  int32_t* d_mlp = nullptr;        // [rows listed + 1] M entry range of each listed row
  int32_t* d_a01p = nullptr;       // [rows listed + 1] A01 entry range of each listed row (empty for 1D rows)
  int32_t* d_a01c = nullptr;       // A01 global column indices (1D nodes)
  double* d_a01v64 = nullptr;
  float* d_a01v32 = nullptr;
  int32_t* d_m3e = nullptr;        // [rows listed] end of each listed row's 3D-column M entries
  // M in factored form, M = B^T W B + R (the stencil-sweep path): a first pass
  // t = W B x over the Gauss points, then B^T t + R x over the listed rows
  int32_t* d_gp = nullptr;         // [Gauss points + 1] entry offsets of W B
  int32_t* d_gsplit = nullptr;     // [Gauss points] end of each point's 3D-column entries
  int32_t* d_gcol = nullptr;       // global x indices
  double* d_gval64 = nullptr;      // W_q B_q entries
  float* d_gval32 = nullptr;
  int32_t* d_sp = nullptr;         // [rows listed + 1] entry offsets of B^T | R
  int32_t* d_scol = nullptr;       // >= 0: a Gauss point (global index into t), < 0: ~(global x index)
  double* d_sval64 = nullptr;
  float* d_sval32 = nullptr;
  double* d_ct = nullptr;          // [Gauss points] t, FP64 or FP32 as the vectors
  double* d_dinv = nullptr;        // [ntot] 1 / diag(A)
  float* d_dinv32 = nullptr;       // the same in FP32 (relaxation steps of the smoothing)
  float* d_dist = nullptr;         // [n_inst * n3d]
  double* d_alpha = nullptr;       // [n_inst]
  // tree factorisation
  int32_t* d_t_off = nullptr;      // [n_inst + 1] node offsets (cumulative n1d)
  int32_t* d_t_lvloff = nullptr;   // [n_inst + 1] offsets into lvl_ptr
  int32_t* d_t_lvlptr = nullptr;   // level pointers, local to each instance's node block
  int32_t* d_t_lvlnodes = nullptr; // local node ids, per instance block
  int32_t* d_t_parent = nullptr;   // local
  int32_t* d_t_childptr = nullptr; // [node + 1] absolute into child_idx (per instance n1d+1 entries)
  int32_t* d_t_childidx = nullptr; // local node ids
  double* d_t_lval = nullptr;
  double* d_t_dinv = nullptr;
  // chain-compressed tree solve (per instance offsets into concatenated arrays)
  struct ChainDev {
    int enabled = 0;                 // all instances fit the on-chip form
    int max_v = 0, max_s = 0;        // largest vertex / segment count
    int max_m = 0;                   // most interior nodes per segment
    size_t lds_bytes = 0;            // dynamic LDS of the solve kernel
    int32_t* meta = nullptr;         // [n_inst][8]: m, S, V, vlvl count, seg off, vtx off, vlvl off, vchild off
    int64_t* soff = nullptr;         // [n_inst][2]: offsets of the [m-1][S] and [m][S] step arrays
    double* fmul = nullptr;
    double* eup = nullptr;
    double* pinv = nullptr;
    double* gp = nullptr;
    double* gq = nullptr;
    double* ap = nullptr;
    double* aq = nullptr;
    int32_t* sp = nullptr;           // local vertex ids
    int32_t* sq = nullptr;
    int32_t* vparent = nullptr;      // local vertex ids
    int32_t* vseg = nullptr;         // local segment ids
    int32_t* vchild_ptr = nullptr;   // [V + 1] per instance, local offsets into the instance's vchild_idx
    int32_t* vchild_idx = nullptr;
    int32_t* vlvl_ptr = nullptr;     // [levels + 1] per instance, local
    int32_t* vlvl_nodes = nullptr;
    double* vlval = nullptr;
    double* vdinv = nullptr;
    double* t01 = nullptr;           // [segments][2] scratch: segment couplings
    double* zv = nullptr;            // [vertices] scratch: FP64 vertex values
  } chain;
  mdnp::Blocks blk;                // whole vectors
  mdnp::Blocks blk3;               // 3D parts only
  mdnp::Blocks mblk;               // coupling-row lists
  mdnp::Blocks mblk3;              // coupling-row lists, 3D rows only
  mdnp::Blocks gblk;               // Gauss-point lists
  // preconditioner
  mdnp_prec_kind kind = MDNP_PREC_NONE;
  bool prec_set = false;
  double alpha_override = 0.0;
  mdnp::CnnState cnn;
  mdnp::SmoothState smooth;
  mdnp::InnerState inner;
  mdnp::SolveWork work;
};
