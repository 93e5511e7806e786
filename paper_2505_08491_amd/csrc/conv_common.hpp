// Layer table of the U-net and the argument block of the convolution kernels.
#pragma once

#include "internal.hpp"

namespace mdnp {

enum { KIND_S1 = 0, KIND_S2 = 1, KIND_T2 = 2, KIND_PT = 3 };

struct LayerSpec {
  int kind, cin, cout, relu;
};

// L0a L0b L1a L1b L2a L2b U1 D1 U0 D0 H (Section 4.2 recursion with three levels)
constexpr int kNumLayers = 11;
constexpr LayerSpec kLayers[kNumLayers] = {
    {KIND_S1, 2, 16, 1},  {KIND_S1, 16, 16, 1}, {KIND_S2, 16, 32, 1}, {KIND_S1, 32, 32, 1},
    {KIND_S2, 32, 64, 1}, {KIND_S1, 64, 64, 1}, {KIND_T2, 64, 32, 0}, {KIND_S1, 64, 32, 1},
    {KIND_T2, 32, 16, 0}, {KIND_S1, 32, 16, 1}, {KIND_PT, 16, 1, 0}};

struct ConvP {
  const void* a = nullptr;   // source A [batch][vox][lda], channels [0, ca)
  int ca = 0, lda = 0;
  const void* b = nullptr;   // source B (channel stacking), channels [ca, ca + cb)
  int cb = 0, ldb = 0;
  int64_t a_bs = 0, b_bs = 0;  // batch strides in elements
  int n_in = 0, n_out = 0;
  const float* wt = nullptr;   // [taps][cin][cout] (direct kernels)
  const float* bias = nullptr;
  int cout = 0;
  void* y = nullptr;
  int ldy = 0, y_choff = 0;
  int64_t y_bs = 0;
  int relu = 0, accumulate = 0;
  const InstState* st = nullptr;  // optional: batch index = instance, skip unless active in want_mode
  int want_mode = 0;
};

// matrix-core path (conv_mfma.hip)
void cnn_prepare_mfma_weights(CnnState& c, const float* d_w, hipStream_t stream);
bool conv_mfma_supported(int layer);
void conv_mfma_layer(const ConvP& p, int kind, int batch, int layer, CnnState& c, hipStream_t stream);
// in-solver first layer (input built from the Krylov vector) and fused D0 + head + unscale
template <typename Tv>
void conv_mfma_in0(const CnnState& c, const Tv* z, const int64_t* off, const double* inv_s, const float* dist,
                   int n, int batch, bf16* a0, const InstState* st, hipStream_t stream);
template <typename Tv>
void conv_mfma_d0_head(const CnnState& c, const bf16* u0, const bf16* s0, int n, int batch, Tv* z,
                       const int64_t* off, const double* alpha, double alpha_override, const double* scale,
                       const InstState* st, hipStream_t stream);

}  // namespace mdnp
