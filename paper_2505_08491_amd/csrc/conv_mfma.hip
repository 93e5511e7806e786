// Matrix-core (MFMA) implicit-GEMM convolutions for the BF16 network on gfx950.
//
// Each layer is a GEMM  Y[cout][voxel] = sum_k W[cout][k] X[k][voxel]  with
// k = (tap, input channel), evaluated 16 couts x 16 voxels x 32 k at a time by
// v_mfma_f32_16x16x32_bf16 (FP32 accumulation).  The weights are the A
// operand (row = output channel), the input voxels the B operand (column =
// voxel), so every lane ends with 4 consecutive output channels of one voxel
// and stores them as one 8-byte write of the channels-last output.
//
// A block of 16 voxels is 16 consecutive entries of the flattened output grid
// (so no voxel is wasted on the n = 2^k + 1 grid sides); input voxels are read
// straight from global memory (L1/L2 give the 27-fold tap reuse), with a
// per-lane validity mask for the zero padding.  The stride-2 transposed
// convolution is split into its 8 output parity classes, inside each of which
// every voxel has the same 1, 2, 4 or 8 taps and no padding.
#include "conv_common.hpp"

namespace mdnp {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;

constexpr int WAVES = 4;

__device__ __forceinline__ bf16x8 load8(const bf16* p) {
  u32x4 v = *(const u32x4*)p;
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8() {
  u32x4 v = {0u, 0u, 0u, 0u};
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even (finite inputs)
  unsigned int u = __builtin_bit_cast(unsigned int, f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Stride-1 / stride-2 convolution, zero padding 1, channel-stacked input [A | B].
template <int CA, int CB, int COUT, int STRIDE, int MB>
__global__ void __launch_bounds__(WAVES * 64) k_conv_mfma(const bf16* __restrict__ srcA, const bf16* __restrict__ srcB,
                                                         const bf16* __restrict__ W, const float* __restrict__ bias,
                                                         bf16* __restrict__ dst, int n_in, int n_out, int relu,
                                                         const InstState* st, int want_mode) {
  constexpr int CIN = CA + CB;
  constexpr int NB = COUT / 16;
  constexpr int KTOT = 27 * CIN;
  constexpr int KCH = (KTOT + 31) / 32;
  const int bt = blockIdx.z;
  if (st && !(st[bt].active && st[bt].mode == want_mode)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const int64_t nvo = (int64_t)n_out * n_out * n_out;
  const int64_t nvi = (int64_t)n_in * n_in * n_in;
  const int64_t mb0 = ((int64_t)blockIdx.x * WAVES + wave) * MB;
  // per M-block: the lane's voxel, its linear input base and axis validity masks
  int64_t vout[MB];
  int64_t ibase[MB];
  unsigned vmask[MB];  // bits 0-2: x taps valid, 3-5: y, 6-8: z
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int64_t v = (mb0 + m) * 16 + r;
    vout[m] = v;
    unsigned msk = 0;
    int64_t base = 0;
    if (v < nvo) {
      const int ox = (int)(v % n_out), oy = (int)((v / n_out) % n_out), oz = (int)(v / ((int64_t)n_out * n_out));
      const int ix = STRIDE * ox, iy = STRIDE * oy, iz = STRIDE * oz;
      base = ((int64_t)iz * n_in + iy) * n_in + ix;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if (ix + t - 1 >= 0 && ix + t - 1 < n_in) msk |= 1u << t;
        if (iy + t - 1 >= 0 && iy + t - 1 < n_in) msk |= 1u << (3 + t);
        if (iz + t - 1 >= 0 && iz + t - 1 < n_in) msk |= 1u << (6 + t);
      }
    }
    ibase[m] = base;
    vmask[m] = msk;
  }
  const bf16* A = srcA + (int64_t)bt * nvi * CA;
  const bf16* B = CB ? srcB + (int64_t)bt * nvi * CB : nullptr;
  f32x4 acc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = {0.f, 0.f, 0.f, 0.f};
  const int64_t nn = (int64_t)n_in * n_in;
#pragma unroll 2
  for (int c = 0; c < KCH; ++c) {
    const int k0 = c * 32 + g * 8;
    const int tap = k0 / CIN;
    const int ci = k0 - tap * CIN;
    const bool tap_ok = tap < 27;
    const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
    const int64_t toff = (int64_t)(tz - 1) * nn + (int64_t)(ty - 1) * n_in + (tx - 1);
    const unsigned need = (1u << tx) | (8u << ty) | (64u << tz);
    bf16x8 wf[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      wf[nb] = tap_ok ? load8(W + ((int64_t)(nb * 16 + r) * 27 + tap) * CIN + ci) : zero8();
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      bf16x8 xf = zero8();
      if (tap_ok && (vmask[m] & need) == need) {
        const int64_t vin = ibase[m] + toff;
        if (CB == 0 || ci < CA) xf = load8(A + vin * CA + ci);
        else xf = load8(B + vin * CB + (ci - CA));
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[nb], xf, acc[m][nb], 0, 0, 0);
    }
  }
  // epilogue: lane holds couts nb*16 + 4g + j of voxel r
  bf16* Y = dst + (int64_t)bt * nvo * COUT;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    if (vout[m] >= nvo) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = nb * 16 + g * 4;
      float y0 = acc[m][nb][0] + bias[co], y1 = acc[m][nb][1] + bias[co + 1];
      float y2 = acc[m][nb][2] + bias[co + 2], y3 = acc[m][nb][3] + bias[co + 3];
      if (relu) {
        y0 = fmaxf(y0, 0.f); y1 = fmaxf(y1, 0.f); y2 = fmaxf(y2, 0.f); y3 = fmaxf(y3, 0.f);
      }
      uint2 pk;
      pk.x = (unsigned)f2bf(y0) | ((unsigned)f2bf(y1) << 16);
      pk.y = (unsigned)f2bf(y2) | ((unsigned)f2bf(y3) << 16);
      *(uint2*)(Y + vout[m] * COUT + co) = pk;
    }
  }
}

// Stride-2 transposed convolution, one output parity class (px, py, pz) per
// blockIdx.y.  Output o = 2 q + p along each axis; p = 0 takes tap 1 from input
// q, p = 1 takes tap 0 from input q + 1 and tap 2 from input q.
template <int CIN, int COUT, int MB>
__global__ void __launch_bounds__(WAVES * 64) k_tconv_mfma(const bf16* __restrict__ src, const bf16* __restrict__ W,
                                                          const float* __restrict__ bias, bf16* __restrict__ dst,
                                                          int n_in, const InstState* st, int want_mode) {
  constexpr int NB = COUT / 16;
  constexpr int CPT = CIN / 32;  // K chunks per tap
  const int bt = blockIdx.z;
  if (st && !(st[bt].active && st[bt].mode == want_mode)) return;
  const int cls = blockIdx.y;
  const int px = cls & 1, py = (cls >> 1) & 1, pz = (cls >> 2) & 1;
  const int cx = n_in - px, cy = n_in - py, cz = n_in - pz;
  const int64_t ncls = (int64_t)cx * cy * cz;
  const int n_out = 2 * n_in - 1;
  const int64_t nvo = (int64_t)n_out * n_out * n_out;
  const int64_t nvi = (int64_t)n_in * n_in * n_in;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const int64_t mb0 = ((int64_t)blockIdx.x * WAVES + wave) * MB;
  if (mb0 * 16 >= ncls) return;
  int64_t vout[MB], ibase[MB];
  bool ok[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int64_t v = (mb0 + m) * 16 + r;
    ok[m] = v < ncls;
    int qx = 0, qy = 0, qz = 0;
    if (ok[m]) {
      qx = (int)(v % cx);
      qy = (int)((v / cx) % cy);
      qz = (int)(v / ((int64_t)cx * cy));
    }
    vout[m] = ((int64_t)(2 * qz + pz) * n_out + (2 * qy + py)) * n_out + (2 * qx + px);
    ibase[m] = ((int64_t)qz * n_in + qy) * n_in + qx;
  }
  const bf16* X = src + (int64_t)bt * nvi * CIN;
  f32x4 acc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = {0.f, 0.f, 0.f, 0.f};
  const int ntap = 1 << (px + py + pz);
  for (int j = 0; j < ntap; ++j) {
    // decode class tap j: one bit per odd axis (x first)
    int b = 0;
    int tx = 1, ty = 1, tz = 1, ox = 0, oy = 0, oz = 0;
    if (px) { const int s = (j >> b++) & 1; tx = s ? 2 : 0; ox = s ? 0 : 1; }
    if (py) { const int s = (j >> b++) & 1; ty = s ? 2 : 0; oy = s ? 0 : 1; }
    if (pz) { const int s = (j >> b++) & 1; tz = s ? 2 : 0; oz = s ? 0 : 1; }
    const int tap = tz * 9 + ty * 3 + tx;
    const int64_t toff = ((int64_t)oz * n_in + oy) * n_in + ox;
    for (int cc = 0; cc < CPT; ++cc) {
      const int ci = cc * 32 + g * 8;
      bf16x8 wf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) wf[nb] = load8(W + ((int64_t)(nb * 16 + r) * 27 + tap) * CIN + ci);
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        const bf16x8 xf = ok[m] ? load8(X + (ibase[m] + toff) * CIN + ci) : zero8();
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[nb], xf, acc[m][nb], 0, 0, 0);
      }
    }
  }
  bf16* Y = dst + (int64_t)bt * nvo * COUT;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    if (!ok[m]) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = nb * 16 + g * 4;
      const float y0 = acc[m][nb][0] + bias[co], y1 = acc[m][nb][1] + bias[co + 1];
      const float y2 = acc[m][nb][2] + bias[co + 2], y3 = acc[m][nb][3] + bias[co + 3];
      uint2 pk;
      pk.x = (unsigned)f2bf(y0) | ((unsigned)f2bf(y1) << 16);
      pk.y = (unsigned)f2bf(y2) | ((unsigned)f2bf(y3) << 16);
      *(uint2*)(Y + vout[m] * COUT + co) = pk;
    }
  }
}

__global__ void k_w_to_bf16(const float* __restrict__ w, bf16* __restrict__ o, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) o[k] = __float2bfloat16(w[k]);
}

template <int CA, int CB, int COUT, int STRIDE, int MB>
void launch_conv(const ConvP& p, int batch, const bf16* w, hipStream_t stream) {
  const int64_t nvo = (int64_t)p.n_out * p.n_out * p.n_out;
  const int64_t nmb = (nvo + 15) / 16;
  const dim3 grid((unsigned)((nmb + WAVES * MB - 1) / (WAVES * MB)), 1, batch);
  hipLaunchKernelGGL((k_conv_mfma<CA, CB, COUT, STRIDE, MB>), grid, dim3(WAVES * 64), 0, stream, (const bf16*)p.a,
                     (const bf16*)p.b, w, p.bias, (bf16*)p.y, p.n_in, p.n_out, p.relu, p.st, p.want_mode);
}

template <int CIN, int COUT, int MB>
void launch_tconv(const ConvP& p, int batch, const bf16* w, hipStream_t stream) {
  const int64_t ncls = (int64_t)p.n_in * p.n_in * p.n_in;  // largest class
  const int64_t nmb = (ncls + 15) / 16;
  const dim3 grid((unsigned)((nmb + WAVES * MB - 1) / (WAVES * MB)), 8, batch);
  hipLaunchKernelGGL((k_tconv_mfma<CIN, COUT, MB>), grid, dim3(WAVES * 64), 0, stream, (const bf16*)p.a, w, p.bias,
                     (bf16*)p.y, p.n_in, p.st, p.want_mode);
}

}  // namespace

void cnn_prepare_mfma_weights(CnnState& c, const float* d_w, hipStream_t stream) {
  int64_t tot = 0;
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerSpec& L = kLayers[l];
    tot += (int64_t)L.cout * (L.kind == KIND_PT ? 1 : 27) * L.cin;
  }
  if (!c.wmf && hipMalloc(&c.wmf, sizeof(bf16) * (size_t)tot) != hipSuccess) {
    c.wmf = nullptr;
    return;
  }
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerSpec& L = kLayers[l];
    const int64_t nw = (int64_t)L.cout * (L.kind == KIND_PT ? 1 : 27) * L.cin;
    hipLaunchKernelGGL(k_w_to_bf16, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, stream, d_w + c.w_off[l],
                       c.wmf + c.wt_off[l], nw);
  }
}

bool conv_mfma_supported(int layer) { return layer >= 1 && layer <= 9; }

// Layers L0b .. D0 (indices 1 .. 9) with their fixed channel counts.
void conv_mfma_layer(const ConvP& p, int kind, int batch, int layer, CnnState& c, hipStream_t stream) {
  const bf16* w = c.wmf + c.wt_off[layer];
  (void)kind;
  switch (layer) {
    case 1: launch_conv<16, 0, 16, 1, 4>(p, batch, w, stream); break;    // L0b
    case 2: launch_conv<16, 0, 32, 2, 4>(p, batch, w, stream); break;    // L1a
    case 3: launch_conv<32, 0, 32, 1, 4>(p, batch, w, stream); break;    // L1b
    case 4: launch_conv<32, 0, 64, 2, 2>(p, batch, w, stream); break;    // L2a
    case 5: launch_conv<64, 0, 64, 1, 2>(p, batch, w, stream); break;    // L2b
    case 6: launch_tconv<64, 32, 4>(p, batch, w, stream); break;         // U1
    case 7: launch_conv<32, 32, 32, 1, 4>(p, batch, w, stream); break;   // D1
    case 8: launch_tconv<32, 16, 4>(p, batch, w, stream); break;         // U0
    case 9: launch_conv<16, 16, 16, 1, 4>(p, batch, w, stream); break;   // D0
    default: break;
  }
}

}  // namespace mdnp
