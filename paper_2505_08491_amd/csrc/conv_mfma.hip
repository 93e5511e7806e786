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
#include <algorithm>
#include <type_traits>

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

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap the linear workgroup id so that every XCD gets a contiguous range
// of tiles: neighbouring tiles, which share halo rows, then meet in one L2.
__device__ __forceinline__ void xcd_remap(int& bx, int& bz) {
  const int gx = gridDim.x, total = gridDim.x * gridDim.z;
  const int lin = blockIdx.x + gx * blockIdx.z;
  const int per = total / 8;
  int tgt = lin;
  if (lin < per * 8) tgt = (lin % 8) * per + lin / 8;
  bx = tgt % gx;
  bz = tgt / gx;
}

struct MfmaArgs {
  const bf16* a = nullptr;      // source A [batch][vox][CA]
  const bf16* b = nullptr;      // source B [batch][vox][CB] (channel stacking)
  const bf16* w = nullptr;      // weights [COUT][27][CIN] bf16
  const bf16* wrows = nullptr;  // 16-channel layers: weights [16][3 ty][KCT * 32] (k_conv16_rows)
  const void* zero16 = nullptr; // 16 zero bytes in device memory (padding source of the LDS loads)
  const float* bias = nullptr;
  bf16* y = nullptr;            // output [batch][vox][COUT]
  int n_in = 0, n_out = 0, relu = 0;
  const InstState* st = nullptr;
  int want_mode = 0;
  // first layer inside the solver: channel 0 = z0 * inv_s, channel 1 = distance
  const void* z = nullptr;
  const int64_t* off = nullptr;
  const double* inv_s = nullptr;
  const float* dist = nullptr;
  // last layers inside the solver: 1x1 head and unscaling into z
  const float* wh = nullptr;
  const float* bh = nullptr;
  void* zout = nullptr;
  const double* alpha = nullptr;
  double alpha_override = 0.0;
  const double* scale = nullptr;
};

__device__ __forceinline__ bf16x8 pack2(float x0, float x1) {
  u32x4 v = {(unsigned)f2bf(x0) | ((unsigned)f2bf(x1) << 16), 0u, 0u, 0u};
  return __builtin_bit_cast(bf16x8, v);
}

// Stride-1 / stride-2 convolution, zero padding 1, channel-stacked input [A | B].
// IN = 1: the input is built on the fly from the Krylov vector (first layer
// inside the solver, CA = 8 with channels 2..7 zero).  EPI = 1: ReLU, the 1x1
// head and the unscaling z0 = ||b0|| / alpha * U are applied in the epilogue
// and written into the Krylov vector (last layers inside the solver).
// EDGE = 1: only the output voxels with x = n_out - 1 (the column the
// LDS-tiled kernel leaves out), enumerated over (y, z).
template <int CA, int CB, int COUT, int STRIDE, int MB, int IN, int EPI, typename Tv, int EDGE = 0>
__global__ void __launch_bounds__(WAVES * 64) k_conv_mfma(MfmaArgs p) {
  constexpr int CIN = CA + CB;
  constexpr int NB = COUT / 16;
  constexpr int KTOT = 27 * CIN;
  constexpr int KCH = (KTOT + 31) / 32;
  int bxr, bt;
  xcd_remap(bxr, bt);
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  const int n_in = p.n_in, n_out = p.n_out;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const int64_t nvo = (int64_t)n_out * n_out * n_out;
  const int64_t nvi = (int64_t)n_in * n_in * n_in;
  const int64_t mb0 = ((int64_t)bxr * WAVES + wave) * MB;
  // per M-block: the lane's voxel, its linear input base and axis validity masks
  int64_t vout[MB];
  int64_t ibase[MB];
  unsigned vmask[MB];  // bits 0-2: x taps valid, 3-5: y, 6-8: z
  bool vok[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int64_t e = (mb0 + m) * 16 + r;
    const bool ok = EDGE ? e < (int64_t)n_out * n_out : e < nvo;
    const int64_t v = EDGE ? e * n_out + (n_out - 1) : e;
    vout[m] = v;
    vok[m] = ok;
    unsigned msk = 0;
    int64_t base = 0;
    if (ok) {
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
  const bf16* A = IN ? nullptr : p.a + (int64_t)bt * nvi * CA;
  const bf16* B = CB ? p.b + (int64_t)bt * nvi * CB : nullptr;
  const Tv* Z = IN ? (const Tv*)p.z + p.off[bt] : nullptr;
  const float* D = IN ? p.dist + (int64_t)bt * nvi : nullptr;
  const float sc = IN ? (float)p.inv_s[bt] : 0.0f;
  f32x4 acc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = {0.f, 0.f, 0.f, 0.f};
  const int64_t nn = (int64_t)n_in * n_in;
  auto fetch = [&](int c, bf16x8 (&wf)[NB], bf16x8 (&xf)[MB]) {
    const int k0 = c * 32 + g * 8;
    const int tap = k0 / CIN;
    const int ci = k0 - tap * CIN;
    const bool tap_ok = tap < 27;
    const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
    const int64_t toff = (int64_t)(tz - 1) * nn + (int64_t)(ty - 1) * n_in + (tx - 1);
    const unsigned need = (1u << tx) | (8u << ty) | (64u << tz);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      wf[nb] = tap_ok ? load8(p.w + ((int64_t)(nb * 16 + r) * 27 + tap) * CIN + ci) : zero8();
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      bf16x8 x = zero8();
      if (tap_ok && (vmask[m] & need) == need) {
        const int64_t vin = ibase[m] + toff;
        if (IN) x = pack2((float)Z[vin] * sc, D[vin]);
        else if (CB == 0 || ci < CA) x = load8(A + vin * CA + ci);
        else x = load8(B + vin * CB + (ci - CA));
      }
      xf[m] = x;
    }
  };
  auto mma = [&](const bf16x8 (&wf)[NB], const bf16x8 (&xf)[MB]) {
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[nb], xf[m], acc[m][nb], 0, 0, 0);
  };
  bf16x8 wA[NB], xA[MB], wB[NB], xB[MB];
  fetch(0, wA, xA);
#pragma unroll
  for (int c = 0; c < KCH; c += 2) {
    if (c + 1 < KCH) fetch(c + 1, wB, xB);
    mma(wA, xA);
    if (c + 2 < KCH) fetch(c + 2, wA, xA);
    if (c + 1 < KCH) mma(wB, xB);
  }
  if (EPI == 0) {
    // lane holds couts nb*16 + 4g + j of voxel r
    bf16* Y = p.y + (int64_t)bt * nvo * COUT;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      if (!vok[m]) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + g * 4;
        float y0 = acc[m][nb][0] + p.bias[co], y1 = acc[m][nb][1] + p.bias[co + 1];
        float y2 = acc[m][nb][2] + p.bias[co + 2], y3 = acc[m][nb][3] + p.bias[co + 3];
        if (p.relu) {
          y0 = fmaxf(y0, 0.f); y1 = fmaxf(y1, 0.f); y2 = fmaxf(y2, 0.f); y3 = fmaxf(y3, 0.f);
        }
        uint2 pk;
        pk.x = (unsigned)f2bf(y0) | ((unsigned)f2bf(y1) << 16);
        pk.y = (unsigned)f2bf(y2) | ((unsigned)f2bf(y3) << 16);
        *(uint2*)(Y + vout[m] * COUT + co) = pk;
      }
    }
  } else {
    // ReLU, then the 1x1 head over the 16 channels held by the 4 lane groups of voxel r
    const double a = p.alpha_override > 0.0 ? p.alpha_override : p.alpha[bt];
    const float f = (float)(p.scale[bt] / a);
    Tv* zo = (Tv*)p.zout + p.off[bt];
    const int co = g * 4;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      float h = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // the layer output is rounded to BF16 as on the stored path
        const float yj = __bfloat162float(__float2bfloat16(fmaxf(acc[m][0][j] + p.bias[co + j], 0.f)));
        h = fmaf(p.wh[co + j], yj, h);
      }
      h += __shfl_xor(h, 16, 64);
      h += __shfl_xor(h, 32, 64);
      const int64_t v = vout[m];
      if (g == 0 && vok[m]) {
        const int ox = (int)(v % n_out), oy = (int)((v / n_out) % n_out), oz = (int)(v / ((int64_t)n_out * n_out));
        const bool bnd = ox == 0 || oy == 0 || oz == 0 || ox == n_out - 1 || oy == n_out - 1 || oz == n_out - 1;
        if (!bnd) zo[v] = (Tv)(f * (h + p.bh[0]));
      }
    }
  }
}

// The column x = n - 1 of a stride-1 layer (left out by the sweep kernels),
// plane oz of instance bt, by the nw = blockDim.x / 64 waves of one workgroup:
// all of that column's blocks of 16 consecutive y (at most YBM of them) are
// covered, so that every weight fragment loaded serves up to YBM MFMAs; wave w
// accumulates the K chunks c = w, w + nw, ...; the partial sums meet in LDS
// (red: nw * nyb * COUT / 16 * 1 KiB) and the waves finish the (block, output
// block) fragments in turn (bias, ReLU, BF16 store).  IN = 1 builds the first
// layer's input.  Called by the sweep kernels' extra workgroups and by
// k_conv_edge.
constexpr int kEdgeGroups = 8;  // partial sums of the edge column's K loop

template <int CA, int CB, int COUT, int IN, typename Tv, int YBM>
__device__ __forceinline__ void edge_plane(const MfmaArgs& p, int oz, int bt, f32x4* red) {
  constexpr int CIN = CA + CB;
  constexpr int NB = COUT / 16;
  constexpr int KCH = (27 * CIN + 31) / 32;
  const int n = p.n_out;
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const int nyb = (n + 15) / 16;
  const int ox = n - 1;
  const int64_t nn = (int64_t)n * n, nv = nn * n;
  int64_t base[YBM];
  unsigned msk[YBM];
#pragma unroll
  for (int m = 0; m < YBM; ++m) {
    const int oy = m * 16 + r;
    const bool ok = m < nyb && oy < n;
    base[m] = ((int64_t)oz * n + (ok ? oy : 0)) * n + ox;
    unsigned mk = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (ox + t - 1 >= 0 && ox + t - 1 < n) mk |= 1u << t;
      if (oy + t - 1 >= 0 && oy + t - 1 < n) mk |= 1u << (3 + t);
      if (oz + t - 1 >= 0 && oz + t - 1 < n) mk |= 1u << (6 + t);
    }
    msk[m] = ok ? mk : 0u;
  }
  const bf16* A = IN ? nullptr : p.a + (int64_t)bt * nv * CA;
  const bf16* B = CB ? p.b + (int64_t)bt * nv * CB : nullptr;
  const Tv* Z = IN ? (const Tv*)p.z + p.off[bt] : nullptr;
  const float* D = IN ? p.dist + (int64_t)bt * nv : nullptr;
  const float sc = IN ? (float)p.inv_s[bt] : 0.0f;
  // K chunks c = k mod kEdgeGroups form partial sum k, summed in the order
  // k = 0, 1, ... whatever the number of waves, so the column does not depend
  // on the workgroup shape of the launch that computes it
  for (int kg = wave; kg < kEdgeGroups; kg += nw) {
    f32x4 acc[YBM][NB];
#pragma unroll
    for (int m = 0; m < YBM; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[m][nb] = {0.f, 0.f, 0.f, 0.f};
    for (int c = kg; c < KCH; c += kEdgeGroups) {
      const int k0 = c * 32 + g * 8;
      const int tap = k0 / CIN;
      const int ci = k0 - tap * CIN;
      const bool tap_ok = tap < 27;
      const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
      const unsigned need = (1u << tx) | (8u << ty) | (64u << tz);
      const int64_t toff = (int64_t)(tz - 1) * nn + (int64_t)(ty - 1) * n + (tx - 1);
      bf16x8 wf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        wf[nb] = tap_ok ? load8(p.w + ((int64_t)(nb * 16 + r) * 27 + tap) * CIN + ci) : zero8();
      bf16x8 x[YBM];
#pragma unroll
      for (int m = 0; m < YBM; ++m) {
        x[m] = zero8();
        if (tap_ok && (msk[m] & need) == need) {
          const int64_t vin = base[m] + toff;
          if (IN) x[m] = pack2((float)Z[vin] * sc, D[vin]);
          else if (CB == 0 || ci < CA) x[m] = load8(A + vin * CA + ci);
          else x[m] = load8(B + vin * CB + (ci - CA));
        }
      }
#pragma unroll
      for (int m = 0; m < YBM; ++m)
        if (m < nyb) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[nb], x[m], acc[m][nb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int m = 0; m < YBM; ++m)
      if (m < nyb) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) red[((kg * nyb + m) * NB + nb) * 64 + lane] = acc[m][nb];
      }
  }
  __syncthreads();
  bf16* Y = p.y + (int64_t)bt * nv * COUT;
  for (int f = wave; f < nyb * NB; f += nw) {
    const int m = f / NB, nb = f - m * NB;
    f32x4 sum = red[(m * NB + nb) * 64 + lane];
    for (int w = 1; w < kEdgeGroups; ++w) {
      const f32x4 o = red[((w * nyb + m) * NB + nb) * 64 + lane];
      sum += o;
    }
    const int oy = m * 16 + r;
    if (oy >= n) continue;
    const int co = nb * 16 + g * 4;
    float y0 = sum[0] + p.bias[co], y1 = sum[1] + p.bias[co + 1];
    float y2 = sum[2] + p.bias[co + 2], y3 = sum[3] + p.bias[co + 3];
    if (p.relu) {
      y0 = fmaxf(y0, 0.f); y1 = fmaxf(y1, 0.f); y2 = fmaxf(y2, 0.f); y3 = fmaxf(y3, 0.f);
    }
    uint2 pk;
    pk.x = (unsigned)f2bf(y0) | ((unsigned)f2bf(y1) << 16);
    pk.y = (unsigned)f2bf(y2) | ((unsigned)f2bf(y3) << 16);
    const int64_t v = ((int64_t)oz * n + oy) * n + ox;
    *(uint2*)(Y + v * COUT + co) = pk;
  }
}

// Edge column of a stride-1 layer as a kernel of its own: one workgroup of
// KSW waves per plane (grid x = planes, z = instances).
template <int CA, int CB, int COUT, int IN, typename Tv, int KSW, int YB>
__global__ void __launch_bounds__(KSW * 64) k_conv_edge(MfmaArgs p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char edge_lds[];
  const int bt = blockIdx.z;
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  edge_plane<CA, CB, COUT, IN, Tv, YB>(p, blockIdx.x, bt, (f32x4*)edge_lds);
}

// Largest n whose edge column the sweep kernels take in extra workgroups, and
// the LDS those workgroups need (one partial sum per K-chunk group).
constexpr int kEdgeYB = 5;
inline size_t edge_lds_bytes(int n, int cout) {
  return (size_t)kEdgeGroups * ((n + 15) / 16) * (cout / 16) * 64 * 16;
}

template <int CA, int CB, int COUT, int IN, typename Tv>
void launch_edge(const MfmaArgs& a, int batch, hipStream_t stream) {
  constexpr int KSW = 8, YB = 5;  // up to 80 rows: n <= 80
  constexpr size_t lds = (size_t)kEdgeGroups * YB * (COUT / 16) * 64 * 16;
  static_assert(lds <= 160 * 1024, "edge partials exceed LDS");
  const int n = a.n_out;
  if (n > 16 * YB) {  // the global-load kernel's edge mode
    constexpr int MBE = 1;
    const int64_t nmb = ((int64_t)n * n + 15) / 16;
    const dim3 grid((unsigned)((nmb + WAVES * MBE - 1) / (WAVES * MBE)), 1, batch);
    hipLaunchKernelGGL((k_conv_mfma<CA, CB, COUT, 1, MBE, IN, 0, Tv, 1>), grid, dim3(WAVES * 64), 0, stream, a);
    return;
  }
  auto kern = k_conv_edge<CA, CB, COUT, IN, Tv, KSW, YB>;
  if (lds > 65536) hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(kern, dim3((unsigned)n, 1, batch), dim3(KSW * 64), lds, stream, a);
}

// Stride-1 convolution with the input tile staged in LDS.  A workgroup owns the
// output rows y0..y0+TY-1 of the planes z0..z0+TZ-1 for x in [0, n-1) (the
// column x = n-1 is left to the EDGE variant of k_conv_mfma, so that every
// M-block is 16 consecutive x of one row: n - 1 = 2^k is a multiple of 16).
// The tile holds planes z0-1..z0+TZ, rows y0-1..y0+TY, x = -1..n-1, zero
// outside the grid, so the tap loop needs no bounds checks.  IN / EPI as in
// k_conv_mfma.
template <int CA, int CB, int COUT, int TZ, int TY, int MB, int IN, int EPI, typename Tv, int WL>
__global__ void __launch_bounds__(512) k_conv_lds(MfmaArgs p) {
  constexpr int CIN = IN ? 8 : CA + CB;  // GEMM channels per tap
  constexpr int CL = IN ? 2 : CA + CB;   // channels stored per tile voxel
  constexpr int NB = COUT / 16;
  constexpr int KCH = (27 * CIN + 31) / 32;
  constexpr int YW = TY + 2, ZW = TZ + 2;
  extern __shared__ unsigned short tile[];
  int bxr, bt;
  xcd_remap(bxr, bt);
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  const int n = p.n_out;
  const int XW = n + 1;
  const int ytiles = (n + TY - 1) / TY;
  const int y0 = (bxr % ytiles) * TY, z0 = (bxr / ytiles) * TZ;
  const int64_t nv = (int64_t)n * n * n;
  const int nthr = blockDim.x;
  // ---- stage the input tile (and the weights when WL): every thread issues
  // a batch of independent global loads before it stores them, so that the
  // load latency is paid once per batch
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int NLD = 8;
  if (IN) {
    const Tv* Z = (const Tv*)p.z + p.off[bt];
    const float* D = p.dist + (int64_t)bt * nv;
    const float sc = (float)p.inv_s[bt];
    const int total = ZW * YW * XW;
    for (int q0 = threadIdx.x; q0 < total; q0 += NLD * nthr) {
      float zv[NLD], dv[NLD];
      bool ok[NLD];
#pragma unroll
      for (int k = 0; k < NLD; ++k) {
        const int q = q0 + k * nthr;
        const int row = q / XW, xx = q - row * XW;
        const int zz = row / YW, yy = row - zz * YW;
        const int gx = xx - 1, gy = y0 + yy - 1, gz = z0 + zz - 1;
        ok[k] = q < total && gx >= 0 && gy >= 0 && gz >= 0 && gx < n && gy < n && gz < n;
        const int64_t v = ok[k] ? ((int64_t)gz * n + gy) * n + gx : 0;
        zv[k] = ok[k] ? (float)Z[v] : 0.0f;
        dv[k] = ok[k] ? D[v] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < NLD; ++k) {
        const int q = q0 + k * nthr;
        if (q < total)
          ((unsigned*)tile)[q] = ok[k] ? ((unsigned)f2bf(zv[k] * sc) | ((unsigned)f2bf(dv[k]) << 16)) : 0u;
      }
    }
  } else {
    constexpr int CPV = CL / 8;
    constexpr int CPA = CA / 8;
    const bf16* A = p.a + (int64_t)bt * nv * CA;
    const bf16* B = CB ? p.b + (int64_t)bt * nv * CB : nullptr;
    const int total = ZW * YW * XW * CPV;
    for (int q0 = threadIdx.x; q0 < total; q0 += NLD * nthr) {
      u32x4 val[NLD];
#pragma unroll
      for (int k = 0; k < NLD; ++k) {
        const int q = q0 + k * nthr;
        const int vt = q / CPV, ch = q - vt * CPV;
        const int row = vt / XW, xx = vt - row * XW;
        const int zz = row / YW, yy = row - zz * YW;
        const int gx = xx - 1, gy = y0 + yy - 1, gz = z0 + zz - 1;
        val[k] = u32x4{0u, 0u, 0u, 0u};
        if (q < total && gx >= 0 && gy >= 0 && gz >= 0 && gx < n && gy < n && gz < n) {
          const int64_t v = ((int64_t)gz * n + gy) * n + gx;
          val[k] = (CB == 0 || ch < CPA) ? *(const u32x4*)(A + v * CA + ch * 8)
                                         : *(const u32x4*)(B + v * CB + (ch - CPA) * 8);
        }
      }
#pragma unroll
      for (int k = 0; k < NLD; ++k) {
        const int q = q0 + k * nthr;
        if (q < total) ((u32x4*)tile)[q] = val[k];
      }
    }
  }
  const int tile_elems = ZW * YW * XW * CL;
  const unsigned short* wsrc = (const unsigned short*)p.w;
  if (WL) {
    constexpr int NW16 = COUT * 27 * CIN / 8;
    u32x4* wdst = (u32x4*)(tile + tile_elems);
    for (int q = threadIdx.x; q < NW16; q += nthr) wdst[q] = ((const u32x4*)p.w)[q];
    wsrc = tile + tile_elems;
  }
  __syncthreads();
  // ---- MFMA over the taps
  const int g = lane >> 4, r = lane & 15;
  const int XB = (n - 1) >> 4;
  int tb[MB];
  int64_t vout[MB];
  bool vok[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int mb = wave * MB + m;
    const int row = mb / XB, xq = mb - row * XB;
    const int zl = row / TY, yl = row - zl * TY;
    const int xl = xq * 16 + r;
    tb[m] = (zl * YW + yl) * XW + xl;
    vok[m] = (z0 + zl < n) && (y0 + yl < n);
    vout[m] = ((int64_t)(z0 + zl) * n + (y0 + yl)) * n + xl;
  }
  f32x4 acc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = {0.f, 0.f, 0.f, 0.f};
  // fragments of chunk c (32 GEMM channels): weights (A operand), tile voxels (B)
  auto fetch = [&](int c, bf16x8 (&wf)[NB], bf16x8 (&xf)[MB]) {
    const int k0 = c * 32 + g * 8;
    const int tap = k0 / CIN;
    const int ci = k0 - tap * CIN;
    const bool tap_ok = tap < 27;
    const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
    const int toff = (tz * YW + ty) * XW + tx;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      wf[nb] = tap_ok ? __builtin_bit_cast(bf16x8, *(const u32x4*)(wsrc + ((nb * 16 + r) * 27 + tap) * CIN + ci))
                      : zero8();
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      if (!tap_ok) {
        xf[m] = zero8();
      } else if (IN) {
        u32x4 v = {*(const unsigned*)(tile + (size_t)(tb[m] + toff) * 2), 0u, 0u, 0u};
        xf[m] = __builtin_bit_cast(bf16x8, v);
      } else {
        xf[m] = __builtin_bit_cast(bf16x8, *(const u32x4*)(tile + (size_t)(tb[m] + toff) * CL + ci));
      }
    }
  };
  auto mma = [&](const bf16x8 (&wf)[NB], const bf16x8 (&xf)[MB]) {
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[nb], xf[m], acc[m][nb], 0, 0, 0);
  };
  // software pipeline: the fragments of the next chunk are in flight while the
  // current chunk's MFMAs run
  bf16x8 wA[NB], xA[MB], wB[NB], xB[MB];
  fetch(0, wA, xA);
#pragma unroll
  for (int c = 0; c < KCH; c += 2) {
    if (c + 1 < KCH) fetch(c + 1, wB, xB);
    mma(wA, xA);
    if (c + 2 < KCH) fetch(c + 2, wA, xA);
    if (c + 1 < KCH) mma(wB, xB);
  }
  // ---- epilogue (as in k_conv_mfma)
  if (EPI == 0) {
    bf16* Y = p.y + (int64_t)bt * nv * COUT;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      if (!vok[m]) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + g * 4;
        float y0v = acc[m][nb][0] + p.bias[co], y1v = acc[m][nb][1] + p.bias[co + 1];
        float y2v = acc[m][nb][2] + p.bias[co + 2], y3v = acc[m][nb][3] + p.bias[co + 3];
        if (p.relu) {
          y0v = fmaxf(y0v, 0.f); y1v = fmaxf(y1v, 0.f); y2v = fmaxf(y2v, 0.f); y3v = fmaxf(y3v, 0.f);
        }
        uint2 pk;
        pk.x = (unsigned)f2bf(y0v) | ((unsigned)f2bf(y1v) << 16);
        pk.y = (unsigned)f2bf(y2v) | ((unsigned)f2bf(y3v) << 16);
        *(uint2*)(Y + vout[m] * COUT + co) = pk;
      }
    }
  } else {
    const double a = p.alpha_override > 0.0 ? p.alpha_override : p.alpha[bt];
    const float f = (float)(p.scale[bt] / a);
    Tv* zo = (Tv*)p.zout + p.off[bt];
    const int co = g * 4;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      float h = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float yj = __bfloat162float(__float2bfloat16(fmaxf(acc[m][0][j] + p.bias[co + j], 0.f)));
        h = fmaf(p.wh[co + j], yj, h);
      }
      h += __shfl_xor(h, 16, 64);
      h += __shfl_xor(h, 32, 64);
      if (g == 0 && vok[m]) {
        const int64_t v = vout[m];
        const int ox = (int)(v % n), oy = (int)((v / n) % n), oz = (int)(v / ((int64_t)n * n));
        const bool bnd = ox == 0 || oy == 0 || oz == 0 || ox == n - 1 || oy == n - 1 || oz == n - 1;
        if (!bnd) zo[v] = (Tv)(f * (h + p.bh[0]));
      }
    }
  }
}

// Stride-1 convolution with 16 output channels (the full-resolution layers).
//
// A workgroup of XB = (n - 1) / 16 waves owns output rows y0 .. y0 + MB - 1
// (x in [0, n - 1); the column x = n - 1 goes to the EDGE variant of
// k_conv_mfma) and sweeps the planes z0 .. z0 + zc - 1.  LDS holds a ring of
// input planes over rows y0 - 1 .. y0 + MB and x = -1 .. n - 1 (zero outside
// the grid), so every input plane is read once per workgroup.  Stored layers
// (IN = 0) fill the ring with direct global-to-LDS loads (16 bytes per lane,
// lane l landing at base + 16 l): a ring of four planes lets plane z + 2
// arrive while the matrix cores work on plane z.  The first layer (IN = 1)
// builds its two channels on the fly over a ring of three planes: the raw
// input values of the next two planes sit in registers (two register sets
// used in turn, so no copy waits for a load) and are converted to BF16 only
// when their plane enters the ring, so every load has a whole plane of work
// to land.
//
// The weights stay in registers for the whole launch, ordered [ty][tz, tx, ci]
// so that one K chunk of 32 belongs to a single ty: an input fragment (input
// row j, taps (tz, tx), channels) then serves the output rows j - 2 .. j with
// ty = 2 .. 0, and each wave reads MB + 2 fragments per chunk for 3 MB MFMAs.
// IN = 1 packs the 3 tx taps of one tz into each lane group: one chunk per ty.
// Tile voxels of 64 or more channels (128-byte stride) carry one 16-byte pad
// slot: that stride would put the lanes of one read on the same LDS banks.
template <int CIN, int IN>
struct RowsK {
  static constexpr int KCT = IN ? 1 : (9 * CIN + 31) / 32;  // K chunks per ty
};

template <int CL, int IN>
struct RowsTile {
  static constexpr int CPV = IN ? 1 : CL / 8;                 // 16-byte slots of data per voxel
  static constexpr int SLOTS = IN ? 1 : CPV + (CL >= 64 ? 1 : 0);
  static constexpr int CLP = IN ? 2 : SLOTS * 8;              // bf16 per tile voxel
  static constexpr int NRING = IN ? 3 : 4;
  // bytes of one ring plane (a multiple of 1 KiB, the span of one wave's load)
  __host__ __device__ static size_t plane_bytes(int mb, int n) {
    const size_t b = (size_t)(mb + 2) * (n + 1) * CLP * 2;
    return (b + 1023) & ~(size_t)1023;
  }
};

// Workgroups aimed at by the z split of the sweep launches (over the batch):
// longer sweeps for the fused last layer and the 64-channel level.
constexpr int kSweepBlocksD0 = 256;
constexpr int kSweepBlocksL2b = 384;

// The autotuned target of `layer` if set, else the default.
inline int sweep_target(const CnnState& c, int layer, int dflt) {
  return c.sweep_blocks[layer] > 0 ? c.sweep_blocks[layer] : dflt;
}

struct RowsGrid {
  int ylo = 0, yhi = 0, zlo = 0, zhi = 0;  // output rows / planes computed
  int zc = 0, ytiles = 0;
  int nedge = 0;  // trailing workgroups per instance that compute the x = n - 1 column, one plane each
  // k_conv16_ks: x ranges per row (each of xbn 16-column blocks) and the
  // columns of a ring row (16 xbn + 2: the range and one halo column each side)
  int nxs = 1, xw = 0;
};

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void gbl_void_t;

template <int CA, int CB, int MB, int IN, int EPI, typename Tv, int NPF>
__global__ void __launch_bounds__(256) k_conv16_rows(MfmaArgs p, RowsGrid q) {
  constexpr int CIN = IN ? 2 : CA + CB;
  constexpr int CL = IN ? 2 : CA + CB;
  typedef RowsTile<CL, IN> T;
  constexpr int CLP = T::CLP;
  constexpr int KCT = RowsK<CIN, IN>::KCT;
  constexpr int YW = MB + 2;
  constexpr int NR = T::NRING;
  extern __shared__ __attribute__((aligned(1024))) unsigned short ring[];
  int bxr, bt;
  xcd_remap(bxr, bt);
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  if (bxr >= (int)gridDim.x - q.nedge) {
    edge_plane<IN ? 8 : CA, CB, 16, IN, Tv, kEdgeYB>(p, bxr - ((int)gridDim.x - q.nedge), bt, (f32x4*)ring);
    return;
  }
  const int n = p.n_out;
  const int XW = q.xw;
  const int y0 = q.ylo + (bxr % q.ytiles) * MB;
  const int xh = (bxr / q.ytiles) % q.nxs;
  const int z0 = q.zlo + (bxr / q.ytiles / q.nxs) * q.zc;
  const int zend = min(q.zhi, z0 + q.zc);
  const int64_t nv = (int64_t)n * n * n;
  const int nthr = blockDim.x, nwaves = nthr >> 6;
  const int plane_elems = (int)(T::plane_bytes(MB, XW - 1) / 2);
  const int x0 = xh * 16 * (int)(blockDim.x >> 6);  // first output column of this workgroup
  const int plane_items = YW * XW * T::SLOTS;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const bf16* A = IN ? nullptr : p.a + (int64_t)bt * nv * CA;
  const bf16* B = CB ? p.b + (int64_t)bt * nv * CB : nullptr;
  const Tv* Z = IN ? (const Tv*)p.z + p.off[bt] : nullptr;
  const float* D = IN ? p.dist + (int64_t)bt * nv : nullptr;
  const float sc = IN ? (float)p.inv_s[bt] : 0.0f;
  // ---- stored layers: one wave-wide DMA per 64 slots of a plane
  auto dma_plane = [&](int gz, int slot) {
    unsigned short* pl = ring + (size_t)slot * plane_elems;
    const int nload = (plane_items + 63) >> 6;
    for (int L = wave; L < nload; L += nwaves) {
      const int it = L * 64 + lane;
      const void* src = p.zero16;
      if (it < plane_items) {
        const int vt = it / T::SLOTS, ch = it - vt * T::SLOTS;
        const int row = vt / XW, xx = vt - row * XW;
        const int gx = x0 + xx - 1, gy = y0 + row - 1;
        if (ch < T::CPV && gz >= 0 && gz < n && gy >= 0 && gy < n && gx >= 0 && gx < n) {
          const int64_t vv = ((int64_t)gz * n + gy) * n + gx;
          constexpr int CPA = CA / 8;
          src = (CB == 0 || ch < CPA) ? (const void*)(A + vv * CA + ch * 8)
                                      : (const void*)(B + vv * CB + (ch - CPA) * 8);
        }
      }
      __builtin_amdgcn_global_load_lds((gbl_void_t*)src, (lds_void_t*)(pl + L * 512), 16, 0, 0);
    }
  };
  // ---- first layer: raw values of a plane in registers, converted on entry to
  // the ring.  The loads are unconditional (voxels outside the grid read
  // voxel 0 and are zeroed by the mask at conversion), so that the compiler can
  // count the loads in flight and wait for the older plane only.
  struct RawPlane {
    Tv zv[NPF];
    float dv[NPF];
    unsigned ok;
  };
  auto load_plane = [&](int gz, RawPlane& buf) {
    buf.ok = 0u;
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int it = threadIdx.x + k * nthr;
      const int row = it / XW, xx = it - row * XW;
      const int gx = x0 + xx - 1, gy = y0 + row - 1;
      const bool ok = it < plane_items && gz >= 0 && gz < n && gy >= 0 && gy < n && gx >= 0 && gx < n;
      const int64_t vv = ok ? ((int64_t)gz * n + gy) * n + gx : 0;
      buf.zv[k] = Z[vv];
      buf.dv[k] = D[vv];
      buf.ok |= ok ? (1u << k) : 0u;
    }
  };
  auto store_plane = [&](int slot, const RawPlane& buf) {
    unsigned short* pl = ring + (size_t)slot * plane_elems;
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int it = threadIdx.x + k * nthr;
      const unsigned v = (buf.ok >> k) & 1u
                             ? (unsigned)f2bf((float)buf.zv[k] * sc) | ((unsigned)f2bf(buf.dv[k]) << 16)
                             : 0u;
      if (it < plane_items) *(unsigned*)(pl + (size_t)it * CLP) = v;
    }
  };
  // weights [16 cout][3 ty][KCT * 32], lane (g, r) holds cout r, k = c * 32 + g * 8 ..
  bf16x8 wr[3][KCT];
  {
    const unsigned short* wsrc = (const unsigned short*)p.wrows;
#pragma unroll
    for (int ty = 0; ty < 3; ++ty)
#pragma unroll
      for (int c = 0; c < KCT; ++c)
        wr[ty][c] = __builtin_bit_cast(bf16x8, *(const u32x4*)(wsrc + (r * 3 + ty) * (KCT * 32) + c * 32 + g * 8));
  }
  // per-lane tap decomposition of each chunk
  int lofs[KCT], ltz[KCT];
  bool lok[KCT];
#pragma unroll
  for (int c = 0; c < KCT; ++c) {
    if (IN) {
      ltz[c] = g;
      lok[c] = g < 3;
      lofs[c] = 0;
    } else {
      const int k = c * 32 + g * 8;
      const int pp = k / CIN, ci = k - pp * CIN;
      lok[c] = pp < 9;
      ltz[c] = lok[c] ? pp / 3 : 0;
      lofs[c] = (lok[c] ? pp % 3 : 0) * CLP + ci;
    }
  }
  const int xl = wave * 16 + r;
  // epilogue parameters, loaded before the sweep so that no load of the
  // epilogue has to wait behind the input loads in flight
  const int co = g * 4;
  float bia[4], whv[4] = {0.f, 0.f, 0.f, 0.f}, bhv = 0.f, fsc = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) bia[j] = p.bias[co + j];
  if (EPI) {
#pragma unroll
    for (int j = 0; j < 4; ++j) whv[j] = p.wh[co + j];
    bhv = p.bh[0];
    const double a = p.alpha_override > 0.0 ? p.alpha_override : p.alpha[bt];
    fsc = (float)(p.scale[bt] / a);
  }
  bf16* Y = EPI ? nullptr : p.y + (int64_t)bt * nv * 16;
  Tv* zo = EPI ? (Tv*)p.zout + p.off[bt] : nullptr;
  const int relu = p.relu;
  // first layer: qa holds the raw values of planes z0 + 1, z0 + 3, ..., qb
  // those of z0 + 2, z0 + 4, ...; plane p is requested at the end of the step
  // of plane p - 3 and enters the ring at the start of the step of plane p - 1
  RawPlane qa, qb;
  if (IN) {
    load_plane(z0 - 1, qa);
    store_plane(0, qa);
    load_plane(z0, qa);
    store_plane(1, qa);
    load_plane(z0 + 1, qa);
    load_plane(z0 + 2, qb);
  } else {
    dma_plane(z0 - 1, 0);
    dma_plane(z0, 1);
    dma_plane(z0 + 1, 2);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  auto plane_step = [&](int z, RawPlane& cur) __attribute__((always_inline)) {
    // ring slots: plane z - 1 at s0, z at s0 + 1, z + 1 at s0 + 2 (mod NR)
    const int s0 = (z - z0) % NR;
    if (IN) {
      store_plane((s0 + 2) % NR, cur);
      __syncthreads();
      // plane z + 3 into the register set just emptied (on every step, also
      // past the sweep's last plane, where the values are never used); the
      // epilogue's stores are unconditional too, so the wait before the next
      // conversion of this set leaves everything issued after it in flight
      load_plane(z + 3, cur);
    } else {
      if (z + 1 < zend) dma_plane(z + 2, (s0 + 3) % NR);
    }
    f32x4 acc[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) acc[m] = {0.f, 0.f, 0.f, 0.f};
    // software pipeline over the K chunks: the MB + 2 fragments of chunk c + 1
    // are in flight while the MFMAs of chunk c run
    auto fetch = [&](int c, bf16x8 (&xf)[MB + 2]) {
      const unsigned short* base =
          ring + (size_t)((s0 + ltz[c]) % NR) * plane_elems + (size_t)xl * CLP + lofs[c];
#pragma unroll
      for (int j = 0; j < MB + 2; ++j) {
        if (IN) {
          const unsigned short* pj = base + (size_t)j * XW * CLP;
          u32x4 v = {0u, 0u, 0u, 0u};
          if (lok[c]) {
            v.x = *(const unsigned*)(pj);
            v.y = *(const unsigned*)(pj + CLP);
            v.z = *(const unsigned*)(pj + 2 * CLP);
          }
          xf[j] = __builtin_bit_cast(bf16x8, v);
        } else {
          xf[j] = lok[c] ? __builtin_bit_cast(bf16x8, *(const u32x4*)(base + (size_t)j * XW * CLP)) : zero8();
        }
      }
    };
    auto mma = [&](int c, const bf16x8 (&xf)[MB + 2]) {
#pragma unroll
      for (int j = 0; j < MB + 2; ++j)
#pragma unroll
        for (int ty = 0; ty < 3; ++ty) {
          const int m = j - ty;
          if (m >= 0 && m < MB) acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[ty][c], xf[j], acc[m], 0, 0, 0);
        }
    };
    bf16x8 xa[MB + 2], xb[MB + 2];
    fetch(0, xa);
#pragma unroll
    for (int c = 0; c < KCT; c += 2) {
      if (c + 1 < KCT) fetch(c + 1, xb);
      __builtin_amdgcn_sched_barrier(0);
      mma(c, xa);
      __builtin_amdgcn_sched_barrier(0);
      if (c + 2 < KCT) fetch(c + 2, xa);
      __builtin_amdgcn_sched_barrier(0);
      if (c + 1 < KCT) mma(c + 1, xb);
      __builtin_amdgcn_sched_barrier(0);
    }
    // epilogue for plane z
    if (EPI == 0) {
      // rows past the grid repeat the store of the last row inside it (the
      // same value to the same place), so that every step issues MB stores
      uint2 pkl = {0u, 0u};
      int64_t vl = 0;
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        const int y = y0 + m;
        const int64_t v = ((int64_t)z * n + y) * n + x0 + xl;
        float y0v = acc[m][0] + bia[0], y1v = acc[m][1] + bia[1];
        float y2v = acc[m][2] + bia[2], y3v = acc[m][3] + bia[3];
        if (relu) {
          y0v = fmaxf(y0v, 0.f); y1v = fmaxf(y1v, 0.f); y2v = fmaxf(y2v, 0.f); y3v = fmaxf(y3v, 0.f);
        }
        uint2 pk;
        pk.x = (unsigned)f2bf(y0v) | ((unsigned)f2bf(y1v) << 16);
        pk.y = (unsigned)f2bf(y2v) | ((unsigned)f2bf(y3v) << 16);
        const bool in = m == 0 || y < q.yhi;  // row y0 is always inside
        pkl.x = in ? pk.x : pkl.x;
        pkl.y = in ? pk.y : pkl.y;
        vl = in ? v : vl;
        *(uint2*)(Y + vl * 16 + co) = pkl;
      }
    } else {
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        float h = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float yj = __bfloat162float(__float2bfloat16(fmaxf(acc[m][j] + bia[j], 0.f)));
          h = fmaf(whv[j], yj, h);
        }
        h += __shfl_xor(h, 16, 64);
        h += __shfl_xor(h, 32, 64);
        const int y = y0 + m;
        // Dirichlet nodes keep the value set before the network runs
        if (g == 0 && y < q.yhi && y > 0 && y < n - 1 && x0 + xl > 0 && z > 0 && z < n - 1)
          zo[((int64_t)z * n + y) * n + x0 + xl] = (Tv)(fsc * (h + bhv));
      }
    }
    if (!IN) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };
  if (IN) {
    // the first step, then pairs of steps: every path into a step has issued
    // the same loads and stores since that step's register set was requested,
    // so the compiler's wait for the set leaves the newer ones in flight
    // (the grid gives every workgroup at least one plane: z0 < zend)
    int z = z0;
    plane_step(z++, qa);
    for (; z + 1 < zend; z += 2) {
      plane_step(z, qb);
      plane_step(z + 1, qa);
    }
    if (z < zend) plane_step(z, qb);
  } else {
    for (int z = z0; z < zend; ++z) plane_step(z, qa);
  }
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations
// and meets the other waves, without the wait for outstanding global memory
// operations that __syncthreads() implies (the ring loads in flight).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Two-waves-per-SIMD form of the 16-channel stride-1 layer for stored inputs:
// 2 XB waves per workgroup.  Waves w and w + XB share x block w and either
// split the output rows (KS = 0: rows [0, MB) and [MB, 2 MB) of the tile) or
// the K chunks (KS = 1: the upper wave runs chunks [0, KH), the lower one
// [KH, KCT) and the epilogue, the partial sums crossing over through a
// double-buffered LDS area).  The ring holds five planes and the loads run
// two planes ahead: plane z + 3 is requested while plane z is computed and the
// end-of-plane wait lets that newest batch stay in flight (vector memory
// operations of a wave complete in issue order).  Every wave issues exactly
// NLW ring loads per plane (surplus lanes and loads fetch the zero block), and
// their source offsets are computed once.
template <int CA, int CB, int MB, int KS, int EPI, typename Tv, int NLW>
__global__ void __launch_bounds__(512) k_conv16_ks(MfmaArgs p, RowsGrid q) {
  constexpr int CIN = CA + CB;
  typedef RowsTile<CIN, 0> T;
  constexpr int CLP = T::CLP;
  // 32-channel tile voxels (64-byte stride) are read 16 voxels by 16 lanes
  // for one 16-byte slot: without a permutation the lanes of a read collide
  // on LDS banks.  Slot s of tile voxel v is stored at position s ^ swz(v).
  constexpr bool SWZ = T::SLOTS == 4 && T::CPV == 4;
  auto swz = [](int v) { return (v >> 2) & 3; };
  constexpr int KCT = RowsK<CIN, 0>::KCT;
  constexpr int KH = KS ? (KCT + 1) / 2 : KCT;   // chunk slots per wave
  constexpr int TYR = KS ? MB : 2 * MB;          // output rows per workgroup
  constexpr int YW = TYR + 2;
  constexpr int NR = 5;
  constexpr int CPA = CA / 8;
  static_assert(NLW <= 4, "the end-of-plane wait covers at most 4 loads");
  extern __shared__ __attribute__((aligned(1024))) unsigned short ring[];
  int bxr, bt;
  xcd_remap(bxr, bt);
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  if (!EPI && bxr >= (int)gridDim.x - q.nedge) {
    edge_plane<CA, CB, 16, 0, Tv, kEdgeYB>(p, bxr - ((int)gridDim.x - q.nedge), bt, (f32x4*)ring);
    return;
  }
  const int n = p.n_out;
  const int XW = q.xw;
  const int y0 = q.ylo + (bxr % q.ytiles) * TYR;
  const int xh = (bxr / q.ytiles) % q.nxs;
  const int z0 = q.zlo + (bxr / q.ytiles / q.nxs) * q.zc;
  const int zend = min(q.zhi, z0 + q.zc);
  const int64_t nn = (int64_t)n * n, nv = nn * n;
  const int nwaves = blockDim.x >> 6, xbn = nwaves >> 1;
  const int x0 = xh * 16 * xbn;  // first output column of this workgroup
  const int plane_elems = (int)(T::plane_bytes(TYR, XW - 1) / 2);
  const int plane_items = YW * XW * T::SLOTS;
  const int nload = (plane_items + 63) >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const int upper = wave >= xbn, xq = upper ? wave - xbn : wave;
  const int rb0 = KS ? 0 : upper * MB;           // first tile row of this wave's outputs
  // LDS after the ring: partial sums [2][xbn][MB][64] x float4 (KS)
  float* red = (float*)(ring + (size_t)NR * plane_elems);
  // ring loads of this wave per plane (wave-uniform, at most NLW)
  const int nlw = min(NLW, (nload - wave + nwaves - 1) / nwaves);
  // wait until at most nlw vector memory operations of this wave are outstanding
  auto wait_vm_newest = [&]() {
    switch (nlw) {
      case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
      case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
      case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
      case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
      default: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
    }
  };
  const bf16* A = p.a + (int64_t)bt * nv * CA;
  const bf16* B = CB ? p.b + (int64_t)bt * nv * CB : nullptr;
  // ring-load sources: byte offset from A (or to the zero block) and bytes per plane (0 for zero slots)
  const char* Ab = (const char*)A;
  const int64_t zero_off = (const char*)p.zero16 - Ab;
  const int64_t b_off = CB ? (const char*)B - Ab : 0;
  int64_t doff[NLW];
  int dstr[NLW];
#pragma unroll
  for (int k = 0; k < NLW; ++k) {
    const int L = wave + k * nwaves;
    const int it = L * 64 + lane;
    int64_t o = zero_off;
    int st = 0;
    if (L < nload && it < plane_items) {
      const int vt = it / T::SLOTS, chp = it - vt * T::SLOTS;
      const int ch = SWZ ? chp ^ swz(vt) : chp;  // the channel slot stored at this position
      const int row = vt / XW, xx = vt - row * XW;
      const int gx = x0 + xx - 1, gy = y0 + row - 1;
      if (ch < T::CPV && gy >= 0 && gy < n && gx >= 0 && gx < n) {
        const int64_t vv = (int64_t)gy * n + gx;
        if (CB == 0 || ch < CPA) {
          o = (vv * CA + ch * 8) * 2;
          st = (int)(nn * CA * 2);
        } else {
          o = b_off + (vv * CB + (ch - CPA) * 8) * 2;
          st = (int)(nn * CB * 2);
        }
      }
    }
    doff[k] = o;
    dstr[k] = st;
  }
  auto dma_plane = [&](int gz, int slot) {
    unsigned short* pl = ring + (size_t)slot * plane_elems;
    const bool zok = gz >= 0 && gz < n;
#pragma unroll
    for (int k = 0; k < NLW; ++k) {
      const int L = wave + k * nwaves;
      if (L < nload) {
        const int64_t o = zok ? doff[k] + (int64_t)gz * dstr[k] : zero_off;
        __builtin_amdgcn_global_load_lds((gbl_void_t*)(Ab + o), (lds_void_t*)(pl + L * 512), 16, 0, 0);
      }
    }
  };
  // this wave's K chunks: all (KS = 0); upper [0, KH), lower [KH, KCT) (KS = 1)
  const int cb = (KS && !upper) ? KH : 0;
  bf16x8 wr[3][KH];
  int lofs[KH], ltz[KH];
  bool lok[KH];
  {
    const unsigned short* wsrc = (const unsigned short*)p.wrows;
#pragma unroll
    for (int i = 0; i < KH; ++i) {
      const int c = cb + i;
      const bool cin = c < KCT;
#pragma unroll
      for (int ty = 0; ty < 3; ++ty)
        wr[ty][i] = cin ? __builtin_bit_cast(bf16x8, *(const u32x4*)(wsrc + (r * 3 + ty) * (KCT * 32) + c * 32 + g * 8))
                        : zero8();
      const int k = c * 32 + g * 8;
      const int pp = k / CIN, ci = k - pp * CIN;
      lok[i] = cin && pp < 9;
      ltz[i] = lok[i] ? pp / 3 : 0;
      lofs[i] = (lok[i] ? pp % 3 : 0) * CLP + ci;
    }
  }
  const int xl = xq * 16 + r;
  // epilogue parameters, loaded before the sweep so that no load of the
  // epilogue has to wait behind the ring loads in flight
  const int co = g * 4;
  float bia[4], whv[4] = {0.f, 0.f, 0.f, 0.f}, bhv = 0.f, fsc = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) bia[j] = p.bias[co + j];
  if (EPI) {
#pragma unroll
    for (int j = 0; j < 4; ++j) whv[j] = p.wh[co + j];
    bhv = p.bh[0];
    const double a = p.alpha_override > 0.0 ? p.alpha_override : p.alpha[bt];
    fsc = (float)(p.scale[bt] / a);
  }
  bf16* Y = EPI ? nullptr : p.y + (int64_t)bt * nv * 16;
  Tv* zo = EPI ? (Tv*)p.zout + p.off[bt] : nullptr;
  const int relu = p.relu;
  dma_plane(z0 - 1, 0);
  dma_plane(z0, 1);
  dma_plane(z0 + 1, 2);
  dma_plane(z0 + 2, 3);
  wait_vm_newest();
  lds_barrier();
  for (int z = z0; z < zend; ++z) {
    const int s0 = (z - z0) % NR;
    const int par = (z - z0) & 1;
    // plane z + 3 into the slot of plane z - 2 (read before the previous barrier)
    dma_plane(z + 3, (s0 + 4) % NR);
    f32x4 acc[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) acc[m] = {0.f, 0.f, 0.f, 0.f};
    auto fetch = [&](int i, bf16x8 (&xf)[MB + 2]) {
      if constexpr (SWZ) {
        // lofs = tx * CLP + slot * 8: tile voxel (rb0 + j) XW + xl + tx, slot permuted
        const unsigned short* pl = ring + (size_t)((s0 + ltz[i]) % NR) * plane_elems;
        const int tx = lofs[i] / CLP, sl = (lofs[i] - tx * CLP) >> 3;
#pragma unroll
        for (int j = 0; j < MB + 2; ++j) {
          const int v = (rb0 + j) * XW + xl + tx;
          xf[j] = lok[i] ? __builtin_bit_cast(bf16x8, *(const u32x4*)(pl + (size_t)v * CLP + ((sl ^ swz(v)) << 3)))
                         : zero8();
        }
      } else {
        const unsigned short* base = ring + (size_t)((s0 + ltz[i]) % NR) * plane_elems +
                                     ((size_t)rb0 * XW + xl) * CLP + lofs[i];
#pragma unroll
        for (int j = 0; j < MB + 2; ++j)
          xf[j] = lok[i] ? __builtin_bit_cast(bf16x8, *(const u32x4*)(base + (size_t)j * XW * CLP)) : zero8();
      }
    };
    auto mma = [&](int i, const bf16x8 (&xf)[MB + 2]) {
#pragma unroll
      for (int j = 0; j < MB + 2; ++j)
#pragma unroll
        for (int ty = 0; ty < 3; ++ty) {
          const int m = j - ty;
          if (m >= 0 && m < MB) acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[ty][i], xf[j], acc[m], 0, 0, 0);
        }
    };
    auto run = [&](auto nchc) {
      constexpr int NCH = decltype(nchc)::value;
      bf16x8 xa[MB + 2], xb[MB + 2];
      fetch(0, xa);
#pragma unroll
      for (int i = 0; i < NCH; i += 2) {
        if (i + 1 < NCH) fetch(i + 1, xb);
        __builtin_amdgcn_sched_barrier(0);
        mma(i, xa);
        __builtin_amdgcn_sched_barrier(0);
        if (i + 2 < NCH) fetch(i + 2, xa);
        __builtin_amdgcn_sched_barrier(0);
        if (i + 1 < NCH) mma(i + 1, xb);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    if (!KS || upper) run(std::integral_constant<int, KH>{});
    else run(std::integral_constant<int, KCT - KH>{});
    f32x4* rbuf = (f32x4*)red + ((size_t)(par * xbn + xq) * MB) * 64 + lane;
    if (KS && upper) {
#pragma unroll
      for (int m = 0; m < MB; ++m) rbuf[m * 64] = acc[m];
    }
    // plane z + 2 (and everything older) has landed; z + 3 may still be in flight
    wait_vm_newest();
    lds_barrier();
    if (!KS || !upper) {
      if (KS) {
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          const f32x4 o = rbuf[m * 64];
          acc[m] += o;
        }
      }
      if (EPI == 0) {
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          const int y = y0 + rb0 + m;
          if (y >= q.yhi) continue;
          const int64_t v = ((int64_t)z * n + y) * n + x0 + xl;
          float y0v = acc[m][0] + bia[0], y1v = acc[m][1] + bia[1];
          float y2v = acc[m][2] + bia[2], y3v = acc[m][3] + bia[3];
          if (relu) {
            y0v = fmaxf(y0v, 0.f); y1v = fmaxf(y1v, 0.f); y2v = fmaxf(y2v, 0.f); y3v = fmaxf(y3v, 0.f);
          }
          uint2 pk;
          pk.x = (unsigned)f2bf(y0v) | ((unsigned)f2bf(y1v) << 16);
          pk.y = (unsigned)f2bf(y2v) | ((unsigned)f2bf(y3v) << 16);
          *(uint2*)(Y + v * 16 + co) = pk;
        }
      } else {
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          float h = 0.f;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float yj = __bfloat162float(__float2bfloat16(fmaxf(acc[m][j] + bia[j], 0.f)));
            h = fmaf(whv[j], yj, h);
          }
          h += __shfl_xor(h, 16, 64);
          h += __shfl_xor(h, 32, 64);
          const int y = y0 + rb0 + m;
          // Dirichlet nodes keep the value set before the network runs
          if (g == 0 && y < q.yhi && y > 0 && y < n - 1 && x0 + xl > 0 && z > 0 && z < n - 1)
            zo[((int64_t)z * n + y) * n + x0 + xl] = (Tv)(fsc * (h + bhv));
        }
      }
    }
  }
  // drain the loads still in flight before the workgroup's LDS is released
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// The last full-resolution layer inside the solver (D0: 32 stacked input
// channels [U0 | skip], 16 outputs, ReLU, then the 1x1 head and the unscaling
// z0 = ||b0|| / alpha * U), as a z sweep that keeps three output planes in
// registers.  Input plane zi feeds output planes zi + 1, zi, zi - 1 (taps
// tz = 0, 1, 2), so each 16-voxel fragment read from LDS serves up to nine
// MFMAs (three tz x three ty) instead of three, and only the plane being read
// and the two being loaded sit in LDS.  After input plane zi, output plane
// zi - 1 is complete: its epilogue runs and its accumulators start plane
// zi + 2.  A workgroup of 2 XB waves owns rows y0 .. y0 + 2 MB - 1 (wave w:
// x block w % XB, rows (w / XB) MB ..) of the planes z0 .. z0 + zc - 1;
// the ring holds rows y0 - 1 .. y0 + 2 MB and x = x0 - 1 .. x0 + 16 XB,
// filled by direct global-to-LDS loads two planes ahead.  All 27 taps' weight
// fragments stay in registers, ordered [tz][ty][tx].  Per output the taps
// are summed in the order (tz, tx, ty), one accumulator: the order of a
// single-wave k_conv16_ks chunk loop.
template <int MB, typename Tv, int NLW>
__global__ void __launch_bounds__(512) k_conv16_zb(MfmaArgs p, RowsGrid q) {
  constexpr int CA = 16, CB = 16, CIN = CA + CB;
  typedef RowsTile<CIN, 0> T;
  constexpr int CLP = T::CLP;
  static_assert(T::SLOTS == 4 && T::CPV == 4, "32-channel tile voxels");
  constexpr int TYR = 2 * MB, YW = TYR + 2, NR = 3;
  constexpr int CPA = CA / 8;
  static_assert(NLW <= 8, "the end-of-plane wait covers at most 8 loads");
  auto swz = [](int v) { return (v >> 2) & 3; };
  extern __shared__ __attribute__((aligned(1024))) unsigned short ring[];
  int bxr, bt;
  xcd_remap(bxr, bt);
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  const int n = p.n_out;
  const int XW = q.xw;
  const int y0 = q.ylo + (bxr % q.ytiles) * TYR;
  const int xh = (bxr / q.ytiles) % q.nxs;
  const int z0 = q.zlo + (bxr / q.ytiles / q.nxs) * q.zc;
  const int zend = min(q.zhi, z0 + q.zc);
  const int64_t nn = (int64_t)n * n, nv = nn * n;
  const int nwaves = blockDim.x >> 6, xbn = nwaves >> 1;
  const int x0 = xh * 16 * xbn;
  const int plane_elems = (int)(T::plane_bytes(TYR, XW - 1) / 2);
  const int plane_items = YW * XW * T::SLOTS;
  const int nload = (plane_items + 63) >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const int hr = wave >= xbn, xq = hr ? wave - xbn : wave;
  const int rb0 = hr * MB;
  const int nlw = min(NLW, (nload - wave + nwaves - 1) / nwaves);
  auto wait_vm_newest = [&]() {
    switch (nlw) {
      case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
      case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
      case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
      case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
      case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
      case 5: asm volatile("s_waitcnt vmcnt(5)" ::: "memory"); break;
      case 6: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
      case 7: asm volatile("s_waitcnt vmcnt(7)" ::: "memory"); break;
      default: asm volatile("s_waitcnt vmcnt(8)" ::: "memory"); break;
    }
  };
  const bf16* A = p.a + (int64_t)bt * nv * CA;
  const bf16* B = p.b + (int64_t)bt * nv * CB;
  const char* Ab = (const char*)A;
  const int64_t zero_off = (const char*)p.zero16 - Ab;
  const int64_t b_off = (const char*)B - Ab;
  int64_t doff[NLW];
  int dstr[NLW];
#pragma unroll
  for (int k = 0; k < NLW; ++k) {
    const int L = wave + k * nwaves;
    const int it = L * 64 + lane;
    int64_t o = zero_off;
    int st = 0;
    if (L < nload && it < plane_items) {
      const int vt = it >> 2, chp = it & 3;
      const int ch = chp ^ swz(vt);  // the channel slot stored at this position
      const int row = vt / XW, xx = vt - row * XW;
      const int gx = x0 + xx - 1, gy = y0 + row - 1;
      if (gy >= 0 && gy < n && gx >= 0 && gx < n) {
        const int64_t vv = (int64_t)gy * n + gx;
        if (ch < CPA) {
          o = (vv * CA + ch * 8) * 2;
          st = (int)(nn * CA * 2);
        } else {
          o = b_off + (vv * CB + (ch - CPA) * 8) * 2;
          st = (int)(nn * CB * 2);
        }
      }
    }
    doff[k] = o;
    dstr[k] = st;
  }
  auto dma_plane = [&](int gz, int slot) {
    unsigned short* pl = ring + (size_t)slot * plane_elems;
    const bool zok = gz >= 0 && gz < n;
#pragma unroll
    for (int k = 0; k < NLW; ++k) {
      const int L = wave + k * nwaves;
      if (L < nload) {
        const int64_t o = zok ? doff[k] + (int64_t)gz * dstr[k] : zero_off;
        __builtin_amdgcn_global_load_lds((gbl_void_t*)(Ab + o), (lds_void_t*)(pl + L * 512), 16, 0, 0);
      }
    }
  };
  // weight fragments w[tz][ty][tx]: rows [16 cout][3 ty][9 (tz, tx) x 32 ci]
  bf16x8 wr[3][3][3];
  {
    const unsigned short* wsrc = (const unsigned short*)p.wrows;
#pragma unroll
    for (int tz = 0; tz < 3; ++tz)
#pragma unroll
      for (int ty = 0; ty < 3; ++ty)
#pragma unroll
        for (int tx = 0; tx < 3; ++tx)
          wr[tz][ty][tx] =
              __builtin_bit_cast(bf16x8, *(const u32x4*)(wsrc + (r * 3 + ty) * (9 * 32) + (tz * 3 + tx) * 32 + g * 8));
  }
  const int xl = xq * 16 + r;
  const int co = g * 4;
  float bia[4], whv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    bia[j] = p.bias[co + j];
    whv[j] = p.wh[co + j];
  }
  const float bhv = p.bh[0];
  const double aa = p.alpha_override > 0.0 ? p.alpha_override : p.alpha[bt];
  const float fsc = (float)(p.scale[bt] / aa);
  Tv* zo_ = (Tv*)p.zout + p.off[bt];
  // tile voxel of row j and tap tx for this lane, and its slot position
  f32x4 acc[3][MB];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int m = 0; m < MB; ++m) acc[a][m] = {0.f, 0.f, 0.f, 0.f};
  const int zi0 = z0 - 1, zi1 = zend;  // input planes zi0 .. zi1
  dma_plane(zi0, 0);
  dma_plane(zi0 + 1, 1);
  wait_vm_newest();
  lds_barrier();
  // one input plane: its fragments feed the accumulators of the planes
  // zi + 1 (slot A0, tz = 0), zi (A1, tz = 1), zi - 1 (A2, tz = 2); then the
  // epilogue of plane zi - 1 and its slot cleared for plane zi + 2
  auto step = [&](int zi, int s, auto a0c, auto a1c, auto a2c) {
    constexpr int A0 = decltype(a0c)::value, A1 = decltype(a1c)::value, A2 = decltype(a2c)::value;
    const bool more = zi + 2 <= zi1;
    if (more) dma_plane(zi + 2, (s + 2) % NR);
    const unsigned short* pl = ring + (size_t)s * plane_elems;
#pragma unroll
    for (int tx = 0; tx < 3; ++tx) {
      bf16x8 xf[MB + 2];
#pragma unroll
      for (int j = 0; j < MB + 2; ++j) {
        const int v = (rb0 + j) * XW + xl + tx;
        xf[j] = __builtin_bit_cast(bf16x8, *(const u32x4*)(pl + (size_t)v * CLP + ((g ^ swz(v)) << 3)));
      }
#pragma unroll
      for (int j = 0; j < MB + 2; ++j)
#pragma unroll
        for (int ty = 0; ty < 3; ++ty) {
          const int m = j - ty;
          if (m >= 0 && m < MB) {
            acc[A0][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[0][ty][tx], xf[j], acc[A0][m], 0, 0, 0);
            acc[A1][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[1][ty][tx], xf[j], acc[A1][m], 0, 0, 0);
            acc[A2][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[2][ty][tx], xf[j], acc[A2][m], 0, 0, 0);
          }
        }
    }
    const int zo = zi - 1;
    if (zo >= z0 && zo < zend) {
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        float h = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float yj = __bfloat162float(__float2bfloat16(fmaxf(acc[A2][m][j] + bia[j], 0.f)));
          h = fmaf(whv[j], yj, h);
        }
        h += __shfl_xor(h, 16, 64);
        h += __shfl_xor(h, 32, 64);
        const int y = y0 + rb0 + m;
        // Dirichlet nodes keep the value set before the network runs
        if (g == 0 && y < q.yhi && y > 0 && y < n - 1 && x0 + xl > 0 && zo > 0 && zo < n - 1)
          zo_[((int64_t)zo * n + y) * n + x0 + xl] = (Tv)(fsc * (h + bhv));
      }
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) acc[A2][m] = {0.f, 0.f, 0.f, 0.f};
    // plane zi + 1 has landed (zi + 2 may still be in flight: its loads and
    // the epilogue stores are this wave's newest memory operations, and they
    // complete in issue order); every wave is done with plane zi before the
    // next step's loads overwrite its slot
    if (more) wait_vm_newest();
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    lds_barrier();
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  // accumulator slot of output plane zo: (zo - zi0 + 2) % 3, so that input
  // plane zi = zi0 + 3 k + ph uses slots (ph + 0, 1, 2) % 3 for zi + 1, zi, zi - 1
  for (int zi = zi0; zi <= zi1; zi += 3) {
    const int s = (zi - zi0) % NR;  // ring slot of plane zi: (zi - zi0) % 3
    step(zi, s, I0{}, I2{}, I1{});
    if (zi + 1 <= zi1) step(zi + 1, (s + 1) % NR, I1{}, I0{}, I2{});
    if (zi + 2 <= zi1) step(zi + 2, (s + 2) % NR, I2{}, I1{}, I0{});
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Launch of k_conv16_zb over the interior planes and rows (x < n - 1); false
// when the grid or the LDS does not fit (then the caller keeps k_conv16_ks).
template <int MB, typename Tv>
bool launch_zb16(const MfmaArgs& a, int batch, hipStream_t stream, int target, int xbmax) {
  constexpr int NLW = 8;
  constexpr int TYR = 2 * MB;
  typedef RowsTile<32, 0> T;
  const int n = a.n_out;
  const int xb = (n - 1) / 16;
  int xbw = std::min(std::max(xb, 1), xbmax > 0 ? std::min(xbmax, 4) : 4);
  while (xb % xbw) --xbw;
  const int nxs = xb / xbw;
  const int xw = 16 * xbw + 2;
  const size_t lds = 3 * T::plane_bytes(TYR, xw - 1);
  const int nload = ((TYR + 2) * xw * T::SLOTS + 63) / 64;
  if (!((n - 1) % 16 == 0 && xb >= 1 && lds <= 160 * 1024 && a.zero16 && nload <= NLW * 2 * xbw)) return false;
  RowsGrid q;
  q.ylo = q.zlo = 1;
  q.yhi = q.zhi = n - 1;
  q.ytiles = (q.yhi - q.ylo + TYR - 1) / TYR;
  q.nxs = nxs;
  q.xw = xw;
  const int planes = q.zhi - q.zlo;
  int nz = (target + q.ytiles * nxs * batch - 1) / (q.ytiles * nxs * batch);
  nz = std::max(1, std::min(nz, planes));
  q.zc = (planes + nz - 1) / nz;
  nz = (planes + q.zc - 1) / q.zc;
  q.nedge = 0;
  auto kern = k_conv16_zb<MB, Tv, NLW>;
  if (lds > 65536) hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(kern, dim3((unsigned)(q.ytiles * nxs * nz), 1, batch), dim3(2 * xbw * 64), lds, stream, a, q);
  return true;
}

// Stride-1 convolution with COUT = 32 or 64 (the coarse levels), z-sweep with
// a three-plane LDS ring over rows y0 - 1 .. y0 + MB (x = -1 .. n - 1, zero
// outside), the next plane staged in registers while the current one is
// computed.  XB * KG waves: wave (xq, kg) owns x block xq and the K chunks
// [kg KPG, (kg + 1) KPG) for all NB = COUT / 16 output blocks, with those
// weights in registers; as in the 16-channel kernels one input fragment (row
// j) serves the output rows j - 2 .. j (chunk slots past the K range are
// skipped).  The KG partial sums meet in LDS and each wave finishes (sum,
// bias, ReLU, store) every KG-th output fragment.
template <int CA, int CB, int COUT, int MB, int KG, int NPF>
__global__ void __launch_bounds__(512) k_convw(MfmaArgs p, RowsGrid q) {
  constexpr int CIN = CA + CB;
  typedef RowsTile<CIN, 0> T;
  constexpr int CLP = T::CLP;
  constexpr int CPV = T::CPV;
  constexpr int NB = COUT / 16;
  constexpr int KCT = RowsK<CIN, 0>::KCT;
  constexpr int KPG = (KCT + KG - 1) / KG;   // chunk slots per wave
  // chunks of the one group with fewer than KPG but more than none (0: no such group)
  constexpr int KREM = KCT % KPG;
  constexpr int YW = MB + 2;
  constexpr int NF = MB * NB;                // output fragments per x block
  constexpr int CPA = CA / 8;
  extern __shared__ __attribute__((aligned(1024))) unsigned short ring[];
  int bxr, bt;
  xcd_remap(bxr, bt);
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  if (bxr >= (int)gridDim.x - q.nedge) {
    edge_plane<CA, CB, COUT, 0, float, kEdgeYB>(p, bxr - ((int)gridDim.x - q.nedge), bt, (f32x4*)ring);
    return;
  }
  const int n = p.n_out;
  const int XW = q.xw;
  const int y0 = q.ylo + (bxr % q.ytiles) * MB;
  const int xh = (bxr / q.ytiles) % q.nxs;
  const int z0 = q.zlo + (bxr / q.ytiles / q.nxs) * q.zc;
  const int zend = min(q.zhi, z0 + q.zc);
  const int64_t nv = (int64_t)n * n * n;
  const int nthr = blockDim.x;
  const int xbn = (XW - 2) / 16;  // x blocks of this workgroup
  const int x0 = xh * 16 * xbn;   // its first output column
  const int plane_elems = (int)(T::plane_bytes(MB, XW - 1) / 2);
  const int plane_items = YW * XW * CPV;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const int xq = wave % xbn, kg = wave / xbn;
  f32x4* red = (f32x4*)(ring + (size_t)3 * plane_elems);  // [KG][xbn][NF][64]
  // the bias in LDS: a global load in the epilogue would wait for the plane
  // loads in flight
  float* sbias = (float*)(red + (size_t)KG * xbn * NF * 64);
  for (int i = threadIdx.x; i < COUT; i += nthr) sbias[i] = p.bias[i];
  const bf16* A = p.a + (int64_t)bt * nv * CA;
  const bf16* B = CB ? p.b + (int64_t)bt * nv * CB : nullptr;
  auto load_plane = [&](int gz, u32x4 (&buf)[NPF]) {
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int it = threadIdx.x + k * nthr;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (it < plane_items) {
        const int vt = it / CPV, ch = it - vt * CPV;
        const int row = vt / XW, xx = vt - row * XW;
        const int gx = x0 + xx - 1, gy = y0 + row - 1;
        if (gz >= 0 && gz < n && gy >= 0 && gy < n && gx >= 0 && gx < n) {
          const int64_t vv = ((int64_t)gz * n + gy) * n + gx;
          v = (CB == 0 || ch < CPA) ? *(const u32x4*)(A + vv * CA + ch * 8)
                                    : *(const u32x4*)(B + vv * CB + (ch - CPA) * 8);
        }
      }
      buf[k] = v;
    }
  };
  auto store_plane = [&](int slot, const u32x4 (&buf)[NPF]) {
    unsigned short* pl = ring + (size_t)slot * plane_elems;
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int it = threadIdx.x + k * nthr;
      if (it < plane_items) {
        const int vt = it / CPV, ch = it - vt * CPV;
        *(u32x4*)(pl + (size_t)vt * CLP + ch * 8) = buf[k];
      }
    }
  };
  // weights of this wave's chunks, [16 cout][3 ty][KCT * 32] per output block
  const int cb = kg * KPG;
  bf16x8 wr[3][KPG][NB];
  int lofs[KPG], ltz[KPG];
  bool lok[KPG];
  {
    const unsigned short* wsrc = (const unsigned short*)p.wrows;
#pragma unroll
    for (int i = 0; i < KPG; ++i) {
      const int c = cb + i;
      const bool cin = c < KCT;
#pragma unroll
      for (int ty = 0; ty < 3; ++ty)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          wr[ty][i][nb] =
              cin ? __builtin_bit_cast(bf16x8, *(const u32x4*)(wsrc + ((nb * 16 + r) * 3 + ty) * (KCT * 32) + c * 32 + g * 8))
                  : zero8();
      const int k = c * 32 + g * 8;
      const int pp = k / CIN, ci = k - pp * CIN;
      lok[i] = cin && pp < 9;
      ltz[i] = lok[i] ? pp / 3 : 0;
      lofs[i] = (lok[i] ? pp % 3 : 0) * CLP + ci;
    }
  }
  const int nch = max(0, min(KPG, KCT - cb));  // chunks of this wave (wave-uniform)
  const int xl = xq * 16 + r;
  u32x4 pf[NPF];
  load_plane(z0 - 1, pf);
  store_plane(0, pf);
  load_plane(z0, pf);
  store_plane(1, pf);
  load_plane(z0 + 1, pf);
  for (int z = z0; z < zend; ++z) {
    const int s0 = (z - z0) % 3;
    store_plane((s0 + 2) % 3, pf);
    __syncthreads();
    if (z + 1 < zend) load_plane(z + 2, pf);
    f32x4 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[m][nb] = {0.f, 0.f, 0.f, 0.f};
    auto fetch = [&](int i, bf16x8 (&xf)[MB + 2]) {
      const unsigned short* base = ring + (size_t)((s0 + ltz[i]) % 3) * plane_elems + (size_t)xl * CLP + lofs[i];
#pragma unroll
      for (int j = 0; j < MB + 2; ++j)
        xf[j] = lok[i] ? __builtin_bit_cast(bf16x8, *(const u32x4*)(base + (size_t)j * XW * CLP)) : zero8();
    };
    auto mma = [&](int i, const bf16x8 (&xf)[MB + 2]) {
#pragma unroll
      for (int j = 0; j < MB + 2; ++j)
#pragma unroll
        for (int ty = 0; ty < 3; ++ty) {
          const int m = j - ty;
          if (m >= 0 && m < MB) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[ty][i][nb], xf[j], acc[m][nb], 0, 0, 0);
          }
        }
    };
    // the chunk loop with a compile-time count (a branch per chunk would make
    // each MFMA wait for the fragment loads issued after its own)
    auto run = [&](auto nchc) {
      constexpr int NCH = decltype(nchc)::value;
      bf16x8 xa[MB + 2], xb[MB + 2];
      fetch(0, xa);
#pragma unroll
      for (int i = 0; i < NCH; i += 2) {
        if (i + 1 < NCH) fetch(i + 1, xb);
        __builtin_amdgcn_sched_barrier(0);
        mma(i, xa);
        __builtin_amdgcn_sched_barrier(0);
        if (i + 2 < NCH) fetch(i + 2, xa);
        __builtin_amdgcn_sched_barrier(0);
        if (i + 1 < NCH) mma(i + 1, xb);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    if (nch == KPG) run(std::integral_constant<int, KPG>{});
    else if constexpr (KREM > 0) {
      if (nch == KREM) run(std::integral_constant<int, KREM>{});
    }
    // partial sums to LDS: red[kg][xq][f][lane], f = m * NB + nb
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        red[((size_t)(kg * xbn + xq) * NF + m * NB + nb) * 64 + lane] = acc[m][nb];
    __syncthreads();
    // this wave finishes fragments f = kg, kg + KG, ... of x block xq
    bf16* Y = p.y + (int64_t)bt * nv * COUT;
    for (int f = kg; f < NF; f += KG) {
      f32x4 sum = red[((size_t)xq * NF + f) * 64 + lane];
      for (int k2 = 1; k2 < KG; ++k2) {
        const f32x4 o = red[((size_t)(k2 * xbn + xq) * NF + f) * 64 + lane];
        sum += o;
      }
      const int m = f / NB, nb = f - m * NB;
      const int y = y0 + m;
      if (y >= q.yhi) continue;
      const int co = nb * 16 + g * 4;
      float y0v = sum[0] + sbias[co], y1v = sum[1] + sbias[co + 1];
      float y2v = sum[2] + sbias[co + 2], y3v = sum[3] + sbias[co + 3];
      if (p.relu) {
        y0v = fmaxf(y0v, 0.f); y1v = fmaxf(y1v, 0.f); y2v = fmaxf(y2v, 0.f); y3v = fmaxf(y3v, 0.f);
      }
      uint2 pk;
      pk.x = (unsigned)f2bf(y0v) | ((unsigned)f2bf(y1v) << 16);
      pk.y = (unsigned)f2bf(y2v) | ((unsigned)f2bf(y3v) << 16);
      const int64_t v = ((int64_t)z * n + y) * n + x0 + xl;
      *(uint2*)(Y + v * COUT + co) = pk;
    }
  }
}

// Transposed stride-2 convolution, all eight output parities per wave.  Along
// each axis the output o = 2 q + p takes tap 1 from input q when p = 0, and
// taps 2 from q and 0 from q + 1 when p = 1.  A wave owns MB blocks of 16
// consecutive coarse voxels q: it loads the input fragments of q + (ox, oy, oz)
// for the 8 offsets once, then for each parity p accumulates the taps of the
// offsets o contained in p (27 (o, p) pairs in all) and stores the 16 output
// voxels 2 q + p.  grid y = output channel block of 16.  Weights come as MFMA
// fragments [27 tap][CIN / 32][COUT / 16][64 lanes][8]; a workgroup copies the
// fragments of its channel block into LDS once (27 KiB per 32 input channels)
// and then takes several groups of WAVES x MB voxel blocks in turn, so the
// weights cross L2 once per workgroup instead of once per wave.
template <int CIN, int COUT, int MB>
__global__ void __launch_bounds__(WAVES * 64) k_tconv_all(const bf16* __restrict__ src, const bf16* __restrict__ WF,
                                                         const float* __restrict__ bias, bf16* __restrict__ dst,
                                                         int n_in, const InstState* st, int want_mode) {
  constexpr int NB = COUT / 16;
  constexpr int CPT = CIN / 32;
  constexpr int NFR = 27 * CPT;  // weight fragments of one output channel block
  __shared__ u32x4 wl[NFR * 64];
  const int bt = blockIdx.z;
  if (st && !(st[bt].active && st[bt].mode == want_mode)) return;
  const int nb = blockIdx.y;
  const int n_out = 2 * n_in - 1;
  const int64_t nn_in = (int64_t)n_in * n_in, nvi = nn_in * n_in;
  const int64_t nvo = (int64_t)n_out * n_out * n_out;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  // this block's weight fragments, once per workgroup, from [tap][cc][nb] to [tap][cc]
  for (int q = threadIdx.x; q < NFR * 64; q += WAVES * 64)
    wl[q] = ((const u32x4*)WF)[((q >> 6) * NB + nb) * 64 + (q & 63)];
  __syncthreads();
  const bf16* X = src + (int64_t)bt * nvi * CIN;
  bf16* Y = dst + (int64_t)bt * nvo * COUT;
  const int co = nb * 16 + g * 4;
  const float b0 = bias[co], b1 = bias[co + 1], b2 = bias[co + 2], b3 = bias[co + 3];
  const int64_t nmb = (nvi + 15) / 16;
  // the workgroups of one (nb, instance) take the groups of WAVES * MB blocks in turn
  for (int64_t grp = blockIdx.x; grp * WAVES * MB < nmb; grp += gridDim.x) {
    const int64_t mb0 = (grp * WAVES + wave) * MB;
    if (mb0 >= nmb) continue;
    int64_t vin[MB], vout[MB];
    unsigned okm[MB];  // bit 0: voxel exists; bits 1-3: q + 1 inside along x, y, z
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int64_t v = (mb0 + m) * 16 + r;
      const bool ok = v < nvi;
      const int64_t vc = ok ? v : 0;
      const int qx = (int)(vc % n_in), qy = (int)((vc / n_in) % n_in), qz = (int)(vc / nn_in);
      okm[m] = ok ? (1u | (qx + 1 < n_in ? 2u : 0u) | (qy + 1 < n_in ? 4u : 0u) | (qz + 1 < n_in ? 8u : 0u)) : 0u;
      vin[m] = vc;
      vout[m] = ((int64_t)(2 * qz) * n_out + 2 * qy) * n_out + 2 * qx;
    }
    bf16x8 xin[MB][8][CPT];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
        const unsigned need = 1u | (ox ? 2u : 0u) | (oy ? 4u : 0u) | (oz ? 8u : 0u);
        const bool valid = (okm[m] & need) == need;
        const int64_t vi = vin[m] + ox + oy * (int64_t)n_in + oz * nn_in;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc)
          xin[m][o][cc] = valid ? load8(X + vi * CIN + cc * 32 + g * 8) : zero8();
      }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
      f32x4 acc[MB];
#pragma unroll
      for (int m = 0; m < MB; ++m) acc[m] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        if (o & ~p) continue;
        const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
        const int tx = px ? (ox ? 0 : 2) : 1, ty = py ? (oy ? 0 : 2) : 1, tz = pz ? (oz ? 0 : 2) : 1;
        const int tap = tz * 9 + ty * 3 + tx;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
          const bf16x8 w = __builtin_bit_cast(bf16x8, wl[(tap * CPT + cc) * 64 + lane]);
#pragma unroll
          for (int m = 0; m < MB; ++m)
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xin[m][o][cc], acc[m], 0, 0, 0);
        }
      }
      const unsigned need = 1u | (px ? 2u : 0u) | (py ? 4u : 0u) | (pz ? 8u : 0u);
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        if ((okm[m] & need) != need) continue;
        const int64_t vo = vout[m] + ((int64_t)pz * n_out + py) * n_out + px;
        uint2 pk;
        pk.x = (unsigned)f2bf(acc[m][0] + b0) | ((unsigned)f2bf(acc[m][1] + b1) << 16);
        pk.y = (unsigned)f2bf(acc[m][2] + b2) | ((unsigned)f2bf(acc[m][3] + b3) << 16);
        *(uint2*)(Y + vo * COUT + co) = pk;
      }
    }
  }
}

__global__ void k_w_to_bf16(const float* __restrict__ w, bf16* __restrict__ o, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) o[k] = __float2bfloat16(w[k]);
}

// Stride-1 layer: LDS-tiled kernel for x < n - 1 and the EDGE variant of the
// global-load kernel for x = n - 1.  Grids with n - 1 < 16 use the global-load
// kernel for everything.
template <int CA, int CB, int COUT, int TY, int IN, int EPI, typename Tv, int WL>
void launch_s1_tiled(const MfmaArgs& a, int batch, size_t lds, int nwaves, hipStream_t stream) {
  constexpr int TZ = 2;
  constexpr int MB = COUT >= 64 ? 2 : 4;
  const int n = a.n_out;
  auto kern = k_conv_lds<CA, CB, COUT, TZ, TY, MB, IN, EPI, Tv, WL>;
  if (lds > 65536) hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const int ytiles = (n + TY - 1) / TY, ztiles = (n + TZ - 1) / TZ;
  hipLaunchKernelGGL(kern, dim3((unsigned)(ytiles * ztiles), 1, batch), dim3(nwaves * 64), lds, stream, a);
}

template <int CA, int CB, int COUT, int IN, int EPI, typename Tv>
void launch_s1(const MfmaArgs& a, int batch, hipStream_t stream) {
  constexpr int CL = IN ? 2 : CA + CB;
  constexpr int TZ = 2;
  constexpr int MB = COUT >= 64 ? 2 : 4;
  constexpr size_t LDS_MAX = 160 * 1024;
  const int n = a.n_out;
  const int64_t nvo = (int64_t)n * n * n;
  const int xb = (n - 1) / 16;
  constexpr int CIN = IN ? 8 : CA + CB;
  constexpr size_t WBYTES = (size_t)COUT * 27 * CIN * 2;
  constexpr bool WSMALL = WBYTES <= 32 * 1024;
  // prefer tiles of 2 x 2 rows that let two workgroups share a CU (weights in
  // LDS when they still fit), else 2 x 4 rows with one workgroup per CU
  const size_t t4 = (size_t)(TZ + 2) * (4 + 2) * (n + 1) * CL * 2;
  const size_t t2 = (size_t)(TZ + 2) * (2 + 2) * (n + 1) * CL * 2;
  const int w4 = TZ * 4 * xb / MB, w2 = TZ * 2 * xb / MB;
  int ty = 0, wl = 0;
  size_t lds = 0;
  if ((n - 1) % 16 == 0 && xb >= 1) {
    if (WSMALL && t2 + WBYTES <= LDS_MAX / 2 && w2 >= 2 && w2 <= 8) { ty = 2; wl = 1; lds = t2 + WBYTES; }
    else if (t2 <= LDS_MAX / 2 && w2 >= 2 && w2 <= 8) { ty = 2; lds = t2; }
    else if (WSMALL && t4 + WBYTES <= LDS_MAX && w4 >= 1 && w4 <= 8) { ty = 4; wl = 1; lds = t4 + WBYTES; }
    else if (t4 <= LDS_MAX && w4 >= 1 && w4 <= 8) { ty = 4; lds = t4; }
    else if (t2 <= LDS_MAX && w2 >= 1 && w2 <= 8) { ty = 2; lds = t2; }
  }
  if (ty == 0) {  // small or very large grids: global-load kernel over all voxels
    constexpr int MBG = 4;
    const int64_t nmb = (nvo + 15) / 16;
    const dim3 grid((unsigned)((nmb + WAVES * MBG - 1) / (WAVES * MBG)), 1, batch);
    hipLaunchKernelGGL((k_conv_mfma<IN ? 8 : CA, CB, COUT, 1, MBG, IN, EPI, Tv, 0>), grid, dim3(WAVES * 64), 0, stream,
                       a);
    return;
  }
  if (ty == 4 && wl) launch_s1_tiled<CA, CB, COUT, 4, IN, EPI, Tv, WSMALL ? 1 : 0>(a, batch, lds, w4, stream);
  else if (ty == 4) launch_s1_tiled<CA, CB, COUT, 4, IN, EPI, Tv, 0>(a, batch, lds, w4, stream);
  else if (wl) launch_s1_tiled<CA, CB, COUT, 2, IN, EPI, Tv, WSMALL ? 1 : 0>(a, batch, lds, w2, stream);
  else launch_s1_tiled<CA, CB, COUT, 2, IN, EPI, Tv, 0>(a, batch, lds, w2, stream);
  // the x = n - 1 column (Dirichlet when the head is fused: nothing to write)
  if (!EPI) launch_edge<IN ? 8 : CA, CB, COUT, IN, Tv>(a, batch, stream);
}

// Full-resolution 16-channel layers: the row-reuse sweep for x < n - 1 plus the
// EDGE kernel for x = n - 1 (not needed with the head: that column is
// Dirichlet).  Falls back to launch_s1 where the grid does not fit the sweep.
template <int CA, int CB, int MB, int IN, int EPI, typename Tv, int NPF>
void launch_rows16_npf(const MfmaArgs& a, const RowsGrid& q, int batch, size_t lds, int xb, hipStream_t stream) {
  auto kern = k_conv16_rows<CA, CB, MB, IN, EPI, Tv, NPF>;
  if (lds > 65536) hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const int nz = (q.zhi - q.zlo + q.zc - 1) / q.zc;
  hipLaunchKernelGGL(kern, dim3((unsigned)(q.nedge + q.ytiles * q.nxs * nz), 1, batch), dim3(xb * 64), lds, stream,
                     a, q);
}

template <int CA, int CB, int MB, int IN, int EPI, typename Tv, int NPF0, int NPF1>
void launch_rows16(const MfmaArgs& a, int batch, hipStream_t stream, int target = 1024, int xbmax = 0) {
  constexpr int CL = IN ? 2 : CA + CB;
  typedef RowsTile<CL, IN> T;
  const int n = a.n_out;
  const int xb = (n - 1) / 16;
  // x blocks (one wave each) per workgroup: the largest divisor of xb up to 4
  // (or xbmax); wider grids take nxs workgroups per row range
  int xbw = std::min(std::max(xb, 1), xbmax > 0 ? std::min(xbmax, 4) : 4);
  while (xb % xbw) --xbw;
  const int nxs = xb / xbw;
  const int xw = 16 * xbw + 2;
  const size_t lds = (size_t)T::NRING * T::plane_bytes(MB, xw - 1);
  const bool fits = (n - 1) % 16 == 0 && xb >= 1 && lds <= 160 * 1024 && (IN || a.zero16);
  const int need = fits ? ((MB + 2) * xw * T::SLOTS + xbw * 64 - 1) / (xbw * 64) : 0;
  if (!fits || (IN && need > NPF1)) {
    launch_s1<IN ? 8 : CA, CB, 16, IN, EPI, Tv>(a, batch, stream);
    return;
  }
  RowsGrid q;
  q.ylo = q.zlo = EPI ? 1 : 0;
  q.yhi = q.zhi = EPI ? n - 1 : n;
  q.ytiles = (q.yhi - q.ylo + MB - 1) / MB;
  q.nxs = nxs;
  q.xw = xw;
  const int planes = q.zhi - q.zlo;
  // about four workgroups per compute unit over the batch
  int nz = (target + q.ytiles * nxs * batch - 1) / (q.ytiles * nxs * batch);
  nz = std::max(1, std::min(nz, planes));
  q.zc = (planes + nz - 1) / nz;
  // the x = n - 1 column in extra workgroups (not needed with the head: Dirichlet)
  q.nedge = (!EPI && n <= 16 * kEdgeYB) ? n : 0;
  const size_t lds_all = std::max(lds, q.nedge ? edge_lds_bytes(n, 16) : (size_t)0);
  if constexpr (!IN) {
    launch_rows16_npf<CA, CB, MB, IN, EPI, Tv, 1>(a, q, batch, lds_all, xbw, stream);
  } else {
    if (need <= NPF0) launch_rows16_npf<CA, CB, MB, IN, EPI, Tv, NPF0>(a, q, batch, lds_all, xbw, stream);
    else launch_rows16_npf<CA, CB, MB, IN, EPI, Tv, NPF1>(a, q, batch, lds_all, xbw, stream);
  }
  if (!EPI && !q.nedge) launch_edge<IN ? 8 : CA, CB, 16, IN, Tv>(a, batch, stream);
}

// Stored 16-channel layers: the two-waves-per-SIMD sweep for x < n - 1 plus
// the EDGE kernel for x = n - 1 (not needed with the head: that column is
// Dirichlet).
template <int CA, int CB, int MB, int KS, int EPI, typename Tv>
void launch_ks16(const MfmaArgs& a, int batch, hipStream_t stream, int target = 1024, int xbmax = 0) {
  constexpr int NLW = 4;
  constexpr int TYR = KS ? MB : 2 * MB;
  typedef RowsTile<CA + CB, 0> T;
  const int n = a.n_out;
  const int xb = (n - 1) / 16;
  // x blocks per workgroup: the largest divisor of xb up to 4 (or xbmax; two
  // waves each); wider grids take nxs workgroups per row range
  int xbw = std::min(std::max(xb, 1), xbmax > 0 ? std::min(xbmax, 4) : 4);
  while (xb % xbw) --xbw;
  const int nxs = xb / xbw;
  const int xw = 16 * xbw + 2;
  const size_t lds = 5 * T::plane_bytes(TYR, xw - 1) + (KS ? (size_t)2 * xbw * MB * 64 * 16 : 0);
  const int nload = ((TYR + 2) * xw * T::SLOTS + 63) / 64;
  const bool fits = (n - 1) % 16 == 0 && xb >= 1 && lds <= 160 * 1024 && a.zero16 && nload <= NLW * 2 * xbw;
  if (!fits) {
    launch_s1<CA, CB, 16, 0, EPI, Tv>(a, batch, stream);
    return;
  }
  RowsGrid q;
  q.ylo = q.zlo = EPI ? 1 : 0;
  q.yhi = q.zhi = EPI ? n - 1 : n;
  q.ytiles = (q.yhi - q.ylo + TYR - 1) / TYR;
  q.nxs = nxs;
  q.xw = xw;
  const int planes = q.zhi - q.zlo;
  int nz = (target + q.ytiles * nxs * batch - 1) / (q.ytiles * nxs * batch);
  nz = std::max(1, std::min(nz, planes));
  q.zc = (planes + nz - 1) / nz;
  nz = (planes + q.zc - 1) / q.zc;
  q.nedge = (!EPI && n <= 16 * kEdgeYB) ? n : 0;
  const size_t lds_all = std::max(lds, q.nedge ? edge_lds_bytes(n, 16) : (size_t)0);
  auto kern = k_conv16_ks<CA, CB, MB, KS, EPI, Tv, NLW>;
  if (lds_all > 65536)
    hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_all);
  hipLaunchKernelGGL(kern, dim3((unsigned)(q.nedge + q.ytiles * nxs * nz), 1, batch), dim3(2 * xbw * 64), lds_all,
                     stream, a, q);
  if (!EPI && !q.nedge) launch_edge<CA, CB, 16, 0, Tv>(a, batch, stream);
}

// Coarse-level stride-1 layers (COUT = 32 or 64): the K-split sweep for
// x < n - 1 plus the EDGE kernel for x = n - 1; launch_s1 where it does not fit.
template <int CA, int CB, int COUT, int MB, int KG, int NPF>
void launch_convw(const MfmaArgs& a, int batch, hipStream_t stream, int target = 1024, int xbmax = 0) {
  typedef RowsTile<CA + CB, 0> T;
  constexpr int NF = MB * (COUT / 16);
  const int n = a.n_out;
  const int xb = (n - 1) / 16;
  // x blocks per workgroup: the largest divisor of xb with at most 8 waves (or
  // xbmax blocks); wider grids take nxs workgroups per row range
  int xbw = std::min(std::max(xb, 1), std::max(1, xbmax > 0 ? std::min(xbmax, 8 / KG) : 8 / KG));
  while (xb % xbw) --xbw;
  const int nxs = xb / xbw;
  const int xw = 16 * xbw + 2;
  // ring, partial sums, bias
  const size_t lds = 3 * T::plane_bytes(MB, xw - 1) + (size_t)KG * xbw * NF * 1024 + 256;
  const bool fits = (n - 1) % 16 == 0 && xb >= 1 && xbw * KG <= 8 && lds <= 160 * 1024 &&
                    (MB + 2) * xw * T::CPV <= NPF * xbw * KG * 64;
  if (!fits) {
    launch_s1<CA, CB, COUT, 0, 0, float>(a, batch, stream);
    return;
  }
  RowsGrid q;
  q.ylo = q.zlo = 0;
  q.yhi = q.zhi = n;
  q.ytiles = (n + MB - 1) / MB;
  q.nxs = nxs;
  q.xw = xw;
  int nz = (target + q.ytiles * nxs * batch - 1) / (q.ytiles * nxs * batch);
  nz = std::max(1, std::min(nz, n));
  q.zc = (n + nz - 1) / nz;
  nz = (n + q.zc - 1) / q.zc;
  q.nedge = n <= 16 * kEdgeYB ? n : 0;
  const size_t lds_all = std::max(lds, q.nedge ? edge_lds_bytes(n, COUT) : (size_t)0);
  auto kern = k_convw<CA, CB, COUT, MB, KG, NPF>;
  if (lds_all > 65536)
    hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_all);
  hipLaunchKernelGGL(kern, dim3((unsigned)(q.nedge + q.ytiles * nxs * nz), 1, batch), dim3(xbw * KG * 64), lds_all,
                     stream, a, q);
  if (!q.nedge) launch_edge<CA, CB, COUT, 0, float>(a, batch, stream);
}

MfmaArgs args_from(const ConvP& p, const bf16* w) {
  MfmaArgs a;
  a.a = (const bf16*)p.a;
  a.b = (const bf16*)p.b;
  a.w = w;
  a.bias = p.bias;
  a.y = (bf16*)p.y;
  a.n_in = p.n_in;
  a.n_out = p.n_out;
  a.relu = p.relu;
  a.st = p.st;
  a.want_mode = p.want_mode;
  return a;
}

template <int CA, int CB, int COUT, int STRIDE, int MB>
void launch_conv(const ConvP& p, int batch, const bf16* w, hipStream_t stream) {
  const int64_t nvo = (int64_t)p.n_out * p.n_out * p.n_out;
  const int64_t nmb = (nvo + 15) / 16;
  const dim3 grid((unsigned)((nmb + WAVES * MB - 1) / (WAVES * MB)), 1, batch);
  const MfmaArgs a = args_from(p, w);
  if (STRIDE == 1) {
    launch_s1<CA, CB, COUT, 0, 0, float>(a, batch, stream);
    return;
  }
  hipLaunchKernelGGL((k_conv_mfma<CA, CB, COUT, STRIDE, MB, 0, 0, float>), grid, dim3(WAVES * 64), 0, stream, a);
}

template <int CIN, int COUT, int MB>
void launch_tconv_all(const ConvP& p, int batch, const bf16* wfrag, hipStream_t stream, int cap = 0) {
  // workgroups per (channel block, instance): all groups of WAVES x MB blocks,
  // or fewer that loop (cap = total workgroups aimed at; 0: 1024)
  const int64_t nmb = ((int64_t)p.n_in * p.n_in * p.n_in + 15) / 16;
  const int64_t groups = (nmb + WAVES * MB - 1) / (WAVES * MB);
  const int target = cap > 0 ? cap : 1024;
  const int64_t per = std::max<int64_t>(1, target / ((COUT / 16) * batch));
  const dim3 grid((unsigned)std::min(groups, per), COUT / 16, batch);
  hipLaunchKernelGGL((k_tconv_all<CIN, COUT, MB>), grid, dim3(WAVES * 64), 0, stream, (const bf16*)p.a, wfrag, p.bias,
                     (bf16*)p.y, p.n_in, p.st, p.want_mode);
}


}  // namespace

// First-layer weights padded to 8 input channels: [16][27][8], channels 2..7 zero.
__global__ void k_w_in8(const float* __restrict__ w, bf16* __restrict__ o) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 16 * 27 * 8) return;
  const int ci = k % 8, t = (k / 8) % 27, co = k / (8 * 27);
  o[k] = __float2bfloat16(ci < 2 ? w[(co * 27 + t) * 2 + ci] : 0.0f);
}

static int64_t mfma_weight_count() {
  int64_t tot = 0;
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerSpec& L = kLayers[l];
    tot += (int64_t)L.cout * (L.kind == KIND_PT ? 1 : 27) * L.cin;
  }
  return tot;
}

// Row-reuse weight layout [COUT][3 ty][KCT * 32] of a stride-1 layer.
// IN = 1 (two input channels): k = 8 tz + 2 tx + ch for tz < 3, else zero.
// Otherwise k = (3 tz + tx) * CIN + ci, zero from 9 CIN on.
template <int CIN, int IN, int COUT = 16>
__global__ void k_w_rows(const float* __restrict__ w, bf16* __restrict__ o) {
  constexpr int KCT = RowsK<CIN, IN>::KCT;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= COUT * 3 * KCT * 32) return;
  const int kk = k % (KCT * 32), ty = (k / (KCT * 32)) % 3, co = k / (3 * KCT * 32);
  float v = 0.0f;
  if (IN) {
    const int tz = kk / 8, e = kk % 8, tx = e / 2, ch = e % 2;
    if (tz < 3 && tx < 3) v = w[(co * 27 + tz * 9 + ty * 3 + tx) * 2 + ch];
  } else {
    const int pp = kk / CIN, ci = kk % CIN;
    if (pp < 9) v = w[(co * 27 + (pp / 3) * 9 + ty * 3 + pp % 3) * CIN + ci];
  }
  o[k] = __float2bfloat16(v);
}

// Transposed-convolution weights as MFMA A fragments: element e of lane
// (g, r) of fragment (tap, cc, nb) is w[nb * 16 + r][tap][cc * 32 + g * 8 + e].
template <int CIN, int COUT>
__global__ void k_w_tfrag(const float* __restrict__ w, bf16* __restrict__ o) {
  constexpr int CPT = CIN / 32, NB = COUT / 16;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 27 * CPT * NB * 512) return;
  const int e = k % 8, lane = (k / 8) % 64, f = k / 512;
  const int nb = f % NB, cc = (f / NB) % CPT, tap = f / (NB * CPT);
  const int g = lane >> 4, r = lane & 15;
  o[k] = __float2bfloat16(w[((int64_t)(nb * 16 + r) * 27 + tap) * CIN + cc * 32 + g * 8 + e]);
}

constexpr int64_t kIn8Count = 16 * 27 * 8;
constexpr int64_t kRowsIn0 = 16 * 3 * RowsK<2, 1>::KCT * 32;
constexpr int64_t kRowsL0b = 16 * 3 * RowsK<16, 0>::KCT * 32;
constexpr int64_t kRowsD0 = 16 * 3 * RowsK<32, 0>::KCT * 32;

constexpr int64_t kRowsL1b = 32 * 3 * RowsK<32, 0>::KCT * 32;
constexpr int64_t kRowsL2b = 64 * 3 * RowsK<64, 0>::KCT * 32;
constexpr int64_t kRowsD1 = 32 * 3 * RowsK<64, 0>::KCT * 32;
constexpr int64_t kTfU1 = 27 * (64 / 32) * (32 / 16) * 512;
constexpr int64_t kTfU0 = 27 * (32 / 32) * (16 / 16) * 512;
constexpr int64_t kZeroCount = 128;  // 256 zero bytes

struct MfmaWeights {
  const bf16* in8;
  const bf16* rows_in0;
  const bf16* rows_l0b;
  const bf16* rows_d0;
  const bf16* rows_l1b;
  const bf16* rows_l2b;
  const bf16* rows_d1;
  const bf16* tf_u1;
  const bf16* tf_u0;
  const bf16* zeros;
};

static MfmaWeights mfma_extra(const CnnState& c) {
  const bf16* e = c.wmf + mfma_weight_count();
  MfmaWeights x;
  x.in8 = e;
  x.rows_in0 = x.in8 + kIn8Count;
  x.rows_l0b = x.rows_in0 + kRowsIn0;
  x.rows_d0 = x.rows_l0b + kRowsL0b;
  x.rows_l1b = x.rows_d0 + kRowsD0;
  x.rows_l2b = x.rows_l1b + kRowsL1b;
  x.rows_d1 = x.rows_l2b + kRowsL2b;
  x.tf_u1 = x.rows_d1 + kRowsD1;
  x.tf_u0 = x.tf_u1 + kTfU1;
  x.zeros = x.tf_u0 + kTfU0;
  return x;
}

void cnn_prepare_mfma_weights(CnnState& c, const float* d_w, hipStream_t stream) {
  const int64_t tot = mfma_weight_count();
  const int64_t extra =
      kIn8Count + kRowsIn0 + kRowsL0b + kRowsD0 + kRowsL1b + kRowsL2b + kRowsD1 + kTfU1 + kTfU0 + kZeroCount;
  if (!c.wmf && hipMalloc(&c.wmf, sizeof(bf16) * (size_t)(tot + extra)) != hipSuccess) {
    c.wmf = nullptr;
    return;
  }
  const MfmaWeights x = mfma_extra(c);
  (void)hipMemsetAsync((void*)x.zeros, 0, sizeof(bf16) * kZeroCount, stream);
  hipLaunchKernelGGL(k_w_in8, dim3((kIn8Count + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[0],
                     (bf16*)x.in8);
  hipLaunchKernelGGL((k_w_rows<2, 1>), dim3((kRowsIn0 + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[0],
                     (bf16*)x.rows_in0);
  hipLaunchKernelGGL((k_w_rows<16, 0>), dim3((kRowsL0b + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[1],
                     (bf16*)x.rows_l0b);
  hipLaunchKernelGGL((k_w_rows<32, 0>), dim3((kRowsD0 + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[9],
                     (bf16*)x.rows_d0);
  hipLaunchKernelGGL((k_w_rows<32, 0, 32>), dim3((kRowsL1b + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[3],
                     (bf16*)x.rows_l1b);
  hipLaunchKernelGGL((k_w_rows<64, 0, 64>), dim3((kRowsL2b + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[5],
                     (bf16*)x.rows_l2b);
  hipLaunchKernelGGL((k_w_rows<64, 0, 32>), dim3((kRowsD1 + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[7],
                     (bf16*)x.rows_d1);
  hipLaunchKernelGGL((k_w_tfrag<64, 32>), dim3((kTfU1 + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[6],
                     (bf16*)x.tf_u1);
  hipLaunchKernelGGL((k_w_tfrag<32, 16>), dim3((kTfU0 + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[8],
                     (bf16*)x.tf_u0);
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerSpec& L = kLayers[l];
    const int64_t nw = (int64_t)L.cout * (L.kind == KIND_PT ? 1 : 27) * L.cin;
    hipLaunchKernelGGL(k_w_to_bf16, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, stream, d_w + c.w_off[l],
                       c.wmf + c.wt_off[l], nw);
  }
}

bool conv_mfma_supported(int layer) { return layer >= 1 && layer <= 9; }

template <typename Tv>
void conv_mfma_in0(const CnnState& c, const Tv* z, const int64_t* off, const double* inv_s, const float* dist,
                   int n, int batch, bf16* a0, const InstState* st, hipStream_t stream) {
  constexpr int MB = 4;
  const int64_t nvo = (int64_t)n * n * n;
  const int64_t nmb = (nvo + 15) / 16;
  MfmaArgs a;
  a.w = mfma_extra(c).in8;
  a.wrows = mfma_extra(c).rows_in0;
  a.bias = c.w + c.b_off[0];
  a.y = a0;
  a.n_in = n;
  a.n_out = n;
  a.relu = 1;
  a.st = st;
  a.z = z;
  a.off = off;
  a.inv_s = inv_s;
  a.dist = dist;
  (void)nmb;
  launch_rows16<0, 0, 5, 1, 0, Tv, 2, 4>(a, batch, stream, sweep_target(c, 0, 1024), c.tile_xb[0]);
}
template void conv_mfma_in0<float>(const CnnState&, const float*, const int64_t*, const double*, const float*, int,
                                   int, bf16*, const InstState*, hipStream_t);
template void conv_mfma_in0<double>(const CnnState&, const double*, const int64_t*, const double*, const float*, int,
                                    int, bf16*, const InstState*, hipStream_t);

template <typename Tv>
void conv_mfma_d0_head(const CnnState& c, const bf16* u0, const bf16* s0, int n, int batch, Tv* z,
                       const int64_t* off, const double* alpha, double alpha_override, const double* scale,
                       const InstState* st, hipStream_t stream) {
  constexpr int MB = 4;
  const int64_t nvo = (int64_t)n * n * n;
  const int64_t nmb = (nvo + 15) / 16;
  MfmaArgs a;
  a.a = u0;
  a.b = s0;
  a.w = c.wmf + c.wt_off[9];
  a.wrows = mfma_extra(c).rows_d0;
  a.zero16 = mfma_extra(c).zeros;
  a.bias = c.w + c.b_off[9];
  a.n_in = n;
  a.n_out = n;
  a.relu = 1;
  a.st = st;
  a.wh = c.w + c.w_off[10];
  a.bh = c.w + c.b_off[10];
  a.zout = z;
  a.off = off;
  a.alpha = alpha;
  a.alpha_override = alpha_override;
  a.scale = scale;
  (void)nmb;
  const int t = sweep_target(c, 9, kSweepBlocksD0);
  const int xm = c.tile_xb[9];
  // the three-plane z sweep with 4, 6 or 8 rows per workgroup (codes 12, 13,
  // 14; 0 = the default, 8 rows); every choice sums each output's taps in the
  // same order.  Grids it does not fit take the K-split sweep (codes 3, 4, 5
  // select that kernel's rows per wave pair directly).
  const int code = c.tile_mb[9] ? c.tile_mb[9] : 14;
  if (code == 12 && launch_zb16<2, Tv>(a, batch, stream, t, xm)) return;
  if (code == 13 && launch_zb16<3, Tv>(a, batch, stream, t, xm)) return;
  if (code == 14 && launch_zb16<4, Tv>(a, batch, stream, t, xm)) return;
  if (code == 3) launch_ks16<16, 16, 3, 1, 1, Tv>(a, batch, stream, t, xm);
  else if (code == 5) launch_ks16<16, 16, 5, 1, 1, Tv>(a, batch, stream, t, xm);
  else launch_ks16<16, 16, 4, 1, 1, Tv>(a, batch, stream, t, xm);
}
template void conv_mfma_d0_head<float>(const CnnState&, const bf16*, const bf16*, int, int, float*, const int64_t*,
                                       const double*, double, const double*, const InstState*, hipStream_t);
template void conv_mfma_d0_head<double>(const CnnState&, const bf16*, const bf16*, int, int, double*,
                                        const int64_t*, const double*, double, const double*, const InstState*,
                                        hipStream_t);

// Layers L0b .. D0 (indices 1 .. 9) with their fixed channel counts.
void conv_mfma_layer(const ConvP& p, int kind, int batch, int layer, CnnState& c, hipStream_t stream) {
  const bf16* w = c.wmf + c.wt_off[layer];
  (void)kind;
  switch (layer) {
    case 1: {                                                             // L0b
      MfmaArgs a = args_from(p, w);
      a.wrows = mfma_extra(c).rows_l0b;
      a.zero16 = mfma_extra(c).zeros;
      const int t = sweep_target(c, 1, 1024);
      const int xm = c.tile_xb[1];
      if (c.tile_mb[1] == 3) launch_ks16<16, 0, 3, 0, 0, float>(a, batch, stream, t, xm);
      else if (c.tile_mb[1] == 5) launch_ks16<16, 0, 5, 0, 0, float>(a, batch, stream, t, xm);
      else if (c.tile_mb[1] == 6) launch_ks16<16, 0, 6, 0, 0, float>(a, batch, stream, t, xm);
      else launch_ks16<16, 0, 4, 0, 0, float>(a, batch, stream, t, xm);
      break;
    }
    case 2:  // L1a: M blocks per wave chosen by the autotuner
      if (c.sweep_blocks[2] == 2) launch_conv<16, 0, 32, 2, 2>(p, batch, w, stream);
      else if (c.sweep_blocks[2] == 8) launch_conv<16, 0, 32, 2, 8>(p, batch, w, stream);
      else launch_conv<16, 0, 32, 2, 4>(p, batch, w, stream);
      break;
    case 3: {                                                             // L1b
      MfmaArgs a = args_from(p, w);
      a.wrows = mfma_extra(c).rows_l1b;
      a.zero16 = mfma_extra(c).zeros;
      const int t = sweep_target(c, 3, 1024);
      const int xm = c.tile_xb[3];
      if (c.tile_mb[3] == 2) launch_convw<32, 0, 32, 2, 3, 2>(a, batch, stream, t, xm);
      else if (c.tile_mb[3] == 4) launch_convw<32, 0, 32, 4, 3, 3>(a, batch, stream, t, xm);
      else if (c.tile_mb[3] == 6) launch_convw<32, 0, 32, 6, 3, 3>(a, batch, stream, t, xm);
      else launch_convw<32, 0, 32, 3, 3, 2>(a, batch, stream, t, xm);
      break;
    }
    case 4:  // L2a
      if (c.sweep_blocks[4] == 1) launch_conv<32, 0, 64, 2, 1>(p, batch, w, stream);
      else if (c.sweep_blocks[4] == 4) launch_conv<32, 0, 64, 2, 4>(p, batch, w, stream);
      else launch_conv<32, 0, 64, 2, 2>(p, batch, w, stream);
      break;
    case 5: {                                                             // L2b
      MfmaArgs a = args_from(p, w);
      a.wrows = mfma_extra(c).rows_l2b;
      a.zero16 = mfma_extra(c).zeros;
      launch_convw<64, 0, 64, 2, 8, 2>(a, batch, stream, sweep_target(c, 5, kSweepBlocksL2b));
      break;
    }
    case 6:  // U1
      if (c.sweep_blocks[6] == 2) launch_tconv_all<64, 32, 2>(p, batch, mfma_extra(c).tf_u1, stream, c.tile_mb[6]);
      else launch_tconv_all<64, 32, 1>(p, batch, mfma_extra(c).tf_u1, stream, c.tile_mb[6]);
      break;
    case 7: {                                                             // D1
      MfmaArgs a = args_from(p, w);
      a.wrows = mfma_extra(c).rows_d1;
      a.zero16 = mfma_extra(c).zeros;
      const int t = sweep_target(c, 7, 1024);
      if (c.tile_mb[7] == 2) launch_convw<32, 32, 32, 2, 4, 3>(a, batch, stream, t, c.tile_xb[7]);
      else launch_convw<32, 32, 32, 3, 4, 3>(a, batch, stream, t, c.tile_xb[7]);
      break;
    }
    case 8:  // U0
      if (c.sweep_blocks[8] == 1) launch_tconv_all<32, 16, 1>(p, batch, mfma_extra(c).tf_u0, stream, c.tile_mb[8]);
      else if (c.sweep_blocks[8] == 4) launch_tconv_all<32, 16, 4>(p, batch, mfma_extra(c).tf_u0, stream, c.tile_mb[8]);
      else launch_tconv_all<32, 16, 2>(p, batch, mfma_extra(c).tf_u0, stream, c.tile_mb[8]);
      break;
    case 9: {                                                             // D0
      MfmaArgs a = args_from(p, w);
      a.wrows = mfma_extra(c).rows_d0;
      a.zero16 = mfma_extra(c).zeros;
      launch_ks16<16, 16, 4, 1, 0, float>(a, batch, stream);
      break;
    }
    default: break;
  }
}

}  // namespace mdnp
