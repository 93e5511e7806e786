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

// Stride-1 convolution sweeping along z.  A workgroup owns output rows
// y0..y0+TY-1 for x in [0, n-1) (the column x = n-1 goes to the EDGE variant of
// k_conv_mfma) and planes z0..z0+ZC-1.  LDS holds a ring of the three input
// planes z-1, z, z+1 (rows y0-1..y0+TY, x = -1..n-1, zero outside the grid);
// while the MFMAs of plane z run, every thread holds its share of input plane
// z+2 in registers and writes it into the ring afterwards, so each input plane
// is read from memory once per workgroup (halo only in y).  Tile voxels are
// padded to CLP channels to spread LDS banks.
template <int CA, int CB, int COUT, int TY, int MB, int IN, int EPI, typename Tv>
__global__ void __launch_bounds__(512) k_conv_sweep(MfmaArgs p, int zc) {
  constexpr int CIN = IN ? 8 : CA + CB;
  constexpr int CL = IN ? 2 : CA + CB;
  constexpr int CLP = (CL >= 32) ? CL + 8 : CL;
  constexpr int NB = COUT / 16;
  constexpr int KCH = (27 * CIN + 31) / 32;
  constexpr int YW = TY + 2;
  constexpr int NPF = 8;  // prefetch registers (16 B each) per thread
  extern __shared__ unsigned short ring[];
  int bxr, bt;
  xcd_remap(bxr, bt);
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  const int n = p.n_out;
  const int XW = n + 1;
  const int ytiles = (n + TY - 1) / TY;
  const int y0 = (bxr % ytiles) * TY, z0 = (bxr / ytiles) * zc;
  const int zend = min(n, z0 + zc);
  const int64_t nv = (int64_t)n * n * n;
  const int nthr = blockDim.x;
  const int plane_elems = YW * XW * CLP;  // bf16 per ring plane
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  // ---- plane loader: element q of a plane = (row, x, 8-channel chunk) or (row, x) for IN
  constexpr int CPV = IN ? 1 : CL / 8;
  const int plane_items = YW * XW * CPV;
  const bf16* A = IN ? nullptr : p.a + (int64_t)bt * nv * CA;
  const bf16* B = CB ? p.b + (int64_t)bt * nv * CB : nullptr;
  const Tv* Z = IN ? (const Tv*)p.z + p.off[bt] : nullptr;
  const float* D = IN ? p.dist + (int64_t)bt * nv : nullptr;
  const float sc = IN ? (float)p.inv_s[bt] : 0.0f;
  auto load_plane = [&](int gz, u32x4 (&buf)[NPF]) {
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int q = threadIdx.x + k * nthr;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (q < plane_items) {
        const int vt = q / CPV, ch = q - vt * CPV;
        const int row = vt / XW, xx = vt - row * XW;
        const int gx = xx - 1, gy = y0 + row - 1;
        if (gz >= 0 && gz < n && gy >= 0 && gy < n && gx >= 0) {
          const int64_t vv = ((int64_t)gz * n + gy) * n + gx;
          if (IN) {
            v.x = (unsigned)f2bf((float)Z[vv] * sc) | ((unsigned)f2bf(D[vv]) << 16);
          } else {
            constexpr int CPA = CA / 8;
            v = (CB == 0 || ch < CPA) ? *(const u32x4*)(A + vv * CA + ch * 8)
                                      : *(const u32x4*)(B + vv * CB + (ch - CPA) * 8);
          }
        }
      }
      buf[k] = v;
    }
  };
  auto store_plane = [&](int slot, const u32x4 (&buf)[NPF]) {
    unsigned short* pl = ring + (size_t)slot * plane_elems;
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int q = threadIdx.x + k * nthr;
      if (q < plane_items) {
        const int vt = q / CPV, ch = q - vt * CPV;
        if (IN) *(unsigned*)(pl + (size_t)vt * CLP) = buf[k].x;
        else *(u32x4*)(pl + (size_t)vt * CLP + ch * 8) = buf[k];
      }
    }
  };
  // M-block geometry inside a plane
  const int XB = (n - 1) >> 4;
  int tb[MB];
  bool vrow[MB];
  int64_t vrowbase[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int mb = wave * MB + m;
    const int row = mb / XB, xq = mb - row * XB;
    const int xl = xq * 16 + r;
    tb[m] = row * XW + xl;  // tap (0, 0) position inside a ring plane
    vrow[m] = y0 + row < n;
    vrowbase[m] = (int64_t)(y0 + row) * n + xl;
  }
  // prologue: planes z0-1 and z0 into the ring, z0+1 into registers
  u32x4 pf[NPF];
  load_plane(z0 - 1, pf);
  store_plane(0, pf);
  load_plane(z0, pf);
  store_plane(1, pf);
  load_plane(z0 + 1, pf);
  __syncthreads();
  const unsigned short* wsrc = (const unsigned short*)p.w;
  for (int z = z0; z < zend; ++z) {
    // ring slots: plane z-1 -> (z - z0) % 3, z -> +1, z+1 -> +2 (written below)
    const int s0 = (z - z0) % 3;
    store_plane((s0 + 2) % 3, pf);
    __syncthreads();
    if (z + 2 < zend + 1) load_plane(z + 2, pf);
    f32x4 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[m][nb] = {0.f, 0.f, 0.f, 0.f};
    auto fetch = [&](int c, bf16x8 (&wf)[NB], bf16x8 (&xf)[MB]) {
      const int k0 = c * 32 + g * 8;
      const int tap = k0 / CIN;
      const int ci = k0 - tap * CIN;
      const bool tap_ok = tap < 27;
      const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
      const unsigned short* pl = ring + (size_t)((s0 + tz) % 3) * plane_elems;
      const int toff = ty * XW + tx;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        wf[nb] = tap_ok ? __builtin_bit_cast(bf16x8, *(const u32x4*)(wsrc + ((nb * 16 + r) * 27 + tap) * CIN + ci))
                        : zero8();
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        if (!tap_ok) {
          xf[m] = zero8();
        } else if (IN) {
          u32x4 v = {*(const unsigned*)(pl + (size_t)(tb[m] + toff) * CLP), 0u, 0u, 0u};
          xf[m] = __builtin_bit_cast(bf16x8, v);
        } else {
          xf[m] = __builtin_bit_cast(bf16x8, *(const u32x4*)(pl + (size_t)(tb[m] + toff) * CLP + ci));
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
    bf16x8 wA[NB], xA[MB], wB[NB], xB[MB];
    fetch(0, wA, xA);
#pragma unroll
    for (int c = 0; c < KCH; c += 2) {
      if (c + 1 < KCH) fetch(c + 1, wB, xB);
      mma(wA, xA);
      if (c + 2 < KCH) fetch(c + 2, wA, xA);
      if (c + 1 < KCH) mma(wB, xB);
    }
    // epilogue for plane z
    if (EPI == 0) {
      bf16* Y = p.y + (int64_t)bt * nv * COUT;
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        if (!vrow[m]) continue;
        const int64_t v = (int64_t)z * n * n + vrowbase[m];
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
          *(uint2*)(Y + v * COUT + co) = pk;
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
        if (g == 0 && vrow[m]) {
          const int64_t v = (int64_t)z * n * n + vrowbase[m];
          const int ox = (int)(v % n), oy = (int)((v / n) % n);
          const bool bnd = ox == 0 || oy == 0 || z == 0 || ox == n - 1 || oy == n - 1 || z == n - 1;
          if (!bnd) zo[v] = (Tv)(f * (h + p.bh[0]));
        }
      }
    }
    __syncthreads();
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
  // the x = n - 1 column
  constexpr int MBE = 4;
  const int64_t nmb = ((int64_t)n * n + 15) / 16;
  const dim3 grid((unsigned)((nmb + WAVES * MBE - 1) / (WAVES * MBE)), 1, batch);
  hipLaunchKernelGGL((k_conv_mfma<IN ? 8 : CA, CB, COUT, 1, MBE, IN, EPI, Tv, 1>), grid, dim3(WAVES * 64), 0, stream,
                     a);
}

template <int CA, int CB, int COUT, int STRIDE, int MB>
void launch_conv(const ConvP& p, int batch, const bf16* w, hipStream_t stream) {
  const int64_t nvo = (int64_t)p.n_out * p.n_out * p.n_out;
  const int64_t nmb = (nvo + 15) / 16;
  const dim3 grid((unsigned)((nmb + WAVES * MB - 1) / (WAVES * MB)), 1, batch);
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
  if (STRIDE == 1) {
    launch_s1<CA, CB, COUT, 0, 0, float>(a, batch, stream);
    return;
  }
  hipLaunchKernelGGL((k_conv_mfma<CA, CB, COUT, STRIDE, MB, 0, 0, float>), grid, dim3(WAVES * 64), 0, stream, a);
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

void cnn_prepare_mfma_weights(CnnState& c, const float* d_w, hipStream_t stream) {
  const int64_t tot = mfma_weight_count();
  if (!c.wmf && hipMalloc(&c.wmf, sizeof(bf16) * (size_t)(tot + 16 * 27 * 8)) != hipSuccess) {
    c.wmf = nullptr;
    return;
  }
  hipLaunchKernelGGL(k_w_in8, dim3((16 * 27 * 8 + 255) / 256), dim3(256), 0, stream, d_w + c.w_off[0], c.wmf + tot);
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
  a.w = c.wmf + mfma_weight_count();
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
  launch_s1<8, 0, 16, 1, 0, Tv>(a, batch, stream);
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
  launch_s1<16, 16, 16, 0, 1, Tv>(a, batch, stream);
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
