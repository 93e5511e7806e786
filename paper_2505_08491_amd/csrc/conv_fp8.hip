// The U-net preconditioner with E4M3 weights and E4M3 activations on the gfx950
// FP8 matrix cores (v_mfma_scale_f32_16x16x128_f8f6f4 with unit block scales,
// FP32 accumulation).
//
// Number formats (the paper runs its network in full precision; these are the
// readings of the 8-bit variant):
//   * weights: E4M3 code x a power-of-two scale per output channel (the
//     per-channel quantisation of the FP8-weight mode, done before packing);
//   * activations: every tensor a 3x3x3 layer reads (the input X and the
//     output of each 3x3x3 layer after its ReLU) is stored as E4M3 codes of
//     value / s with one power-of-two scale s per tensor; the two tensors
//     stacked into one layer input share one scale, so a K range never mixes
//     scales;
//   * a layer's output is acc * (s_in * s_w[co]) + bias, ReLU, then the code of
//     that / s_out (round to nearest, ties to even mantissa, saturating at
//     448); the 1x1 head reads the D0 output on its E4M3 grid in FP32.
//
// Each layer is an implicit GEMM D[co][voxel] = sum over k = (tap, ci) of
// W[co][k] X[k][voxel], 16 couts x 16 voxels x 128 k per MFMA.  Lane l = 16 g + r
// supplies row r of the A (weight) and column r of the B (input) operand with
// the 32 k-values 32 (4 c + g) .. + 31 of chunk c; any assignment of k-values to
// bytes works as long as both operands use the same one, and here byte j of
// lane group g is k = 32 (4 c + g) + j, k = tap * CIN + ci (channels of source
// A first).  The result lands as D[4 g + q][r] in accumulator q: lane (g, r)
// holds output channels 4 g .. + 3 of voxel r.  Inputs are read straight from
// global memory (16-byte loads; L1 and L2 serve the 27-fold tap reuse).  The
// transposed layers use the 8-parity split of the BF16 kernels: per output
// parity p the k range is (input offset o contained in p, ci).

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "conv_common.hpp"
#include "kernels.hpp"

namespace mdnp {

namespace {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
typedef __attribute__((ext_vector_type(8))) int i32x8;

constexpr int kWaves8 = 4;   // waves per workgroup
constexpr int kMB8 = 2;      // 16-voxel blocks per wave

__host__ __device__ inline int64_t cube8(int n) { return (int64_t)n * n * n; }

// E4M3 code of x (round to nearest, ties to even mantissa; |x| >= 448 and NaN
// give +-448).  Exponent bias 7, subnormals m / 8 * 2^-6.
__host__ __device__ inline unsigned e4m3_code(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  const unsigned u = __float_as_uint(x);
#else
  unsigned u;
  std::memcpy(&u, &x, 4);
#endif
  const unsigned sgn = (u >> 24) & 0x80u;
  const unsigned ua = u & 0x7FFFFFFFu;
  float a;
#ifdef __HIP_DEVICE_COMPILE__
  a = __uint_as_float(ua);
#else
  std::memcpy(&a, &ua, 4);
#endif
  unsigned c;
  if (!(a < 448.0f)) {
    c = 0x7Eu;
  } else if (a < 0.015625f) {
    c = (unsigned)rintf(a * 512.0f);  // m * 2^-9, m = 8 is the first normal
  } else {
    int e = (int)(ua >> 23) - 127;    // -6 .. 8
    unsigned r = (ua >> 20) & 7u;
    const unsigned rem = ua & 0xFFFFFu;
    if (rem > 0x80000u || (rem == 0x80000u && (r & 1u))) ++r;
    if (r == 8u) {
      r = 0u;
      ++e;
    }
    c = ((unsigned)(e + 7) << 3) | r;
    if (c > 0x7Eu) c = 0x7Eu;
  }
  return sgn | c;
}

__device__ inline float e4m3_value(unsigned c) {
  const unsigned e = (c >> 3) & 15u, m = c & 7u;
  const float v = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;
  return (c & 0x80u) ? -v : v;
}

struct Fp8Args {
  const uint8_t* a = nullptr;  // source A (E4M3) [batch][vox][CA]
  const uint8_t* b = nullptr;  // source B (E4M3) [batch][vox][CB]
  const uint8_t* w = nullptr;  // packed weight fragments of the layer
  const float* wsc = nullptr;  // [COUT] weight scales
  const float* bias = nullptr;
  uint8_t* y = nullptr;        // output (E4M3) [batch][vox][COUT]
  float s_in = 1.f;            // scale of the input tensor(s)
  float inv_s_out = 1.f;       // 1 / scale of the output tensor
  int n_in = 0, n_out = 0, relu = 0;
  const InstState* st = nullptr;
  int want_mode = 0;
  // first layer: channel 0 = z * inv_s, channel 1 = distance, both / s_in
  const void* z = nullptr;
  const int64_t* off = nullptr;
  const double* inv_s = nullptr;
  const float* dist = nullptr;
  // last layer: the D0 output on its grid (scale s_out), the 1x1 head and the unscaling
  float s_out = 1.f;
  const float* wh = nullptr;
  const float* bh = nullptr;
  void* zout = nullptr;
  const double* alpha = nullptr;
  double alpha_override = 0.0;
  const double* scale = nullptr;
  int all_nodes = 0;           // natural boundary: write every node
};

__device__ inline i32x8 zero32() {
  i32x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
  return v;
}

__device__ inline i32x8 join(u32x4 lo, u32x4 hi) {
  i32x8 v = {(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
  return v;
}

__device__ inline u32x4 ld16(const uint8_t* p) { return *(const u32x4*)p; }

__device__ inline f32x4 mfma8(const i32x8& a, const i32x8& b, const f32x4& c) {
  // E4M3 x E4M3 (format code 0), block scales 2^0 (E8M0 127)
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

// Stride-1 / stride-2 convolution, zero padding 1, channel-stacked input [A | B].
// IN = 1: the first layer, input built from the Krylov vector (2 channels).
// EPI = 1: the last layer (16 outputs) with the 1x1 head and the unscaling
// z0 = ||b0|| / alpha * U written into the Krylov vector (interior nodes, or
// every node with all_nodes).
template <int CA, int CB, int COUT, int STRIDE, int IN, int EPI, typename Tv>
__global__ void __launch_bounds__(kWaves8 * 64) k_conv8(Fp8Args p) {
  constexpr int CIN = IN ? 2 : CA + CB;
  constexpr int NB = COUT / 16;
  constexpr int KE = 27 * CIN;
  constexpr int NCH = (KE + 127) / 128;
  constexpr int MB = kMB8;
  const int bt = blockIdx.z;
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  const int n_in = p.n_in, n_out = p.n_out;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const int64_t nvo = cube8(n_out), nvi = cube8(n_in);
  const int64_t mb0 = ((int64_t)blockIdx.x * kWaves8 + wave) * MB;
  int64_t vout[MB], ibase[MB];
  unsigned vmask[MB];  // bits 0-2: x offsets -1, 0, +1 inside; 3-5: y; 6-8: z
  bool vok[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int64_t v = (mb0 + m) * 16 + r;
    const bool ok = v < nvo;
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
  const uint8_t* A = IN ? nullptr : p.a + (int64_t)bt * nvi * CA;
  const uint8_t* B = CB ? p.b + (int64_t)bt * nvi * CB : nullptr;
  const Tv* Z = IN ? (const Tv*)p.z + p.off[bt] : nullptr;
  const float* D = IN ? p.dist + (int64_t)bt * nvi : nullptr;
  const float zsc = IN ? (float)p.inv_s[bt] / p.s_in : 0.0f, dsc = IN ? 1.0f / p.s_in : 0.0f;
  const int64_t nn = (int64_t)n_in * n_in;
  auto tap_in = [&](int tap, int m, int64_t& vin) -> bool {
    const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
    const unsigned need = (1u << tx) | (8u << ty) | (64u << tz);
    vin = ibase[m] + (int64_t)(tz - 1) * nn + (int64_t)(ty - 1) * n_in + (tx - 1);
    return tap < 27 && (vmask[m] & need) == need;
  };
  f32x4 acc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = {0.f, 0.f, 0.f, 0.f};
  // the 32 input bytes of lane group g in chunk c for voxel block m
  auto xfrag = [&](int c, int m) -> i32x8 {
    const int s = 4 * c + g;  // sub-chunk: k = 32 s .. 32 s + 31
    if constexpr (IN) {
      // taps 16 s .. 16 s + 15, two channels each
      unsigned wd[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        int64_t vin;
        if (tap_in(16 * s + j, m, vin)) {
          const unsigned c0 = e4m3_code((float)Z[vin] * zsc), c1 = e4m3_code(D[vin] * dsc);
          wd[j >> 1] |= (c0 | (c1 << 8)) << (16 * (j & 1));
        }
      }
      i32x8 v = {(int)wd[0], (int)wd[1], (int)wd[2], (int)wd[3], (int)wd[4], (int)wd[5], (int)wd[6], (int)wd[7]};
      return v;
    } else if constexpr (CIN == 16) {
      int64_t v0, v1;
      const bool ok0 = tap_in(2 * s, m, v0), ok1 = tap_in(2 * s + 1, m, v1);
      const u32x4 z4 = {0u, 0u, 0u, 0u};
      return join(ok0 ? ld16(A + v0 * 16) : z4, ok1 ? ld16(A + v1 * 16) : z4);
    } else if constexpr (CIN == 32) {
      int64_t v0;
      if (!tap_in(s, m, v0)) return zero32();
      if constexpr (CB == 0) return join(ld16(A + v0 * 32), ld16(A + v0 * 32 + 16));
      else return join(ld16(A + v0 * CA), ld16(B + v0 * CB));  // 16 + 16 stacked
    } else {  // CIN == 64: tap s / 2, channels 32 (s % 2) ..
      int64_t v0;
      if (!tap_in(s >> 1, m, v0)) return zero32();
      const int h = s & 1;
      if constexpr (CB == 0) return join(ld16(A + v0 * 64 + 32 * h), ld16(A + v0 * 64 + 32 * h + 16));
      else {
        const uint8_t* src = h ? B + v0 * CB : A + v0 * CA;  // 32 + 32 stacked
        return join(ld16(src), ld16(src + 16));
      }
    }
  };
  const i32x8* W = (const i32x8*)p.w;  // [NB][NCH][64 lanes]
  auto chunk = [&](int c, i32x8 (&wf)[NB], i32x8 (&xf)[MB]) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) wf[nb] = W[((int64_t)nb * NCH + c) * 64 + lane];
#pragma unroll
    for (int m = 0; m < MB; ++m) xf[m] = xfrag(c, m);
  };
  auto mma = [&](const i32x8 (&wf)[NB], const i32x8 (&xf)[MB]) {
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[m][nb] = mfma8(wf[nb], xf[m], acc[m][nb]);
  };
  // two chunks per pass, the loads of the next chunk before the MFMAs of this
  // one; the loop is not unrolled further (the fragments of all chunks would
  // not fit the registers)
  i32x8 wA[NB], xA[MB], wB[NB], xB[MB];
  chunk(0, wA, xA);
#pragma unroll 1
  for (int c = 0; c < NCH; c += 2) {
    if (c + 1 < NCH) chunk(c + 1, wB, xB);
    mma(wA, xA);
    if (c + 2 < NCH) chunk(c + 2, wA, xA);
    if (c + 1 < NCH) mma(wB, xB);
  }
  if constexpr (EPI == 0) {
    uint8_t* Y = p.y + (int64_t)bt * nvo * COUT;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      if (!vok[m]) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + g * 4;
        unsigned word = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float y = acc[m][nb][q] * (p.wsc[co + q] * p.s_in) + p.bias[co + q];
          if (p.relu) y = fmaxf(y, 0.f);
          word |= e4m3_code(y * p.inv_s_out) << (8 * q);
        }
        *(unsigned*)(Y + vout[m] * COUT + co) = word;
      }
    }
  } else {
    // ReLU, the D0 output on its E4M3 grid, then the 1x1 head over the 16
    // channels held by the 4 lane groups of voxel r
    const double a = p.alpha_override > 0.0 ? p.alpha_override : p.alpha[bt];
    const float f = (float)(p.scale[bt] / a);
    Tv* zo = (Tv*)p.zout + p.off[bt];
    const int co = g * 4;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      float h = 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float y = fmaxf(acc[m][0][q] * (p.wsc[co + q] * p.s_in) + p.bias[co + q], 0.f);
        const float yq = e4m3_value(e4m3_code(y * p.inv_s_out)) * p.s_out;
        h = fmaf(p.wh[co + q], yq, h);
      }
      h += __shfl_xor(h, 16, 64);
      h += __shfl_xor(h, 32, 64);
      const int64_t v = vout[m];
      if (g == 0 && vok[m]) {
        const int ox = (int)(v % n_out), oy = (int)((v / n_out) % n_out), oz = (int)(v / ((int64_t)n_out * n_out));
        const bool bnd = ox == 0 || oy == 0 || oz == 0 || ox == n_out - 1 || oy == n_out - 1 || oz == n_out - 1;
        if (p.all_nodes || !bnd) zo[v] = (Tv)(f * (h + p.bh[0]));
      }
    }
  }
}

// Transposed stride-2 convolution (n_out = 2 n_in - 1): along each axis the
// output o = 2 q + p takes tap 1 from input q when p = 0, and taps 2 from q and
// 0 from q + 1 when p = 1.  A wave owns MB blocks of 16 consecutive input
// voxels q and, for each of the 8 parities p, accumulates over the offsets o
// contained in p (o ascending) times CIN channels: sub-chunk s of parity p is
// offset number s / (CIN / 32), channels 32 (s % (CIN / 32)) .. + 31.
// Weights: [8 parity][CIN / 16 chunks][NB][64 lanes] fragments.
template <int CIN, int COUT>
__global__ void __launch_bounds__(kWaves8 * 64) k_tconv8(Fp8Args p) {
  constexpr int NB = COUT / 16;
  constexpr int HPO = CIN / 32;      // sub-chunks per offset
  constexpr int NCHP = CIN / 16;     // chunk slots per parity (8 offsets)
  constexpr int MB = kMB8;
  const int bt = blockIdx.z;
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  const int n_in = p.n_in, n_out = p.n_out;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, r = lane & 15;
  const int64_t nvi = cube8(n_in), nvo = cube8(n_out);
  const int64_t nn = (int64_t)n_in * n_in;
  const int64_t mb0 = ((int64_t)blockIdx.x * kWaves8 + wave) * MB;
  int qx[MB], qy[MB], qz[MB];
  int64_t vq[MB];
  bool qok[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int64_t v = (mb0 + m) * 16 + r;
    qok[m] = v < nvi;
    const int64_t vv = qok[m] ? v : 0;
    vq[m] = vv;
    qx[m] = (int)(vv % n_in);
    qy[m] = (int)((vv / n_in) % n_in);
    qz[m] = (int)(vv / nn);
  }
  const uint8_t* X = p.a + (int64_t)bt * nvi * CIN;
  uint8_t* Y = p.y + (int64_t)bt * nvo * COUT;
  const i32x8* W = (const i32x8*)p.w;
#pragma unroll
  for (int par = 0; par < 8; ++par) {
    const int px = par & 1, py = (par >> 1) & 1, pz = par >> 2;
    const int nofs = 1 << (px + py + pz);
    const int nch = (nofs * HPO + 3) / 4;
    f32x4 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[m][nb] = {0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < nch; ++c) {
      const int s = 4 * c + g;
      const int oi = s / HPO, h = s - oi * HPO;
      // the oi-th offset contained in par (ascending)
      int o = -1;
      for (int k = 0, cnt = 0; k < 8; ++k)
        if ((k & ~par) == 0) {
          if (cnt == oi) o = k;
          ++cnt;
        }
      const int ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
      i32x8 wf[NB], xf[MB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) wf[nb] = W[(((int64_t)par * NCHP + c) * NB + nb) * 64 + lane];
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        const bool ok = o >= 0 && qok[m] && qx[m] + ox < n_in && qy[m] + oy < n_in && qz[m] + oz < n_in;
        if (ok) {
          const uint8_t* src = X + (vq[m] + ox + oy * (int64_t)n_in + oz * nn) * CIN + 32 * h;
          xf[m] = join(ld16(src), ld16(src + 16));
        } else {
          xf[m] = zero32();
        }
      }
#pragma unroll
      for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[m][nb] = mfma8(wf[nb], xf[m], acc[m][nb]);
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int oxo = 2 * qx[m] + px, oyo = 2 * qy[m] + py, ozo = 2 * qz[m] + pz;
      if (!qok[m] || oxo >= n_out || oyo >= n_out || ozo >= n_out) continue;
      const int64_t vo = ((int64_t)ozo * n_out + oyo) * n_out + oxo;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + g * 4;
        unsigned word = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float y = acc[m][nb][q] * (p.wsc[co + q] * p.s_in) + p.bias[co + q];
          if (p.relu) y = fmaxf(y, 0.f);
          word |= e4m3_code(y * p.inv_s_out) << (8 * q);
        }
        *(unsigned*)(Y + vo * COUT + co) = word;
      }
    }
  }
}

// largest magnitude (non-negative floats compare as unsigned integers)
__global__ void k_amax_f32(const float* __restrict__ x, int64_t n, unsigned* __restrict__ out) {
  float m = 0.f;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(x[k]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// the first layer's input: max over instances and nodes of |z inv_s| and |d|
template <typename Tv>
__global__ void k_amax_x(const Tv* __restrict__ z, const int64_t* __restrict__ off, const double* __restrict__ inv_s,
                         const float* __restrict__ dist, int64_t nv, unsigned* __restrict__ out) {
  const int bt = blockIdx.y;
  const Tv* zb = z + off[bt];
  const float* db = dist + (int64_t)bt * nv;
  const float sc = (float)inv_s[bt];
  float m = 0.f;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nv; k += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fmaxf(fabsf((float)zb[k] * sc), fabsf(db[k])));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void k_zero_u32(unsigned* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// output offsets o contained in parity p, ascending (host)
int parity_offsets(int par, int* o) {
  int cnt = 0;
  for (int k = 0; k < 8; ++k)
    if ((k & ~par) == 0) o[cnt++] = k;
  return cnt;
}

float pow2_scale(float amax) {
  // smallest power of two s with amax / s <= 448 (1 for amax = 0)
  if (!(amax > 0.f)) return 1.f;
  int k = (int)std::ceil(std::log2((double)amax / 448.0));
  while ((double)amax / std::ldexp(1.0, k) > 448.0) ++k;
  while ((double)amax / std::ldexp(1.0, k - 1) <= 448.0) --k;
  return (float)std::ldexp(1.0, k);
}

}  // namespace

// Byte offsets of the E4M3 activations of the layers L0a .. U0 (index = layer)
// in the network scratch, 256-aligned; returns the total.
static int64_t fp8_layout(int batch, int n, int64_t offs[10]) {
  const int n1 = (n + 1) / 2, n2 = (n1 + 1) / 2;
  const int64_t sz[10] = {16 * cube8(n), 16 * cube8(n), 32 * cube8(n1), 32 * cube8(n1), 64 * cube8(n2),
                          64 * cube8(n2), 32 * cube8(n1), 32 * cube8(n1), 16 * cube8(n), 0};
  int64_t o = 0;
  for (int k = 0; k < 10; ++k) {
    offs[k] = o;
    o += (sz[k] * batch + 255) / 256 * 256;
  }
  return o;
}

int64_t fp8_act_bytes(int batch, int n) {
  int64_t offs[10];
  return fp8_layout(batch, n, offs);
}

bool fp8_prepare_weights(CnnState& c, hipStream_t stream) {
  // master weights (already E4M3 x per-channel powers of two) to the host
  int64_t total = 0;
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerSpec& L = kLayers[l];
    total += (int64_t)L.cout * (L.kind == KIND_PT ? 1 : 27) * L.cin + L.cout;
  }
  std::vector<float> w((size_t)total);
  if (hipMemcpyAsync(w.data(), c.w, sizeof(float) * (size_t)total, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return false;
  c.w8_off.assign(kNumLayers, 0);
  c.w8s_off.assign(kNumLayers, 0);
  std::vector<uint8_t> packed;
  std::vector<float> scales;
  for (int l = 0; l < kNumLayers - 1; ++l) {  // the ten 3x3x3 layers
    const LayerSpec& L = kLayers[l];
    const float* W = w.data() + c.w_off[l];
    const int cin = L.cin, cout = L.cout, nb_n = cout / 16;
    c.w8_off[l] = (int64_t)packed.size();
    c.w8s_off[l] = (int64_t)scales.size();
    std::vector<float> sw(cout);
    for (int co = 0; co < cout; ++co) {
      float amax = 0.f;
      for (int k = 0; k < 27 * cin; ++k) amax = std::fmax(amax, std::fabs(W[(int64_t)co * 27 * cin + k]));
      sw[co] = pow2_scale(amax);
      scales.push_back(sw[co]);
    }
    auto code = [&](int co, int tap, int ci) -> uint8_t {
      return (uint8_t)e4m3_code(W[((int64_t)co * 27 + tap) * cin + ci] / sw[co]);
    };
    if (L.kind != KIND_T2) {
      const int nch = (27 * cin + 127) / 128;
      const size_t base = packed.size();
      packed.resize(base + (size_t)nb_n * nch * 64 * 32, 0);
      for (int nb = 0; nb < nb_n; ++nb)
        for (int ch = 0; ch < nch; ++ch)
          for (int lane = 0; lane < 64; ++lane)
            for (int j = 0; j < 32; ++j) {
              const int g = lane >> 4, r = lane & 15;
              const int k = 32 * (4 * ch + g) + j;
              if (k >= 27 * cin) continue;
              packed[base + (((size_t)nb * nch + ch) * 64 + lane) * 32 + j] = code(nb * 16 + r, k / cin, k % cin);
            }
    } else {
      const int hpo = cin / 32, nchp = cin / 16;
      const size_t base = packed.size();
      packed.resize(base + (size_t)8 * nchp * nb_n * 64 * 32, 0);
      for (int par = 0; par < 8; ++par) {
        int ofs[8];
        const int nofs = parity_offsets(par, ofs);
        for (int ch = 0; ch < nchp; ++ch)
          for (int nb = 0; nb < nb_n; ++nb)
            for (int lane = 0; lane < 64; ++lane) {
              const int g = lane >> 4, r = lane & 15;
              const int s = 4 * ch + g, oi = s / hpo, h = s % hpo;
              if (oi >= nofs) continue;
              const int o = ofs[oi];
              // per axis: parity 0 takes tap 1; parity 1 takes tap 2 from offset 0, tap 0 from offset 1
              int t[3];
              for (int ax = 0; ax < 3; ++ax) {
                const int pa = (par >> ax) & 1, oa = (o >> ax) & 1;
                t[ax] = pa ? (oa ? 0 : 2) : 1;
              }
              const int tap = t[2] * 9 + t[1] * 3 + t[0];
              for (int j = 0; j < 32; ++j)
                packed[base + ((((size_t)par * nchp + ch) * nb_n + nb) * 64 + lane) * 32 + j] =
                    code(nb * 16 + r, tap, 32 * h + j);
            }
      }
    }
  }
  if (c.w8) hipFree(c.w8);
  if (c.w8s) hipFree(c.w8s);
  c.w8 = nullptr;
  c.w8s = nullptr;
  if (hipMalloc(&c.w8, packed.size()) != hipSuccess) return false;
  if (hipMalloc(&c.w8s, sizeof(float) * scales.size()) != hipSuccess) return false;
  if (hipMemcpyAsync(c.w8, packed.data(), packed.size(), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(c.w8s, scales.data(), sizeof(float) * scales.size(), hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return false;
  return true;
}

template <typename Tv>
void cnn_apply_fp8(mdnp_sys* s, const Tv* zin, Tv* z, const InstState* st, hipStream_t stream,
                   const double* isc) {
  CnnState& c = s->cnn;
  const int n = s->n, batch = s->n_inst;
  const int n1 = (n + 1) / 2, n2 = (n1 + 1) / 2;
  const int nn[3] = {n, n1, n2};
  int64_t offs[10];
  fp8_layout(batch, n, offs);
  uint8_t* act[10];
  for (int k = 0; k < 10; ++k) act[k] = (uint8_t*)c.act[0] + offs[k];
  const float* sc = c.act8_scale;  // X, L0a, L0b, L1a, L1b, L2a, L2b, U1, D1, U0, D0
  auto args = [&](int layer, int lin, int lout) {
    Fp8Args p;
    p.w = c.w8 + c.w8_off[layer];
    p.wsc = c.w8s + c.w8s_off[layer];
    p.bias = c.w + c.b_off[layer];
    p.n_in = nn[lin];
    p.n_out = nn[lout];
    p.relu = kLayers[layer].relu;
    p.st = st;
    p.want_mode = 0;
    p.inv_s_out = 1.0f / sc[layer + 1];
    return p;
  };
  auto grid = [&](int64_t nvox) {
    return dim3((unsigned)((nvox + 16 * kMB8 * kWaves8 - 1) / (16 * kMB8 * kWaves8)), 1, (unsigned)batch);
  };
  const dim3 blk(kWaves8 * 64);
  {  // L0a from the Krylov vector
    Fp8Args p = args(0, 0, 0);
    p.z = zin;
    p.off = s->d_off;
    p.inv_s = isc;
    p.dist = s->d_dist;
    p.s_in = sc[0];
    p.y = act[0];
    hipLaunchKernelGGL((k_conv8<8, 0, 16, 1, 1, 0, Tv>), grid(cube8(n)), blk, 0, stream, p);
  }
  {  // L0b
    Fp8Args p = args(1, 0, 0);
    p.a = act[0];
    p.s_in = sc[1];
    p.y = act[1];
    hipLaunchKernelGGL((k_conv8<16, 0, 16, 1, 0, 0, Tv>), grid(cube8(n)), blk, 0, stream, p);
  }
  {  // L1a (stride 2)
    Fp8Args p = args(2, 0, 1);
    p.a = act[1];
    p.s_in = sc[2];
    p.y = act[2];
    hipLaunchKernelGGL((k_conv8<16, 0, 32, 2, 0, 0, Tv>), grid(cube8(n1)), blk, 0, stream, p);
  }
  {  // L1b
    Fp8Args p = args(3, 1, 1);
    p.a = act[2];
    p.s_in = sc[3];
    p.y = act[3];
    hipLaunchKernelGGL((k_conv8<32, 0, 32, 1, 0, 0, Tv>), grid(cube8(n1)), blk, 0, stream, p);
  }
  {  // L2a (stride 2)
    Fp8Args p = args(4, 1, 2);
    p.a = act[3];
    p.s_in = sc[4];
    p.y = act[4];
    hipLaunchKernelGGL((k_conv8<32, 0, 64, 2, 0, 0, Tv>), grid(cube8(n2)), blk, 0, stream, p);
  }
  {  // L2b
    Fp8Args p = args(5, 2, 2);
    p.a = act[4];
    p.s_in = sc[5];
    p.y = act[5];
    hipLaunchKernelGGL((k_conv8<64, 0, 64, 1, 0, 0, Tv>), grid(cube8(n2)), blk, 0, stream, p);
  }
  {  // U1 (transposed)
    Fp8Args p = args(6, 2, 1);
    p.a = act[5];
    p.s_in = sc[6];
    p.y = act[6];
    hipLaunchKernelGGL((k_tconv8<64, 32>), grid(cube8(n2)), blk, 0, stream, p);
  }
  {  // D1 on [U1 | L1b] (one scale for the pair)
    Fp8Args p = args(7, 1, 1);
    p.a = act[6];
    p.b = act[3];
    p.s_in = sc[7];
    p.y = act[7];
    hipLaunchKernelGGL((k_conv8<32, 32, 32, 1, 0, 0, Tv>), grid(cube8(n1)), blk, 0, stream, p);
  }
  {  // U0 (transposed)
    Fp8Args p = args(8, 1, 0);
    p.a = act[7];
    p.s_in = sc[8];
    p.y = act[8];
    hipLaunchKernelGGL((k_tconv8<32, 16>), grid(cube8(n1)), blk, 0, stream, p);
  }
  {  // D0 on [U0 | L0b], the head and the unscaling
    Fp8Args p = args(9, 0, 0);
    p.a = act[8];
    p.b = act[1];
    p.s_in = sc[9];
    p.s_out = sc[10];
    p.wh = c.w + c.w_off[10];
    p.bh = c.w + c.b_off[10];
    p.zout = z;
    p.off = s->d_off;
    p.alpha = s->d_alpha;
    p.alpha_override = s->alpha_override;
    p.scale = isc + s->n_inst;
    p.all_nodes = s->neumann ? 1 : 0;
    hipLaunchKernelGGL((k_conv8<16, 16, 16, 1, 0, 1, Tv>), grid(cube8(n)), blk, 0, stream, p);
  }
}
template void cnn_apply_fp8<float>(mdnp_sys*, const float*, float*, const InstState*, hipStream_t, const double*);
template void cnn_apply_fp8<double>(mdnp_sys*, const double*, double*, const InstState*, hipStream_t,
                                    const double*);

void fp8_zero_amax(unsigned* d_amax, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, d_amax, 11);
}

template <typename Tv>
void fp8_record_amax(mdnp_sys* s, const Tv* zin, const double* isc, void* const act[12], unsigned* d_amax,
                     hipStream_t stream) {
  const int n = s->n, batch = s->n_inst;
  const int n1 = (n + 1) / 2, n2 = (n1 + 1) / 2;
  hipLaunchKernelGGL((k_amax_x<Tv>), dim3(64, (unsigned)batch), dim3(256), 0, stream, zin, s->d_off, isc, s->d_dist,
                     cube8(n), d_amax);
  // FP32 outputs of L0a .. D0 in act[1] .. act[10]
  const int chans[10] = {16, 16, 32, 32, 64, 64, 32, 32, 16, 16};
  const int lvl[10] = {0, 0, 1, 1, 2, 2, 1, 1, 0, 0};
  const int nn[3] = {n, n1, n2};
  for (int l = 0; l < 10; ++l) {
    const int64_t cnt = (int64_t)batch * cube8(nn[lvl[l]]) * chans[l];
    hipLaunchKernelGGL(k_amax_f32, dim3(512), dim3(256), 0, stream, (const float*)act[l + 1], cnt, d_amax + 1 + l);
  }
}
template void fp8_record_amax<float>(mdnp_sys*, const float*, const double*, void* const[12], unsigned*,
                                     hipStream_t);
template void fp8_record_amax<double>(mdnp_sys*, const double*, const double*, void* const[12], unsigned*,
                                      hipStream_t);

void fp8_scales_from_amax(const float amax_in[11], float out[11]) {
  float amax[11];
  for (int k = 0; k < 11; ++k) amax[k] = amax_in[k];
  // stacked pairs share one scale: (L1b, U1) = (4, 7), (L0b, U0) = (2, 9)
  const int tied[2][2] = {{4, 7}, {2, 9}};
  for (const auto& t : tied) amax[t[0]] = amax[t[1]] = std::fmax(amax[t[0]], amax[t[1]]);
  for (int k = 0; k < 11; ++k) out[k] = pow2_scale(2.0f * amax[k]);
}

}  // namespace mdnp
