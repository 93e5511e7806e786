// The U-net preconditioner of Section 4.2 (three levels, 16/32/64 channels,
// 3x3x3 kernels, stride-2 convolutions down, stride-2 transposed convolutions
// up, skip connections by channel stacking) and its training objective of
// Section 5.1, on channels-last [batch][z][y][x][channel] activations.
//
// This file holds the direct (non-MFMA) kernels: FP32 arithmetic on FP32 or
// BF16 storage, used for the FP32 network, for the first and last layers of
// every network, for the backward pass, the loss and Adam.  The matrix-core
// kernels of the BF16 network live in conv_mfma.hip.
#include <cmath>
#include <mutex>
#include <type_traits>

#include "conv_common.hpp"
#include "kernels.hpp"

namespace mdnp {

namespace {

constexpr int BS = 256;

__device__ __forceinline__ float ld(const float* p) { return *p; }
__device__ __forceinline__ float ld(const bf16* p) { return __bfloat162float(*p); }
typedef float f32x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_(float* p, float v) { *p = v; }
__device__ __forceinline__ void st_(bf16* p, float v) { *p = __float2bfloat16(v); }

__device__ __forceinline__ bool is_bnd(int r, int n) {
  int i = r % n, j = (r / n) % n, k = r / (n * n);
  return i == 0 || j == 0 || k == 0 || i == n - 1 || j == n - 1 || k == n - 1;
}

// Input voxel of output voxel o for tap t along one axis, or -1.
template <int MODE>
__device__ __forceinline__ int in_coord(int o, int t, int n_in) {
  if (MODE == KIND_S1) {
    int i = o + t - 1;
    return (i >= 0 && i < n_in) ? i : -1;
  } else if (MODE == KIND_S2) {
    int i = 2 * o + t - 1;
    return (i >= 0 && i < n_in) ? i : -1;
  } else if (MODE == KIND_T2) {
    int num = o + 1 - t;
    if (num < 0 || (num & 1)) return -1;
    int i = num >> 1;
    return i < n_in ? i : -1;
  } else {
    return o;
  }
}

// Direct convolution: one thread per output voxel, CO output channels per block
// row; weights [taps][cin][cout] read with block-uniform addresses.
template <typename Tin, typename Tout, int MODE, int CO>
__global__ void __launch_bounds__(BS) k_conv(ConvP p) {
  const int64_t nvox = (int64_t)p.n_out * p.n_out * p.n_out;
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int co0 = blockIdx.y * CO;
  const int bt = blockIdx.z;
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  if (v >= nvox) return;
  const int ox = (int)(v % p.n_out), oy = (int)((v / p.n_out) % p.n_out), oz = (int)(v / ((int64_t)p.n_out * p.n_out));
  const int cin = p.ca + p.cb;
  float acc[CO];
#pragma unroll
  for (int c = 0; c < CO; ++c) acc[c] = p.bias ? p.bias[co0 + c] : 0.0f;
  const Tin* A = (const Tin*)p.a + (int64_t)bt * p.a_bs;
  const Tin* B = (const Tin*)p.b + (int64_t)bt * p.b_bs;
  const int ntap = (MODE == KIND_PT) ? 1 : 27;
  for (int t = 0; t < ntap; ++t) {
    const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
    const int iz = in_coord<MODE>(oz, tz, p.n_in);
    const int iy = in_coord<MODE>(oy, ty, p.n_in);
    const int ix = in_coord<MODE>(ox, tx, p.n_in);
    if (iz < 0 || iy < 0 || ix < 0) continue;
    const int64_t vin = ((int64_t)iz * p.n_in + iy) * p.n_in + ix;
    const float* wt = p.wt + (int64_t)t * cin * p.cout + co0;
    const Tin* xa = A + vin * p.lda;
    for (int ci = 0; ci < p.ca; ++ci) {
      const float x = ld(xa + ci);
      const float* w = wt + (int64_t)ci * p.cout;
#pragma unroll
      for (int c = 0; c < CO; ++c) acc[c] = fmaf(w[c], x, acc[c]);
    }
    if (p.cb) {
      const Tin* xb = B + vin * p.ldb;
      for (int ci = 0; ci < p.cb; ++ci) {
        const float x = ld(xb + ci);
        const float* w = wt + (int64_t)(p.ca + ci) * p.cout;
#pragma unroll
        for (int c = 0; c < CO; ++c) acc[c] = fmaf(w[c], x, acc[c]);
      }
    }
  }
  Tout* y = (Tout*)p.y + (int64_t)bt * p.y_bs + v * p.ldy + p.y_choff + co0;
#pragma unroll
  for (int c = 0; c < CO; ++c) {
    float r = acc[c];
    if (p.relu) r = fmaxf(r, 0.0f);
    if (p.accumulate) r += ld(y + c);
    st_(y + c, r);
  }
}

// First layer inside the solver: input channel 0 = z0 * inv_s (3D part of a
// Krylov vector), channel 1 = distance field; 2 -> 16, ReLU.
template <typename Tv, typename Tout>
__global__ void __launch_bounds__(BS) k_conv_in0(const Tv* __restrict__ z, const int64_t* off,
                                                 const double* inv_s, const float* __restrict__ dist,
                                                 const float* __restrict__ wt, const float* __restrict__ bias,
                                                 int n, Tout* __restrict__ y, const InstState* st) {
  const int64_t nvox = (int64_t)n * n * n;
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int i = blockIdx.z;
  if (st && !(st[i].active && st[i].mode == 0)) return;
  if (v >= nvox) return;
  const int ox = (int)(v % n), oy = (int)((v / n) % n), oz = (int)(v / ((int64_t)n * n));
  const float sc = (float)inv_s[i];
  const Tv* zi = z + off[i];
  const float* di = dist + (int64_t)i * nvox;
  float acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = bias[c];
  for (int t = 0; t < 27; ++t) {
    const int iz = oz + t / 9 - 1, iy = oy + (t / 3) % 3 - 1, ix = ox + t % 3 - 1;
    if (iz < 0 || iy < 0 || ix < 0 || iz >= n || iy >= n || ix >= n) continue;
    const int64_t vin = ((int64_t)iz * n + iy) * n + ix;
    const float x0 = (float)zi[vin] * sc;
    const float x1 = di[vin];
    const float* w = wt + t * 2 * 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = fmaf(w[c], x0, fmaf(w[16 + c], x1, acc[c]));
  }
  Tout* yo = y + ((int64_t)i * nvox + v) * 16;
#pragma unroll
  for (int c = 0; c < 16; ++c) st_(yo + c, fmaxf(acc[c], 0.0f));
}

// Last layer inside the solver: 1x1 16 -> 1, then z0 = s / alpha * U on the free
// nodes (with the Dirichlet condition, boundary nodes are left alone; with the
// natural one, all_nodes = 1, every node is free).
template <typename Tv, typename Tin>
__global__ void __launch_bounds__(BS) k_head_out(const Tin* __restrict__ d0, const float* __restrict__ wt,
                                                 const float* __restrict__ bias, int n, Tv* __restrict__ z,
                                                 const int64_t* off, const double* alpha, double alpha_override,
                                                 const double* scale, const InstState* st, int all_nodes) {
  const int64_t nvox = (int64_t)n * n * n;
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int i = blockIdx.z;
  if (st && !(st[i].active && st[i].mode == 0)) return;
  if (v >= nvox) return;
  if (!all_nodes && is_bnd((int)v, n)) return;
  const Tin* x = d0 + ((int64_t)i * nvox + v) * 16;
  float out = bias[0];
#pragma unroll
  for (int c = 0; c < 16; ++c) out = fmaf(wt[c], ld(x + c), out);
  const double a = alpha_override > 0.0 ? alpha_override : alpha[i];
  const double s = scale[i];
  z[off[i] + v] = (Tv)((s / a) * (double)out);
}

// Weight copies: forward [taps][cin][cout]; adjoint [taps][cout][cin] with the
// taps reversed for the stride-1 convolution (the transpose of a correlation
// is the correlation with the flipped kernel).
__global__ void k_wt_fwd(const float* __restrict__ w, float* __restrict__ wt, int cout, int taps, int cin) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)cout * taps * cin;
  if (k >= tot) return;
  const int co = (int)(k / ((int64_t)taps * cin));
  const int t = (int)((k / cin) % taps);
  const int ci = (int)(k % cin);
  wt[((int64_t)t * cin + ci) * cout + co] = w[k];
}

__global__ void k_wt_adj(const float* __restrict__ w, float* __restrict__ wt, int cout, int taps, int cin, int flip) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)cout * taps * cin;
  if (k >= tot) return;
  const int co = (int)(k / ((int64_t)taps * cin));
  const int t = (int)((k / cin) % taps);
  const int ci = (int)(k % cin);
  const int tt = flip ? taps - 1 - t : t;
  // adjoint layer: input channels = cout, output channels = cin
  wt[((int64_t)tt * cout + co) * cin + ci] = w[k];
}

__global__ void k_wt_adj_split(const float* __restrict__ w, float* __restrict__ w1, float* __restrict__ w2,
                               int cout, int taps, int cin, int ca, int flip) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)cout * taps * cin;
  if (k >= tot) return;
  const int co = (int)(k / ((int64_t)taps * cin));
  const int t = (int)((k / cin) % taps);
  const int ci = (int)(k % cin);
  const int tt = flip ? taps - 1 - t : t;
  const int cb = cin - ca;
  if (ci < ca) w1[((int64_t)tt * cout + co) * ca + ci] = w[k];
  else w2[((int64_t)tt * cout + co) * cb + (ci - ca)] = w[k];
}

__global__ void k_relu_mask(float* __restrict__ g, const void* __restrict__ out, int out_is_bf16, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float o = out_is_bf16 ? __bfloat162float(((const bf16*)out)[k]) : ((const float*)out)[k];
  if (!(o > 0.0f)) g[k] = 0.0f;
}

// Weight gradient on v_mfma_f32_16x16x4_f32 (FP32 products and sums) for
// layers whose channel counts are multiples of 16.  An element is an output
// voxel of one instance (an input voxel for the transposed convolution, whose
// output o = 2 i + t - 1 then depends on the tap).  A wave owns NTG tap
// groups (the taps with one tz: 9 each; the 1x1 layer has one tap), NBO x NBI
// tiles of 16 x 16 (co, ci) and a range of elements.  Per step of 4 elements
// lane l holds element l / 16 and channel l % 16: the operand fixed over the
// taps (dz for the stride-1/2 and 1x1 layers, x for the transposed one) is
// loaded once, the other per tap, and the MFMA of tap t and tile (bo, bi) adds
// D[co][ci] += sum over the 4 elements of dz[e][co] x[in(e, t)][ci] (lane l
// ends with co = 4 (l / 16) .. + 3, ci = l % 16).  The element's input
// coordinates and their bounds are worked out once per step; a tap adds a
// constant offset.  Partial tiles go to part [split][cout][27 or 1][cin] and
// are summed in a second kernel.
template <typename Tin, int MODE, int NTG, int NBO, int NBI>
__global__ void __launch_bounds__(64) k_dw_m(const float* __restrict__ dz, int cout, const void* xa_, int ca,
                                             int lda, const void* xb_, int cb, int ldb, int n_in, int n_out,
                                             int batch, int64_t a_bs, int64_t b_bs, float* __restrict__ part,
                                             int nsplit) {
  constexpr int TPG = MODE == KIND_PT ? 1 : 9;   // taps per group
  constexpr int NTAP = MODE == KIND_PT ? 1 : 27;
  constexpr int NT = NTG * TPG;                  // taps of this wave
  const int cin = ca + cb;
  const int nbi = cin / (16 * NBI);
  const int nwt = (cout / (16 * NBO)) * nbi;     // tile groups
  const int tgw = blockIdx.x / nwt, tl = blockIdx.x - tgw * nwt;
  const int co0 = (tl / nbi) * 16 * NBO, ci0 = (tl % nbi) * 16 * NBI;
  const int tz0 = tgw * NTG;                     // first tz of this wave
  const int split = blockIdx.z;
  const int lane = threadIdx.x;
  const int ke = lane >> 4, c = lane & 15;
  const int nvo = n_out * n_out * n_out, nvi = n_in * n_in * n_in;
  const int nit = MODE == KIND_T2 ? nvi : nvo;   // elements per instance
  const int total = nit * batch;
  const int per = ((total + nsplit - 1) / nsplit + 7) & ~7;
  const int e0 = split * per, e1 = min(total, e0 + per);
  // the input channel of this lane in each ci tile (a 16-channel tile lies in one source)
  const Tin* xs[NBI];
  int xl[NBI];
  int64_t xbsv[NBI];
#pragma unroll
  for (int bi = 0; bi < NBI; ++bi) {
    const int cib = ci0 + 16 * bi;
    const bool in_a = cib < ca;
    xs[bi] = (const Tin*)(in_a ? xa_ : xb_) + (in_a ? cib : cib - ca) + c;
    xl[bi] = in_a ? lda : ldb;
    xbsv[bi] = in_a ? a_bs : b_bs;
  }
  const float* dzc = dz + co0 + c;
  f32x4v acc[NT][NBO][NBI];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int bo = 0; bo < NBO; ++bo)
#pragma unroll
      for (int bi = 0; bi < NBI; ++bi) acc[t][bo][bi] = f32x4v{0.f, 0.f, 0.f, 0.f};
  // one step of 4 elements: raw operands as loaded (every load is issued, at a
  // valid address; entries outside the grid or the range are zeroed by the
  // mask when the MFMAs use them), so that the loads of the next step stay in
  // flight while this step's MFMAs run
  constexpr bool T2 = MODE == KIND_T2;
  // x as stored (BF16 bits or FP32): converted only when used, so that no
  // instruction waits for a load before the MFMAs need it
  typedef typename std::conditional<std::is_same<Tin, bf16>::value, unsigned short, float>::type XRaw;
  auto xf = [](XRaw r) -> float {
    if constexpr (std::is_same<XRaw, float>::value) return r;
    else return __uint_as_float((unsigned)r << 16);
  };
  struct Step {
    float d[T2 ? NT : 1][NBO];   // dz: per tap (transposed layer) or per element
    XRaw x[T2 ? 1 : NT][NBI];    // x: per element (transposed layer) or per tap
    unsigned ok;                 // bit t: tap t inside; bit 31: element inside
  };
  auto load = [&](int eb, Step& st) {
    const int e = eb + ke;
    const bool eok = e < e1;
    const int ee = eok ? e : e0;
    const int bt = ee / nit, u = ee - bt * nit;
    const float* dzb = dzc + (int64_t)bt * nvo * cout;
    unsigned ok = eok ? 0x80000000u : 0u;
    if constexpr (T2) {
      const int ix = u % n_in, iy = (u / n_in) % n_in, iz = u / (n_in * n_in);
#pragma unroll
      for (int bi = 0; bi < NBI; ++bi) st.x[0][bi] = *(const XRaw*)(xs[bi] + (int64_t)bt * xbsv[bi] + (int64_t)u * xl[bi]);
      const int ox0 = 2 * ix - 1, oy0 = 2 * iy - 1, oz0 = 2 * iz - 1;
      const int obase = (oz0 * n_out + oy0) * n_out + ox0;
      unsigned bx = 0, by = 0, bz = 0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        bx |= (ox0 + d >= 0 && ox0 + d < n_out) ? 1u << d : 0u;
        by |= (oy0 + d >= 0 && oy0 + d < n_out) ? 1u << d : 0u;
        bz |= (oz0 + d >= 0 && oz0 + d < n_out) ? 1u << d : 0u;
      }
#pragma unroll
      for (int g = 0; g < NTG; ++g) {
        const int tz = tz0 + g;
#pragma unroll
        for (int t9 = 0; t9 < 9; ++t9) {
          const int ty = t9 / 3, tx = t9 % 3;
          const bool in = (bz >> tz) & (by >> ty) & (bx >> tx) & 1u;
          const int off = in ? obase + (tz * n_out + ty) * n_out + tx : 0;
          ok |= in ? 1u << (g * 9 + t9) : 0u;
#pragma unroll
          for (int bo = 0; bo < NBO; ++bo) st.d[g * 9 + t9][bo] = dzb[(int64_t)off * cout + 16 * bo];
        }
      }
    } else {
      const int ox = u % n_out, oy = (u / n_out) % n_out, oz = u / (n_out * n_out);
#pragma unroll
      for (int bo = 0; bo < NBO; ++bo) st.d[0][bo] = dzb[(int64_t)u * cout + 16 * bo];
      constexpr int S = MODE == KIND_S2 ? 2 : 1;
      constexpr int SH = MODE == KIND_PT ? 0 : 1;  // tap offset of the first tap
      const int ix0 = S * ox - SH, iy0 = S * oy - SH, iz0 = S * oz - SH;
      const int ibase = (iz0 * n_in + iy0) * n_in + ix0;
      unsigned bx = 0, by = 0, bz = 0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        bx |= (ix0 + d >= 0 && ix0 + d < n_in) ? 1u << d : 0u;
        by |= (iy0 + d >= 0 && iy0 + d < n_in) ? 1u << d : 0u;
        bz |= (iz0 + d >= 0 && iz0 + d < n_in) ? 1u << d : 0u;
      }
#pragma unroll
      for (int g = 0; g < NTG; ++g) {
        const int tz = tz0 + g;
#pragma unroll
        for (int t9 = 0; t9 < TPG; ++t9) {
          const int ty = t9 / 3, tx = t9 % 3;
          const bool in = (bz >> tz) & (by >> ty) & (bx >> tx) & 1u;
          const int off = in ? ibase + (tz * n_in + ty) * n_in + tx : 0;
          ok |= in ? 1u << (g * TPG + t9) : 0u;
#pragma unroll
          for (int bi = 0; bi < NBI; ++bi)
            st.x[g * TPG + t9][bi] = *(const XRaw*)(xs[bi] + (int64_t)bt * xbsv[bi] + (int64_t)off * xl[bi]);
        }
      }
    }
    st.ok = ok;
  };
  auto mma = [&](const Step& st) {
    const bool eok = st.ok >> 31;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bool in = (st.ok >> t) & 1u;
#pragma unroll
      for (int bo = 0; bo < NBO; ++bo)
#pragma unroll
        for (int bi = 0; bi < NBI; ++bi) {
          // the element's own operand is zeroed outside the range, the tap's outside the grid
          const float a = T2 ? (in ? st.d[t][bo] : 0.0f) : (eok ? st.d[0][bo] : 0.0f);
          const float b = T2 ? (eok ? xf(st.x[0][bi]) : 0.0f) : (in ? xf(st.x[t][bi]) : 0.0f);
          acc[t][bo][bi] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t][bo][bi], 0, 0, 0);
        }
    }
  };
  // two steps per pass (the range is a multiple of 8 elements), each step's
  // loads issued before the previous step's MFMAs
  if (e0 < e1) {
    Step sa, sb;
    load(e0, sa);
    for (int eb = e0; eb < e1; eb += 8) {
      load(eb + 4, sb);
      __builtin_amdgcn_sched_barrier(0);
      mma(sa);
      __builtin_amdgcn_sched_barrier(0);
      load(eb + 8, sa);
      __builtin_amdgcn_sched_barrier(0);
      mma(sb);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // part layout [split][cout][ntap][cin]; lane: co = co0 + 16 bo + 4 ke + q, ci = ci0 + 16 bi + c
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int tap = tz0 * TPG + t;
#pragma unroll
    for (int bo = 0; bo < NBO; ++bo)
#pragma unroll
      for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int co = co0 + 16 * bo + 4 * ke + q;
          part[(((int64_t)split * cout + co) * NTAP + tap) * cin + ci0 + 16 * bi + c] = acc[t][bo][bi][q];
        }
  }
}

// Weight gradient of the first layer (2 FP32 input channels, 16 outputs,
// stride 1) on the same MFMA: the 54 (tap, input channel) pairs are the
// columns of four 16-wide tiles (column j: tap j / 2, channel j % 2; columns
// 54 .. 63 stay zero), dz[e][co] the rows.
__global__ void __launch_bounds__(64) k_dw_first(const float* __restrict__ dz, const float* __restrict__ x, int n,
                                                 int batch, float* __restrict__ part, int nsplit) {
  const int lane = threadIdx.x;
  const int ke = lane >> 4, c = lane & 15;
  const int nv = n * n * n, total = nv * batch;
  const int per = ((total + nsplit - 1) / nsplit + 3) & ~3;
  const int split = blockIdx.x;
  const int e0 = split * per, e1 = min(total, e0 + per);
  // this lane's column in each tile: tap offsets and channel
  int toff[4], tci[4], tmask[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int j = 16 * nt + c, tap = j >> 1;
    const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
    toff[nt] = ((tz - 1) * n + (ty - 1)) * n + (tx - 1);
    tci[nt] = j & 1;
    tmask[nt] = tap < 27 ? (1 << (tz * 9 + ty * 3 + tx)) : 0;
  }
  f32x4v acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4v{0.f, 0.f, 0.f, 0.f};
  for (int eb = e0; eb < e1; eb += 4) {
    const int e = eb + ke;
    const bool eok = e < e1;
    const int ee = eok ? e : e0;
    const int bt = ee / nv, u = ee - bt * nv;
    const int ox = u % n, oy = (u / n) % n, oz = u / (n * n);
    // taps inside the grid as a 27-bit mask
    unsigned in = 0;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int ix = ox + t % 3 - 1, iy = oy + (t / 3) % 3 - 1, iz = oz + t / 9 - 1;
      in |= (ix >= 0 && iy >= 0 && iz >= 0 && ix < n && iy < n && iz < n) ? 1u << t : 0u;
    }
    const float dv = eok ? dz[((int64_t)bt * nv + u) * 16 + c] : 0.0f;
    const float* xb = x + (int64_t)bt * nv * 2;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const bool ok = eok && (in & (unsigned)tmask[nt]);
      const float xv = ok ? xb[(int64_t)(u + toff[nt]) * 2 + tci[nt]] : 0.0f;
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(dv, xv, acc[nt], 0, 0, 0);
    }
  }
  // part layout [split][16][27][2]
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int j = 16 * nt + c;
    if (j >= 54) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int co = 4 * ke + q;
      part[(((int64_t)split * 16 + co) * 27 + (j >> 1)) * 2 + (j & 1)] = acc[nt][q];
    }
  }
}

// Bias gradient (x = nullptr) or weight gradient of the 1x1 head with one
// output (x: [rows][cin]), first pass: block b sums its row range per channel,
// sum of dz[r][co] (bias; cout <= 64) or of dz[r] x[r][ci] (head), into part[b][.].
template <typename Tin>
__global__ void __launch_bounds__(256) k_rows_part(const float* __restrict__ dz, const Tin* __restrict__ x, int nch,
                                                   int64_t nrows, float* __restrict__ part) {
  __shared__ float sh[256];
  const int64_t per = (nrows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(nrows, r0 + per);
  const int ch = threadIdx.x % nch, rs = threadIdx.x / nch, nrs = 256 / nch;
  float s = 0.0f;
  if (x) {
    for (int64_t r = r0 + rs; r < r1; r += nrs) s = fmaf(dz[r], ld(x + r * nch + ch), s);
  } else {
    for (int64_t r = r0 + rs; r < r1; r += nrs) s += dz[r * nch + ch];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < nch) {
    float t = 0.0f;
    for (int k = 0; k < nrs; ++k) t += sh[k * nch + threadIdx.x];
    part[(int64_t)blockIdx.x * nch + threadIdx.x] = t;
  }
}

// out[k] = sum over q of part[q][k] (q ascending per split lane, then the 8
// lanes in order): 32 consecutive k per block, 8 split lanes.
__global__ void __launch_bounds__(256) k_sum_parts(const float* __restrict__ part, float* __restrict__ out,
                                                   int64_t n, int nsplit) {
  __shared__ float sh[8][32];
  const int kx = threadIdx.x & 31, sq = threadIdx.x >> 5;
  const int64_t k = (int64_t)blockIdx.x * 32 + kx;
  float s = 0.0f;
  if (k < n)
    for (int q = sq; q < nsplit; q += 8) s += part[(int64_t)q * n + k];
  sh[sq][kx] = s;
  __syncthreads();
  if (sq == 0 && k < n) {
    float t = sh[0][kx];
    for (int j = 1; j < 8; ++j) t += sh[j][kx];
    out[k] = t;
  }
}



// ---------------------------------------------------------------- training objective

// The network output on the free nodes: zero on the Dirichlet boundary (none
// is fixed under the natural condition, dirichlet = 0).
__global__ void __launch_bounds__(BS) k_mask_bnd(const float* __restrict__ u, float* __restrict__ um, int n,
                                                 int64_t n3d, int dirichlet) {
  const int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int slot = blockIdx.y;
  if (k >= n3d) return;
  const int64_t g = (int64_t)slot * n3d + k;
  um[g] = dirichlet && is_bnd((int)k, n) ? 0.0f : u[g];
}

// e = r - Cu / alpha, partial sums of e^2 (one row of partials per slot).
__global__ void __launch_bounds__(BS) k_loss_e(const float* __restrict__ r, float* __restrict__ cu_e,
                                               const int32_t* inst, const double* alpha, int64_t n3d,
                                               double* __restrict__ part, int nbx) {
  __shared__ double sh[BS / 64];
  const int slot = blockIdx.y;
  const double ia = 1.0 / alpha[inst[slot]];
  double loc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x; k < n3d; k += (int64_t)nbx * BS) {
    const int64_t g = (int64_t)slot * n3d + k;
    const double e = (double)r[g] - (double)cu_e[g] * ia;
    cu_e[g] = (float)e;
    loc += e * e;
  }
  // block sum
  for (int o = 32; o > 0; o >>= 1) loc += __shfl_xor(loc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = loc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < BS / 64; ++w) t += sh[w];
    part[(int64_t)slot * nbx + blockIdx.x] = t;
  }
}

__global__ void k_loss_sum(const double* part, int nbx, int n_slots, double* loss) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_slots) return;
  double t = 0.0;
  for (int b = 0; b < nbx; ++b) t += part[(int64_t)s * nbx + b];
  loss[s] = t;
}

// du = -2 C e / alpha on the free nodes, 0 on the Dirichlet nodes.
__global__ void __launch_bounds__(BS) k_loss_grad_fin(const float* __restrict__ ce, float* __restrict__ du,
                                                      const int32_t* inst, const double* alpha, int n,
                                                      int64_t n3d, int dirichlet) {
  const int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int slot = blockIdx.y;
  if (k >= n3d) return;
  const int64_t g = (int64_t)slot * n3d + k;
  du[g] = dirichlet && is_bnd((int)k, n) ? 0.0f : (float)(-2.0 * (double)ce[g] / alpha[inst[slot]]);
}

__global__ void __launch_bounds__(BS) k_pack_input(const float* __restrict__ r, const float* __restrict__ dist,
                                                   const int32_t* inst, int64_t n3d, float* __restrict__ x) {
  const int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int slot = blockIdx.y;
  if (k >= n3d) return;
  const int64_t g = (int64_t)slot * n3d + k;
  x[2 * g] = r[g];
  x[2 * g + 1] = dist[(int64_t)inst[slot] * n3d + k];
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

}  // namespace

// ---------------------------------------------------------------- host side

int64_t cnn_layer_count() { return kNumLayers; }

static inline int64_t cube(int n) { return (int64_t)n * n * n; }

// ---------------------------------------------------------------- FP8 (E4M3) weights

// Nearest E4M3 value of v (1 sign, 4 exponent bits with bias 7, 3 mantissa
// bits, subnormals down to 2^-9, largest finite 448), ties to even, saturating
// at +-448: the quantum of the binade of |v| (at least that of the
// subnormals, 2^-9) is a power of two, so scaling by it and rounding to an
// integer in the default round-to-nearest-even mode is exact.
__device__ __forceinline__ float round_e4m3(float v) {
  const float a = fabsf(v);
  if (a >= 448.0f) return copysignf(448.0f, v);
  int e;
  (void)frexpf(a, &e);                       // a = f 2^e, f in [0.5, 1): binade 2^(e - 1)
  const int qe = max(e - 1, -6) - 3;         // quantum 2^qe
  return copysignf(ldexpf(rintf(ldexpf(a, -qe)), qe), v);
}

// One workgroup per output channel of one layer (its taps x cin weights,
// contiguous): the scale is the smallest power of two 2^k with
// amax / 2^k <= 448 = 0.875 * 2^9, then w = round_e4m3(w / 2^k) * 2^k in place.
__global__ void __launch_bounds__(256) k_quant_e4m3(float* __restrict__ w, int nper) {
  __shared__ float red[4];
  float* row = w + (int64_t)blockIdx.x * nper;
  float a = 0.0f;
  for (int k = threadIdx.x; k < nper; k += 256) a = fmaxf(a, fabsf(row[k]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a = fmaxf(a, __shfl_xor(a, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  const float amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  int k = 0;
  if (amax > 0.0f) {
    int e;
    const float f = frexpf(amax, &e);
    k = f <= 0.875f ? e - 9 : e - 8;
  }
  for (int q = threadIdx.x; q < nper; q += 256) row[q] = ldexpf(round_e4m3(ldexpf(row[q], -k)), k);
}

void cnn_quantize_e4m3(float* d_w, hipStream_t stream) {
  int64_t off = 0;
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerSpec& L = kLayers[l];
    const int taps = L.kind == KIND_PT ? 1 : 27;
    const int nper = taps * L.cin;
    hipLaunchKernelGGL(k_quant_e4m3, dim3((unsigned)L.cout), dim3(256), 0, stream, d_w + off, nper);
    off += (int64_t)L.cout * nper + L.cout;  // weights [cout][taps][cin], then the biases
  }
}

void cnn_prepare_weights(CnnState& c, const float* d_w, hipStream_t stream) {
  int64_t off = 0, toff = 0;
  c.w_off.assign(kNumLayers, 0);
  c.b_off.assign(kNumLayers, 0);
  c.wt_off.assign(kNumLayers, 0);
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerSpec& L = kLayers[l];
    const int taps = L.kind == KIND_PT ? 1 : 27;
    const int64_t nw = (int64_t)L.cout * taps * L.cin;
    c.w_off[l] = off;
    c.b_off[l] = off + nw;
    c.wt_off[l] = toff;
    off += nw + L.cout;
    toff += nw;
  }
  if (!c.wt) hipMalloc(&c.wt, sizeof(float) * (size_t)toff);
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerSpec& L = kLayers[l];
    const int taps = L.kind == KIND_PT ? 1 : 27;
    const int64_t nw = (int64_t)L.cout * taps * L.cin;
    hipLaunchKernelGGL(k_wt_fwd, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, stream, d_w + c.w_off[l],
                       c.wt + c.wt_off[l], L.cout, taps, L.cin);
  }
  cnn_prepare_mfma_weights(c, d_w, stream);
}

// Offsets of the saved tensors (bytes, 256-aligned) in the order
// X a0 s0 a1 s1 a2 b2 u1 d1 u0 d0 y.
// offs[12] receives the total size.
void saved_layout(int batch, int n, mdnp_dtype dtype, int64_t offs[13]) {
  const int n1 = (n + 1) / 2, n2 = (n1 + 1) / 2;
  const int64_t es = dtype == MDNP_BF16 ? 2 : 4;
  const int64_t sz[12] = {4 * batch * cube(n) * 2, es * batch * cube(n) * 16, es * batch * cube(n) * 16,
                          es * batch * cube(n1) * 32, es * batch * cube(n1) * 32, es * batch * cube(n2) * 64,
                          es * batch * cube(n2) * 64, es * batch * cube(n1) * 32, es * batch * cube(n1) * 32,
                          es * batch * cube(n) * 16, es * batch * cube(n) * 16, 4 * batch * cube(n)};
  int64_t o = 0;
  for (int k = 0; k < 12; ++k) {
    offs[k] = o;
    o += (sz[k] + 255) / 256 * 256;
  }
  offs[12] = o;
}

int64_t cnn_saved_bytes(int batch, int n, mdnp_dtype dtype) {
  int64_t offs[13];
  saved_layout(batch, n, dtype, offs);
  return offs[12];
}

// ---------------------------------------------------------------- FP32 convolutions on the matrix cores


// FP32 implicit-GEMM convolution on v_mfma_f32_16x16x4_f32 (FP32 products and
// sums): per output voxel block of 16 consecutive flattened voxels and per
// block of 16 output channels, D[co][v] = sum over (tap, ci) of W[co][t][ci]
// X[in(v, t)][ci] in chunks of 16 input channels.  Lane l of a wave reads
// input channels 4 (l / 16) .. + 3 of voxel l % 16 as one 16-byte load and
// issues four MFMAs with them (k = l / 16 of MFMA m is channel 4 (l / 16) + m;
// the weight operand follows the same order), so each wave owns MBV voxel
// blocks x NB channel blocks of accumulators; lane l ends with output
// channels 4 (l / 16) .. + 3 of voxel l % 16 and stores them as one 16-byte
// write.  Zero padding and the transposed stride by in_coord, as in the
// direct kernel; weights [taps][cin][cout].  Needs ca, cb, cout and the
// leading dimensions multiples of 16.
template <int MODE, int NB, int MBV>
__global__ void __launch_bounds__(256) k_conv_f32m(ConvP p) {
  const int64_t nvox = (int64_t)p.n_out * p.n_out * p.n_out;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bt = blockIdx.z;
  if (p.st && !(p.st[bt].active && p.st[bt].mode == p.want_mode)) return;
  const int64_t vb0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * MBV);  // first voxel of this wave
  if (vb0 >= nvox) return;
  const int co0 = blockIdx.y * 16 * NB;
  const int cin = p.ca + p.cb;
  const int r16 = lane & 15, kq = lane >> 4;
  int oz[MBV], oy[MBV], ox[MBV];
  bool vin_ok[MBV];
#pragma unroll
  for (int m = 0; m < MBV; ++m) {
    const int64_t v = vb0 + m * 16 + r16;
    vin_ok[m] = v < nvox;
    const int64_t vv = vin_ok[m] ? v : 0;
    ox[m] = (int)(vv % p.n_out);
    oy[m] = (int)((vv / p.n_out) % p.n_out);
    oz[m] = (int)(vv / ((int64_t)p.n_out * p.n_out));
  }
  f32x4v acc[NB][MBV];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int m = 0; m < MBV; ++m) acc[b][m] = f32x4v{0.f, 0.f, 0.f, 0.f};
  const float* A = (const float*)p.a + (int64_t)bt * p.a_bs;
  const float* B = p.cb ? (const float*)p.b + (int64_t)bt * p.b_bs : nullptr;
  const int ntap = (MODE == KIND_PT) ? 1 : 27;
  for (int t = 0; t < ntap; ++t) {
    const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
    int64_t vin[MBV];
    bool ok[MBV];
#pragma unroll
    for (int m = 0; m < MBV; ++m) {
      const int iz = in_coord<MODE>(oz[m], tz, p.n_in);
      const int iy = in_coord<MODE>(oy[m], ty, p.n_in);
      const int ix = in_coord<MODE>(ox[m], tx, p.n_in);
      ok[m] = vin_ok[m] && iz >= 0 && iy >= 0 && ix >= 0;
      vin[m] = ok[m] ? ((int64_t)iz * p.n_in + iy) * p.n_in + ix : 0;
    }
    const float* wt = p.wt + (int64_t)t * cin * p.cout + co0 + r16;
    for (int c0 = 0; c0 < cin; c0 += 16) {
      const bool in_a = c0 < p.ca;
      const float* src = in_a ? A : B;
      const int ld = in_a ? p.lda : p.ldb;
      const int cc = (in_a ? c0 : c0 - p.ca) + 4 * kq;
      f32x4v xv[MBV];
#pragma unroll
      for (int m = 0; m < MBV; ++m)
        xv[m] = ok[m] ? *(const f32x4v*)(src + vin[m] * ld + cc) : f32x4v{0.f, 0.f, 0.f, 0.f};
      const float* wc = wt + (int64_t)(c0 + 4 * kq) * p.cout;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        float w4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) w4[j] = wc[(int64_t)j * p.cout + b * 16];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int m = 0; m < MBV; ++m)
            acc[b][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4[j], xv[m][j], acc[b][m], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < MBV; ++m) {
    if (!vin_ok[m]) continue;
    const int64_t v = vb0 + m * 16 + r16;
    float* y = (float*)p.y + (int64_t)bt * p.y_bs + v * p.ldy + p.y_choff;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int co = co0 + b * 16 + 4 * kq;
      f32x4v r = acc[b][m];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (p.bias) r[j] += p.bias[co + j];
        if (p.relu) r[j] = fmaxf(r[j], 0.0f);
      }
      if (p.accumulate) r += *(const f32x4v*)(y + co);
      *(f32x4v*)(y + co) = r;
    }
  }
}

static bool conv_f32m_fits(const ConvP& p, int kind) {
  return kind != KIND_PT && p.ca % 16 == 0 && p.cb % 16 == 0 && p.cout % 16 == 0 && p.ca > 0 &&
         p.lda % 4 == 0 && (p.cb == 0 || p.ldb % 4 == 0) && p.ldy % 4 == 0 && p.y_choff % 4 == 0;
}

template <int MODE>
static void launch_f32m(const ConvP& p, int batch, hipStream_t stream) {
  const int64_t nvox = cube(p.n_out);
  constexpr int MBV = 2;
  const int nb = p.cout % 64 == 0 ? 4 : p.cout % 32 == 0 ? 2 : 1;
  const dim3 grid((unsigned)((nvox + 4 * 16 * MBV - 1) / (4 * 16 * MBV)), p.cout / (16 * nb), batch);
  if (nb == 4) hipLaunchKernelGGL((k_conv_f32m<MODE, 4, MBV>), grid, dim3(256), 0, stream, p);
  else if (nb == 2) hipLaunchKernelGGL((k_conv_f32m<MODE, 2, MBV>), grid, dim3(256), 0, stream, p);
  else hipLaunchKernelGGL((k_conv_f32m<MODE, 1, MBV>), grid, dim3(256), 0, stream, p);
}

// FP32 layers whose channel counts are multiples of 16 run on the matrix cores
// (k_conv_f32m); the others (2-channel first layer and its adjoint, the 1x1
// head) and the BF16 fallback shapes on the direct kernel.
template <typename Tin, typename Tout>
static void conv_direct(const ConvP& p, int kind, int batch, hipStream_t stream) {
  if constexpr (std::is_same<Tin, float>::value && std::is_same<Tout, float>::value) {
    if (conv_f32m_fits(p, kind)) {
      switch (kind) {
        case KIND_S1: launch_f32m<KIND_S1>(p, batch, stream); return;
        case KIND_S2: launch_f32m<KIND_S2>(p, batch, stream); return;
        case KIND_T2: launch_f32m<KIND_T2>(p, batch, stream); return;
        default: break;
      }
    }
  }
  const int64_t nvox = cube(p.n_out);
  const int co_chunk = p.cout >= 16 ? 16 : 1;
  dim3 grid((unsigned)((nvox + BS - 1) / BS), p.cout / co_chunk, batch);
#define LAUNCH_K(MODE)                                                                              \
  do {                                                                                              \
    if (co_chunk == 16) hipLaunchKernelGGL((k_conv<Tin, Tout, MODE, 16>), grid, dim3(BS), 0, stream, p); \
    else hipLaunchKernelGGL((k_conv<Tin, Tout, MODE, 1>), grid, dim3(BS), 0, stream, p);            \
  } while (0)
  switch (kind) {
    case KIND_S1: LAUNCH_K(KIND_S1); break;
    case KIND_S2: LAUNCH_K(KIND_S2); break;
    case KIND_T2: LAUNCH_K(KIND_T2); break;
    default: LAUNCH_K(KIND_PT); break;
  }
#undef LAUNCH_K
}

// Dispatch one layer: MFMA kernels for the BF16 interior layers, direct otherwise.
template <typename Tin, typename Tout>
static void conv_layer(const ConvP& p, int kind, int batch, mdnp_dtype dtype, int layer, CnnState& c,
                       hipStream_t stream) {
  if (dtype == MDNP_BF16 && conv_mfma_supported(layer) && std::is_same<Tin, bf16>::value &&
      std::is_same<Tout, bf16>::value) {
    conv_mfma_layer(p, kind, batch, layer, c, stream);
    return;
  }
  conv_direct<Tin, Tout>(p, kind, batch, stream);
}

// Layers 1..9 (L0b .. D0) on activations of type T, given the buffer set.
template <typename T>
static void unet_middle(CnnState& c, const float* d_w, void* const* act, int batch, int n, mdnp_dtype dtype,
                        const InstState* st, hipStream_t stream, int last_layer = 9, int first_layer = 1) {
  const int n1 = (n + 1) / 2, n2 = (n1 + 1) / 2;
  const int nn[3] = {n, n1, n2};
  // act indices: 1 a0, 2 s0, 3 a1, 4 s1, 5 a2, 6 b2, 7 u1, 8 d1, 9 u0, 10 d0
  struct Step { int layer, src_a, src_b, dst, lvl_in, lvl_out; };
  const Step steps[] = {{1, 1, -1, 2, 0, 0}, {2, 2, -1, 3, 0, 1}, {3, 3, -1, 4, 1, 1}, {4, 4, -1, 5, 1, 2},
                        {5, 5, -1, 6, 2, 2}, {6, 6, -1, 7, 2, 1}, {7, 7, 4, 8, 1, 1},  {8, 8, -1, 9, 1, 0},
                        {9, 9, 2, 10, 0, 0}};
  for (const Step& s : steps) {
    if (s.layer > last_layer) break;
    if (s.layer < first_layer) continue;
    const LayerSpec& L = kLayers[s.layer];
    ConvP p{};
    const int ca = s.src_b >= 0 ? L.cin / 2 : L.cin;
    p.a = act[s.src_a];
    p.ca = ca;
    p.lda = ca;
    p.a_bs = cube(nn[s.lvl_in]) * ca;
    if (s.src_b >= 0) {
      p.b = act[s.src_b];
      p.cb = L.cin - ca;
      p.ldb = p.cb;
      p.b_bs = cube(nn[s.lvl_in]) * p.cb;
    }
    p.n_in = nn[s.lvl_in];
    p.n_out = nn[s.lvl_out];
    p.wt = c.wt + c.wt_off[s.layer];
    p.bias = d_w + c.b_off[s.layer];
    p.cout = L.cout;
    p.y = act[s.dst];
    p.ldy = L.cout;
    p.y_bs = cube(nn[s.lvl_out]) * L.cout;
    p.relu = L.relu;
    p.st = st;
    p.want_mode = 0;
    conv_layer<T, T>(p, L.kind, batch, dtype, s.layer, c, stream);
  }
}

// Channels of the packed network input [v][2] into two arrays.
__global__ void k_split_input(const float* __restrict__ x, float* __restrict__ c0, float* __restrict__ c1,
                              int64_t nvox) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= nvox) return;
  const float2 a = ((const float2*)x)[v];
  c0[v] = a.x;
  c1[v] = a.y;
}

// The 1x1 head 16 -> 1 over all voxels: y = b + sum_c w_c x_c, channels in order.
template <typename T>
__global__ void __launch_bounds__(BS) k_head16(const T* __restrict__ x, const float* __restrict__ w,
                                               const float* __restrict__ b, float* __restrict__ y, int64_t nvox) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= nvox) return;
  const T* xv = x + v * 16;
  float acc = b[0];
#pragma unroll
  for (int ch = 0; ch < 16; ++ch) acc = fmaf(w[ch], ld(xv + ch), acc);
  y[v] = acc;
}

static bool ensure_split(CnnState& c, int batch, int n, hipStream_t stream) {
  const size_t nv = (size_t)batch * cube(n);
  if (c.split && c.split_n >= nv && c.std_batch == batch && c.std_n == n) return true;
  if (c.split) (void)hipFree(c.split);
  if (c.std_off) (void)hipFree(c.std_off);
  if (c.std_ones) (void)hipFree(c.std_ones);
  c.split = nullptr; c.std_off = nullptr; c.std_ones = nullptr;
  c.split_n = 0;
  if (hipMalloc(&c.split, sizeof(float) * 2 * nv) != hipSuccess) { c.split = nullptr; return false; }
  if (hipMalloc(&c.std_off, sizeof(int64_t) * batch) != hipSuccess) return false;
  if (hipMalloc(&c.std_ones, sizeof(double) * batch) != hipSuccess) return false;
  std::vector<int64_t> off(batch);
  std::vector<double> ones(batch, 1.0);
  for (int k = 0; k < batch; ++k) off[k] = (int64_t)k * cube(n);
  (void)hipMemcpyAsync(c.std_off, off.data(), sizeof(int64_t) * batch, hipMemcpyHostToDevice, stream);
  (void)hipMemcpyAsync(c.std_ones, ones.data(), sizeof(double) * batch, hipMemcpyHostToDevice, stream);
  (void)hipStreamSynchronize(stream);
  c.split_n = nv;
  c.std_batch = batch;
  c.std_n = n;
  return true;
}

template <typename T>
static void forward_t(CnnState& c, const float* in, float* out, void* saved, int batch, int n, mdnp_dtype dtype,
                      hipStream_t stream) {
  int64_t offs[13];
  saved_layout(batch, n, dtype, offs);
  char* base = (char*)saved;
  void* act[12];
  for (int k = 0; k < 12; ++k) act[k] = base + offs[k];
  hipMemcpyAsync(act[0], in, sizeof(float) * 2 * batch * cube(n), hipMemcpyDeviceToDevice, stream);
  const float* d_w = c.w;
  if (dtype == MDNP_BF16 && ensure_split(c, batch, n, stream)) {
    // L0a on MFMA: the first-layer kernel of the solver reading the two channels
    const int64_t nv = (int64_t)batch * cube(n);
    hipLaunchKernelGGL(k_split_input, dim3((unsigned)((nv + BS - 1) / BS)), dim3(BS), 0, stream,
                       (const float*)act[0], c.split, c.split + nv, nv);
    conv_mfma_in0<float>(c, c.split, c.std_off, c.std_ones, c.split + nv, n, batch, (bf16*)act[1], nullptr, stream);
  } else {  // L0a: FP32 input, direct
    const LayerSpec& L = kLayers[0];
    ConvP p{};
    p.a = act[0]; p.ca = 2; p.lda = 2; p.a_bs = cube(n) * 2;
    p.n_in = n; p.n_out = n;
    p.wt = c.wt + c.wt_off[0]; p.bias = d_w + c.b_off[0]; p.cout = L.cout;
    p.y = act[1]; p.ldy = 16; p.y_bs = cube(n) * 16; p.relu = 1;
    conv_direct<float, T>(p, KIND_S1, batch, stream);
  }
  unet_middle<T>(c, d_w, act, batch, n, dtype, nullptr, stream);
  {  // H: 16 -> 1, FP32 output
    const int64_t nv = (int64_t)batch * cube(n);
    hipLaunchKernelGGL((k_head16<T>), dim3((unsigned)((nv + BS - 1) / BS)), dim3(BS), 0, stream, (const T*)act[10],
                       d_w + c.w_off[10], d_w + c.b_off[10], (float*)act[11], nv);
  }
  if (out) hipMemcpyAsync(out, act[11], sizeof(float) * batch * cube(n), hipMemcpyDeviceToDevice, stream);
}

static bool ensure_scratch(CnnState& c, size_t bytes) {
  if (c.act_bytes >= bytes) return true;
  if (c.act[0]) hipFree(c.act[0]);
  c.act[0] = nullptr;
  c.act_bytes = 0;
  if (hipMalloc(&c.act[0], bytes) != hipSuccess) { c.act[0] = nullptr; return false; }
  c.act_bytes = bytes;
  return true;
}

bool cnn_reserve(CnnState& c, int batch, int n, mdnp_dtype dtype) {
  return ensure_scratch(c, (size_t)cnn_saved_bytes(batch, n, dtype));
}

void cnn_forward_batch(CnnState& c, const float* in, float* out, void* saved, int batch, int n, mdnp_dtype dtype,
                       hipStream_t stream) {
  if (!saved) {
    if (!ensure_scratch(c, (size_t)cnn_saved_bytes(batch, n, dtype))) return;
    saved = c.act[0];
  }
  if (dtype == MDNP_BF16) forward_t<bf16>(c, in, out, saved, batch, n, dtype, stream);
  else forward_t<float>(c, in, out, saved, batch, n, dtype, stream);
}

template <typename Tv>
void cnn_apply_in_solver(mdnp_sys* s, const Tv* zin, Tv* z, const InstState* st, hipStream_t stream,
                         const double* scales, int only_stage) {
  CnnState& c = s->cnn;
  const double* isc = scales ? scales : c.inv_s;
  const int n = s->n, batch = s->n_inst;
  // the E4M3 network (its calibration runs the FP32 one and records magnitudes)
  const bool fp8 = c.dtype == MDNP_FP8E4M3_ACT;
  const mdnp_dtype dt = fp8 ? MDNP_F32 : c.dtype;
  if (!ensure_scratch(c, (size_t)cnn_saved_bytes(batch, n, dt))) return;
  if (fp8 && !c.fp8_calibrating) {
    cnn_apply_fp8<Tv>(s, zin, z, st, stream, isc);
    return;
  }
  int64_t offs[13];
  saved_layout(batch, n, dt, offs);
  void* act[12];
  for (int k = 0; k < 12; ++k) act[k] = (char*)c.act[0] + offs[k];
  const dim3 grid((unsigned)((cube(n) + BS - 1) / BS), 1, batch);
  const bool all = only_stage < 0;
  const int mid_lo = all ? 1 : only_stage, mid_hi = all ? 9 : only_stage;
  if (c.dtype == MDNP_BF16 && !s->neumann) {
    // first layer reads the Krylov vector directly; D0, ReLU, the 1x1 head and the
    // unscaling are one kernel writing z0 on the free (interior) nodes
    if (all || only_stage == 0)
      conv_mfma_in0<Tv>(c, zin, s->d_off, isc, s->d_dist, n, batch, (bf16*)act[1], st, stream);
    unet_middle<bf16>(c, c.w, act, batch, n, c.dtype, st, stream, std::min(mid_hi, 8), mid_lo);
    if (all || only_stage == 9)
      conv_mfma_d0_head<Tv>(c, (const bf16*)act[9], (const bf16*)act[2], n, batch, z, s->d_off, s->d_alpha,
                            s->alpha_override, isc + s->n_inst, st, stream);
  } else if (c.dtype == MDNP_BF16) {
    // natural boundary: every node is free, so D0 writes its whole grid and
    // the head and the unscaling write z0 everywhere
    if (all || only_stage == 0)
      conv_mfma_in0<Tv>(c, zin, s->d_off, isc, s->d_dist, n, batch, (bf16*)act[1], st, stream);
    unet_middle<bf16>(c, c.w, act, batch, n, c.dtype, st, stream, mid_hi, mid_lo);
    if (all || only_stage == 9)
      hipLaunchKernelGGL((k_head_out<Tv, bf16>), grid, dim3(BS), 0, stream, (const bf16*)act[10],
                         c.wt + c.wt_off[10], c.w + c.b_off[10], n, z, s->d_off, s->d_alpha, s->alpha_override,
                         isc + s->n_inst, st, 1);
  } else {
    if (all || only_stage == 0)
      hipLaunchKernelGGL((k_conv_in0<Tv, float>), grid, dim3(BS), 0, stream, zin, s->d_off, isc, s->d_dist,
                         c.wt + c.wt_off[0], c.w + c.b_off[0], n, (float*)act[1], st);
    unet_middle<float>(c, c.w, act, batch, n, dt, st, stream, mid_hi, mid_lo);
    if (fp8) fp8_record_amax<Tv>(s, zin, isc, act, c.fp8_amax, stream);
    if (all || only_stage == 9)
      hipLaunchKernelGGL((k_head_out<Tv, float>), grid, dim3(BS), 0, stream, (const float*)act[10],
                         c.wt + c.wt_off[10], c.w + c.b_off[10], n, z, s->d_off, s->d_alpha, s->alpha_override,
                         isc + s->n_inst, st, s->neumann ? 1 : 0);
  }
}
template void cnn_apply_in_solver<float>(mdnp_sys*, const float*, float*, const InstState*, hipStream_t,
                                         const double*, int);
template void cnn_apply_in_solver<double>(mdnp_sys*, const double*, double*, const InstState*, hipStream_t,
                                          const double*, int);

template <typename Tv>
static bool layer_times_t(mdnp_sys* s, hipStream_t stream, int reps, float* ms) {
  Tv* tmp = nullptr;  // [2][ntot]: fixed input, output
  double* ones = nullptr;
  hipEvent_t ev[2] = {};
  const size_t nt = (size_t)s->ntot;
  bool ok = hipMalloc(&tmp, sizeof(Tv) * 2 * nt) == hipSuccess &&
            hipMalloc(&ones, sizeof(double) * 2 * s->n_inst) == hipSuccess;
  for (int k = 0; k < 2 && ok; ++k) ok = hipEventCreate(&ev[k]) == hipSuccess;
  if (ok) {
    std::vector<Tv> h(nt, (Tv)1e-3);
    std::vector<double> o(2 * (size_t)s->n_inst, 1.0);
    ok = hipMemcpyAsync(tmp, h.data(), sizeof(Tv) * nt, hipMemcpyHostToDevice, stream) == hipSuccess &&
         hipMemcpyAsync(ones, o.data(), sizeof(double) * o.size(), hipMemcpyHostToDevice, stream) == hipSuccess &&
         hipStreamSynchronize(stream) == hipSuccess;
  }
  if (ok) {
    // one whole application puts every stage's inputs in place; then each
    // stage alone, `reps` launches back to back between two events
    cnn_apply_in_solver<Tv>(s, tmp, tmp + nt, nullptr, stream, ones);
    for (int l = 0; l < 10 && ok; ++l) {
      cnn_apply_in_solver<Tv>(s, tmp, tmp + nt, nullptr, stream, ones, l);  // warm-up of this stage
      ok = hipEventRecord(ev[0], stream) == hipSuccess;
      for (int r = 0; r < reps && ok; ++r) cnn_apply_in_solver<Tv>(s, tmp, tmp + nt, nullptr, stream, ones, l);
      float t = 0.f;
      ok = ok && hipEventRecord(ev[1], stream) == hipSuccess && hipEventSynchronize(ev[1]) == hipSuccess &&
           hipEventElapsedTime(&t, ev[0], ev[1]) == hipSuccess;
      ms[l] = t / (float)reps;
    }
  }
  for (int k = 0; k < 2; ++k)
    if (ev[k]) (void)hipEventDestroy(ev[k]);
  if (tmp) (void)hipFree(tmp);
  if (ones) (void)hipFree(ones);
  return ok;
}

bool cnn_layer_times(mdnp_sys* s, hipStream_t stream, int reps, float* ms) {
  return s->vec_dtype == MDNP_F64 ? layer_times_t<double>(s, stream, reps, ms)
                                  : layer_times_t<float>(s, stream, reps, ms);
}

// ---------------------------------------------------------------- autotuning

// Chooses the launch shape of each BF16 layer on the system's own batch and
// grid: for the sweep layers the workgroup count their z split aims at and
// their output rows per workgroup, for the stride-2 and transposed layers the
// 16-voxel M blocks per wave, for the transposed layers also the workgroup
// count (each workgroup stages its weights once and loops over voxel blocks).
// Two rounds of coordinate descent over the layers, each candidate timed as the best of
// `reps` whole in-solver network applications with HIP events.  The shape only
// decides which wave computes which outputs, in the same order of
// accumulation, so results are the same for every choice.
struct TuneLayer {
  int layer, n;
  int cand[8];
  int rows = 0;  // 1: the candidates go to tile_mb (output rows, or workgroups of U1 / U0), 2: to tile_xb, else to sweep_blocks
};
static const TuneLayer kTune[] = {
    {1, 4, {3, 4, 5, 6}, 1},                         // L0b  output rows per workgroup (per wave pair)
    {3, 4, {2, 3, 4, 6}, 1},                         // L1b
    {7, 2, {2, 3}, 1},                               // D1
    {9, 3, {12, 13, 14}, 1},                         // D0 (+ head): rows of the three-plane z sweep
    {6, 5, {256, 512, 1024, 2048, 4096}, 1},         // U1   workgroups (each loops over voxel blocks)
    {0, 3, {1, 2, 4}, 2},                            // L0a  x blocks per workgroup
    {1, 3, {1, 2, 4}, 2},                            // L0b
    {3, 2, {1, 2}, 2},                               // L1b
    {7, 2, {1, 2}, 2},                               // D1
    {9, 3, {1, 2, 4}, 2},                            // D0
    {8, 5, {256, 512, 1024, 2048, 4096}, 1},         // U0
    {0, 7, {256, 384, 512, 768, 1024, 1536, 2048}},  // L0a  z split
    {1, 7, {256, 384, 512, 768, 1024, 1536, 2048}},  // L0b
    {2, 3, {2, 4, 8}},                               // L1a  M blocks per wave
    {3, 7, {256, 384, 512, 768, 1024, 1536, 2048}},  // L1b
    {4, 3, {1, 2, 4}},                               // L2a
    {5, 7, {256, 384, 512, 768, 1024, 1536, 2048}},  // L2b
    {6, 2, {1, 2}},                                  // U1
    {7, 7, {256, 384, 512, 768, 1024, 1536, 2048}},  // D1
    {8, 3, {1, 2, 4}},                               // U0
    {9, 7, {256, 384, 512, 768, 1024, 1536, 2048}},  // D0 (+ head)
};

template <typename Tv>
static bool autotune_t(mdnp_sys* s, hipStream_t stream, int reps) {
  CnnState& c = s->cnn;
  Tv* tmp = nullptr;  // [2][ntot]: fixed input, output
  double* ones = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t nt = (size_t)s->ntot;
  bool ok = hipMalloc(&tmp, sizeof(Tv) * 2 * nt) == hipSuccess &&
            hipMalloc(&ones, sizeof(double) * 2 * s->n_inst) == hipSuccess &&
            hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  if (ok) {
    std::vector<Tv> h(nt, (Tv)1e-3);
    std::vector<double> o(2 * (size_t)s->n_inst, 1.0);
    ok = hipMemcpyAsync(tmp, h.data(), sizeof(Tv) * nt, hipMemcpyHostToDevice, stream) == hipSuccess &&
         hipMemcpyAsync(ones, o.data(), sizeof(double) * o.size(), hipMemcpyHostToDevice, stream) == hipSuccess &&
         hipStreamSynchronize(stream) == hipSuccess;
  }
  auto time_once = [&]() {
    float best = 1e30f;
    for (int r = 0; r < reps; ++r) {
      (void)hipEventRecord(e0, stream);
      cnn_apply_in_solver<Tv>(s, tmp, tmp + nt, nullptr, stream, ones);
      (void)hipEventRecord(e1, stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, ms);
    }
    return best;
  };
  if (ok) {
    time_once();  // warm-up
    // two rounds of coordinate descent: the second revisits each layer with
    // the others at their tuned shapes
    for (int round = 0; round < 2; ++round) {
      for (const TuneLayer& tl : kTune) {
        const int layer = tl.layer;
        int* slot = tl.rows == 1 ? &c.tile_mb[layer] : tl.rows == 2 ? &c.tile_xb[layer] : &c.sweep_blocks[layer];
        int best_t = *slot;
        float best = 1e30f;
        for (int q = 0; q < tl.n; ++q) {
          const int t = tl.cand[q];
          *slot = t;
          const float ms = time_once();
          if (ms < best) {
            best = ms;
            best_t = t;
          }
        }
        *slot = best_t;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (tmp) (void)hipFree(tmp);
  if (ones) (void)hipFree(ones);
  return ok;
}

bool cnn_autotune(mdnp_sys* s, hipStream_t stream, int reps) {
  return s->vec_dtype == MDNP_F64 ? autotune_t<double>(s, stream, reps) : autotune_t<float>(s, stream, reps);
}

// ---------------------------------------------------------------- backward

namespace {
struct BwdBufs {
  float* g[12];     // gradients w.r.t. the saved tensors (FP32), same shapes
  float* wadj;      // adjoint weights scratch
  float* part;      // split partials
  int64_t part_n;
};
}  // namespace

template <typename T>
static void backward_t(CnnState& c, const void* saved, const float* dy, float* dx, float* dw, int batch, int n,
                       mdnp_dtype dtype, hipStream_t stream) {
  const int n1 = (n + 1) / 2, n2 = (n1 + 1) / 2;
  const int nn[3] = {n, n1, n2};
  int64_t offs[13];
  saved_layout(batch, n, dtype, offs);
  const void* act[12];
  for (int k = 0; k < 12; ++k) act[k] = (const char*)saved + offs[k];
  // gradient buffers: one FP32 tensor per saved tensor (except y)
  const int chans[12] = {2, 16, 16, 32, 32, 64, 64, 32, 32, 16, 16, 1};
  const int lvl[12] = {0, 0, 0, 1, 1, 2, 2, 1, 1, 0, 0, 0};
  int64_t goff[12], gtot = 0;
  for (int k = 0; k < 12; ++k) {
    goff[k] = gtot;
    gtot += ((int64_t)batch * cube(nn[lvl[k]]) * chans[k] + 63) / 64 * 64;
  }
  const int nsplit = 64;
  const int64_t part_n = (int64_t)nsplit * 27 * 64 * 64;
  const int64_t wadj_n = 27 * 64 * 64;
  const size_t need = sizeof(float) * (size_t)(gtot + part_n + wadj_n);
  if (c.bwd_bytes < need) {
    if (c.bwd) hipFree(c.bwd);
    c.bwd = nullptr;
    if (hipMalloc(&c.bwd, need) != hipSuccess) { c.bwd = nullptr; c.bwd_bytes = 0; return; }
    c.bwd_bytes = need;
  }
  float* scratch = (float*)c.bwd;
  float* G[12];
  for (int k = 0; k < 12; ++k) G[k] = scratch + goff[k];
  float* part = scratch + gtot;
  float* wadj = part + part_n;
  hipMemsetAsync(scratch, 0, sizeof(float) * (size_t)gtot, stream);
  // dy -> G[11]
  hipMemcpyAsync(G[11], dy, sizeof(float) * batch * cube(n), hipMemcpyDeviceToDevice, stream);

  struct BStep { int layer, in_a, in_b, out; };
  // reverse order; inputs as in the forward
  const BStep steps[] = {{10, 10, -1, 11}, {9, 9, 2, 10}, {8, 8, -1, 9}, {7, 7, 4, 8}, {6, 6, -1, 7},
                         {5, 5, -1, 6},   {4, 4, -1, 5}, {3, 3, -1, 4}, {2, 2, -1, 3}, {1, 1, -1, 2},
                         {0, 0, -1, 1}};
  for (const BStep& s : steps) {
    const LayerSpec& L = kLayers[s.layer];
    const int taps = L.kind == KIND_PT ? 1 : 27;
    const int lin = lvl[s.in_a], lout = lvl[s.out];
    const int64_t nout_vox = (int64_t)batch * cube(nn[lout]);
    float* dz = G[s.out];
    // ReLU mask from the saved output
    if (L.relu)
      hipLaunchKernelGGL(k_relu_mask, dim3((unsigned)((nout_vox * L.cout + 255) / 256)), dim3(256), 0, stream, dz,
                         act[s.out], dtype == MDNP_BF16 ? 1 : 0, nout_vox * L.cout);
    // weight gradient
    const int ca = s.in_b >= 0 ? L.cin / 2 : L.cin;
    const int cb = L.cin - ca;
    const bool in_fp32 = (s.in_a == 0);  // X is stored in FP32
    const int64_t nw = (int64_t)L.cout * taps * L.cin;
    // about 4096 waves over element ranges (splits), within the partial buffer
    auto splits = [&](int waves_per_split) {
      return (int)std::max<int64_t>(1, std::min<int64_t>(4096 / waves_per_split, part_n / nw));
    };
    int ns;
    if (in_fp32) {
      // the first layer: 2 FP32 input channels, 16 outputs, stride 1
      ns = splits(1);
      hipLaunchKernelGGL(k_dw_first, dim3((unsigned)ns), dim3(64), 0, stream, dz, (const float*)act[0], n, batch,
                         part, ns);
    } else if (L.cout == 1) {
      // the 1x1 head with one output: a weighted row sum
      ns = 512;
      hipLaunchKernelGGL((k_rows_part<T>), dim3((unsigned)ns), dim3(256), 0, stream, dz, (const T*)act[s.in_a],
                         L.cin, nout_vox, part);
    } else {
      // channel counts in multiples of 16 on the matrix cores: the 9 taps of
      // one tz per wave (the 1x1 layer: its one tap), and two 16-channel blocks
      // of the operand loaded once per element where there are two (co for the
      // stride-1/2 layers, ci for the transposed ones)
      const bool t2 = L.kind == KIND_T2;
      const int nbo = (!t2 && L.cout >= 32) ? 2 : 1, nbi = (t2 && L.cin >= 32) ? 2 : 1;
      const int ntg = L.kind == KIND_PT ? 1 : 3;  // wave groups along tz
      const int nwt = (L.cout / (16 * nbo)) * (L.cin / (16 * nbi));
      ns = splits(ntg * nwt);
      const dim3 g((unsigned)(ntg * nwt), 1, (unsigned)ns);
#define DWM_ARGS                                                                                              \
  g, dim3(64), 0, stream, dz, L.cout, act[s.in_a], ca, ca, s.in_b >= 0 ? act[s.in_b] : nullptr, cb, cb, nn[lin], \
      nn[lout], batch, cube(nn[lin]) * ca, cube(nn[lin]) * cb, part, ns
      if (t2) {
        if (nbi == 2) hipLaunchKernelGGL((k_dw_m<T, KIND_T2, 1, 1, 2>), DWM_ARGS);
        else hipLaunchKernelGGL((k_dw_m<T, KIND_T2, 1, 1, 1>), DWM_ARGS);
      } else if (nbo == 2) {
        switch (L.kind) {
          case KIND_S1: hipLaunchKernelGGL((k_dw_m<T, KIND_S1, 1, 2, 1>), DWM_ARGS); break;
          case KIND_S2: hipLaunchKernelGGL((k_dw_m<T, KIND_S2, 1, 2, 1>), DWM_ARGS); break;
          default: hipLaunchKernelGGL((k_dw_m<T, KIND_PT, 1, 2, 1>), DWM_ARGS); break;
        }
      } else {
        switch (L.kind) {
          case KIND_S1: hipLaunchKernelGGL((k_dw_m<T, KIND_S1, 1, 1, 1>), DWM_ARGS); break;
          case KIND_S2: hipLaunchKernelGGL((k_dw_m<T, KIND_S2, 1, 1, 1>), DWM_ARGS); break;
          default: hipLaunchKernelGGL((k_dw_m<T, KIND_PT, 1, 1, 1>), DWM_ARGS); break;
        }
      }
#undef DWM_ARGS
    }
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((nw + 31) / 32)), dim3(256), 0, stream, part,
                       dw + c.w_off[s.layer], nw, ns);
    // bias gradient: 512 row ranges, then their sum (the partials reuse `part`)
    hipLaunchKernelGGL((k_rows_part<float>), dim3(512), dim3(256), 0, stream, dz, (const float*)nullptr, L.cout,
                       nout_vox, part);
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((L.cout + 31) / 32)), dim3(256), 0, stream, part,
                       dw + c.b_off[s.layer], (int64_t)L.cout, 512);
    // data gradient: adjoint layer (input channels = cout, output channels = cin)
    if (s.layer == 0 && !dx) continue;
    const int flip = L.kind == KIND_S1 ? 1 : 0;
    hipLaunchKernelGGL(k_wt_adj, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, stream, c.w + c.w_off[s.layer],
                       wadj, L.cout, taps, L.cin, flip);
    ConvP p{};
    p.a = dz; p.ca = L.cout; p.lda = L.cout; p.a_bs = cube(nn[lout]) * L.cout;
    p.n_in = nn[lout]; p.n_out = nn[lin];
    p.wt = wadj; p.bias = nullptr; p.relu = 0; p.accumulate = 1;
    const int adj_kind = L.kind == KIND_S1 ? KIND_S1 : L.kind == KIND_S2 ? KIND_T2 : L.kind == KIND_T2 ? KIND_S2 : KIND_PT;
    if (s.in_b < 0) {
      p.cout = L.cin;
      p.y = (s.layer == 0) ? (void*)dx : (void*)G[s.in_a];
      p.ldy = L.cin;
      p.y_bs = cube(nn[lin]) * L.cin;
      if (s.layer == 0) p.accumulate = 0;
      conv_direct<float, float>(p, adj_kind, batch, stream);
    } else {
      // channel-stacked input: the adjoint output channels [0, ca) go to source A's
      // gradient and [ca, cin) to source B's; two compact adjoint weight copies
      float* w1 = wadj;
      float* w2 = wadj + (int64_t)taps * L.cout * ca;
      hipLaunchKernelGGL(k_wt_adj_split, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, stream,
                         c.w + c.w_off[s.layer], w1, w2, L.cout, taps, L.cin, ca, flip);
      ConvP pa = p;
      pa.wt = w1; pa.cout = ca; pa.y = G[s.in_a]; pa.ldy = ca; pa.y_bs = cube(nn[lin]) * ca;
      conv_direct<float, float>(pa, adj_kind, batch, stream);
      ConvP pb = p;
      pb.wt = w2; pb.cout = cb; pb.y = G[s.in_b]; pb.ldy = cb; pb.y_bs = cube(nn[lin]) * cb;
      conv_direct<float, float>(pb, adj_kind, batch, stream);
    }
  }
}

void cnn_backward_batch(CnnState& c, const void* saved, const float* dy, float* dx, float* dw, int batch, int n,
                        mdnp_dtype dtype, hipStream_t stream) {
  if (dtype == MDNP_BF16) backward_t<bf16>(c, saved, dy, dx, dw, batch, n, dtype, stream);
  else backward_t<float>(c, saved, dy, dx, dw, batch, n, dtype, stream);
}

namespace {
constexpr int kLossParts = 64;  // partial sums per slot of the loss reduction
}

size_t loss_grad_scratch_bytes(int64_t n3d, int n_slots) {
  return (size_t)n_slots * n3d * 2 * sizeof(float) + (size_t)n_slots * kLossParts * sizeof(double);
}

// The loss and its gradient with the scratch at `buf` (loss_grad_scratch_bytes
// of it): the masked output and C e per slot, then the partial sums.  Every
// scratch word is written before it is read.
static void loss_grad_core(mdnp_sys* s, const int32_t* inst, int n_slots, const float* r, const float* u,
                           float* du, double* loss, void* scratch_buf, hipStream_t stream) {
  const int64_t n3d = s->n3d;
  const int nbx = kLossParts;
  float* buf = (float*)scratch_buf;
  float* um = buf;
  float* ce = buf + (size_t)n_slots * n3d;
  double* part = (double*)(buf + (size_t)n_slots * n3d * 2);
  const dim3 g2((unsigned)((n3d + BS - 1) / BS), n_slots);
  hipLaunchKernelGGL(k_mask_bnd, g2, dim3(BS), 0, stream, u, um, s->n, n3d, s->neumann ? 0 : 1);
  launch_spmv_a00_slots(s, inst, n_slots, um, ce, stream);
  hipLaunchKernelGGL(k_loss_e, dim3(nbx, n_slots), dim3(BS), 0, stream, r, ce, inst, s->d_alpha, n3d, part, nbx);
  hipLaunchKernelGGL(k_loss_sum, dim3((n_slots + 63) / 64), dim3(64), 0, stream, part, nbx, n_slots, loss);
  launch_spmv_a00_slots(s, inst, n_slots, ce, um, stream);
  hipLaunchKernelGGL(k_loss_grad_fin, g2, dim3(BS), 0, stream, um, du, inst, s->d_alpha, s->n, n3d,
                     s->neumann ? 0 : 1);
}

void launch_loss_grad(mdnp_sys* s, const int32_t* inst, int n_slots, const float* r, const float* u, float* du,
                      double* loss, hipStream_t stream) {
  const size_t need = loss_grad_scratch_bytes(s->n3d, n_slots);
  CnnState& c = s->cnn;
  if (c.loss_bytes < need) {
    if (c.loss) hipFree(c.loss);
    c.loss = nullptr;
    if (hipMalloc(&c.loss, need) != hipSuccess) { c.loss = nullptr; c.loss_bytes = 0; return; }
    c.loss_bytes = need;
  }
  loss_grad_core(s, inst, n_slots, r, u, du, loss, c.loss, stream);
}

// ---------------------------------------------------------------- allocation-free loss

// Fixed workspace of mdnp_loss_grad_noalloc, one copy per GPU the library runs
// on, held until the process ends.  Host code never passes `scratch` itself to
// a kernel (on the host it names a stand-in, not device memory): it uses the
// per-device address resolved once by loss_scratch_resolve.
static __device__ __align__(256) unsigned char scratch[kLossScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

bool loss_scratch_resolve(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return true;
}

void launch_loss_grad_fixed(mdnp_sys* s, const int32_t* inst, int n_slots, const float* r, const float* u,
                            float* du, double* loss, void* scratch_ptr, hipStream_t stream) {
  loss_grad_core(s, inst, n_slots, r, u, du, loss, scratch_ptr, stream);
}

void launch_pack_input(mdnp_sys* s, const int32_t* inst, int n_slots, const float* r, float* x,
                       hipStream_t stream) {
  const int64_t n3d = s->n3d;
  const dim3 g2((unsigned)((n3d + BS - 1) / BS), n_slots);
  hipLaunchKernelGGL(k_pack_input, g2, dim3(BS), 0, stream, r, s->d_dist, inst, n3d, x);
}

void launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t stream) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, w, g, m, v, n, lr, b1, b2,
                     eps, c1, c2);
}

void cnn_release(CnnState& c) {
  if (c.w_own) hipFree(c.w_own);
  if (c.bwd) hipFree(c.bwd);
  if (c.loss) hipFree(c.loss);
  if (c.wt) hipFree(c.wt);
  if (c.wmf) hipFree(c.wmf);
  if (c.act[0]) hipFree(c.act[0]);
  if (c.inv_s) hipFree(c.inv_s);
  if (c.split) hipFree(c.split);
  if (c.std_off) hipFree(c.std_off);
  if (c.std_ones) hipFree(c.std_ones);
  if (c.w8) hipFree(c.w8);
  if (c.w8s) hipFree(c.w8s);
  if (c.fp8_amax) hipFree(c.fp8_amax);
  c = CnnState();
}

}  // namespace mdnp
