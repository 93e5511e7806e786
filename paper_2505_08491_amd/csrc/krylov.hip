// Krylov kernels of the flexible GMRES iteration (Section 4, restarted FGMRES
// with right preconditioning) and of the block preconditioner of Section 2.2.
//
// Layout: the vectors of all instances are concatenated; reductions are done
// per contiguous chunk ("block") inside one instance, each block writing one
// FP64 partial sum; every consumer sums the partials of its instance in a
// fixed order, so results are bitwise reproducible run to run.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "kernels.hpp"

namespace mdnp {

namespace {

constexpr int BS = 256;  // threads per block for vector kernels

template <typename T> __device__ __forceinline__ double to_d(T v) { return (double)v; }
template <> __device__ __forceinline__ double to_d<bf16>(bf16 v) { return (double)__bfloat162float(v); }
template <typename T> __device__ __forceinline__ T from_d(double v) { return (T)v; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block; result valid in every thread.
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += sh[k];
  __syncthreads();
  return t;
}

// block_sum with barriers that wait for LDS traffic only (global loads issued
// before it stay in flight); same order, same result.
__device__ double block_sum_lds(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) sh[wid] = v;
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += sh[k];
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
  return t;
}

// block_sum_lds of NV values at once (one pair of barriers); sh holds
// NV * (BS / 64) doubles.  Result valid in every thread.
template <int NV>
__device__ void block_sums_lds(double (&v)[NV], double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    v[q] = wave_sum(v[q]);
    if (lane == 0) sh[q * (BS / 64) + wid] = v[q];
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = 0.0;
    for (int k = 0; k < nw; ++k) t += sh[q * (BS / 64) + k];
    v[q] = t;
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Sum of the partials of instance i (fixed order), result in every thread.
__device__ double inst_sum(const double* part, const int32_t* first, int i, double* sh) {
  double t = 0.0;
  for (int b = first[i] + threadIdx.x; b < first[i + 1]; b += blockDim.x) t += part[b];
  return block_sum(t, sh);
}

// Sum of the partials part[first[i] .. first[i+1]) by one wavefront in a fixed
// order (lane-strided, then a butterfly), result in every lane.
__device__ __forceinline__ double wave_inst_sum(const double* part, const int32_t* first, int i) {
  double t = 0.0;
  for (int b = first[i] + (int)(threadIdx.x & 63); b < first[i + 1]; b += 64) t += part[b];
  return wave_sum(t);
}

__device__ __forceinline__ int find_inst(const int64_t* off, int n_inst, int64_t g) {
  int lo = 0, hi = n_inst;  // off[lo] <= g < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ bool is_boundary(int r, int n) {
  int i = r % n, j = (r / n) % n, k = r / (n * n);
  return i == 0 || j == 0 || k == 0 || i == n - 1 || j == n - 1 || k == n - 1;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// For a grid of 8 * ceil(nlog / 8) workgroups this returns the logical block
// of the calling workgroup such that every XCD runs a contiguous range of
// logical blocks (blocks are ordered by instance, so an XCD's L2 sees about
// n_inst / 8 instances), or -1 for the padding workgroups.
__device__ __forceinline__ int xcd_logical_block(int nlog) {
  const int per = (nlog + 7) / 8;
  const int p = blockIdx.x;
  const int b = (p % 8) * per + p / 8;
  return b < nlog ? b : -1;
}

inline unsigned xcd_grid(int nlog) { return (unsigned)(8 * ((nlog + 7) / 8)); }

// ---------------------------------------------------------------- operator A = S + M

// (S x)[r] for 3D row r of the instance whose vector starts at x + base: the
// constant 27-point stencil grouped by the number of differing coordinates
// (centre, 6 faces, 12 edges, 8 corners); neighbours on the boundary are left
// out, and a boundary row is st4[4] times the unit row (1 for the Dirichlet
// condition; 0 for the natural one, whose boundary rows the coupling-row part
// holds).
template <typename Tv, typename Tacc>
__device__ __forceinline__ Tacc stencil_row(const Tv* __restrict__ x, int64_t base, int r, int n,
                                            const double* __restrict__ st4) {
  const int ix = r % n, iy = (r / n) % n, iz = r / (n * n);
  const Tv* xc = x + base + r;
  if (ix == 0 || iy == 0 || iz == 0 || ix == n - 1 || iy == n - 1 || iz == n - 1)
    return (Tacc)st4[4] * (Tacc)xc[0];
  const bool vx[3] = {ix > 1, true, ix < n - 2};
  const bool vy[3] = {iy > 1, true, iy < n - 2};
  const bool vz[3] = {iz > 1, true, iz < n - 2};
  const int64_t nn = (int64_t)n * n;
  Tacc grp[4] = {0, 0, 0, 0};
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int nd = (dx != 1) + (dy != 1) + (dz != 1);
        if (vx[dx] && vy[dy] && vz[dz]) grp[nd] += (Tacc)xc[(dz - 1) * nn + (dy - 1) * n + (dx - 1)];
      }
  return (Tacc)st4[0] * grp[0] + (Tacc)st4[1] * grp[1] + (Tacc)st4[2] * grp[2] + (Tacc)st4[3] * grp[3];
}

// y = S x on the 3D rows, sweeping z, for n <= SW_NMAX nodes per side.  A
// wave owns rows y0 .. y0 + SW_TY - 1 of planes z0 .. z0 + zc - 1 of one
// instance, lane l holding columns x = l + 1 + 64 k for k < NX (the interior
// columns and the x = n - 1 boundary column; NX = 1 up to 65 nodes, 2 up to
// 129).  For every input plane it loads rows y0 - 1 .. y0 + SW_TY, zeroes the
// nodes on the boundary (Dirichlet: their columns are eliminated; natural
// condition: the coupling-row part adds those columns), takes the
// x-neighbour sums by lane shifts (the neighbours across the two column
// blocks by lane reads) and forms per output row the 2D partials centre,
// 4 in-plane faces and 4 in-plane corners.  Output plane z gathers them from
// z' = z (offsets 0, 1, 2 differing coordinates) and z' = z +- 1 (1, 2, 3), so
// two accumulators per row ride along the sweep.  Boundary rows get wb x
// (wb = 1: Dirichlet unit rows; wb = 0: natural condition, the coupling-row
// part holds those rows).  Planes are loaded SW_PD steps ahead into a ring of
// register sets; the loop is unrolled over the ring, so no set is copied and a
// step waits only for its own plane.  No LDS, no barriers.  The x = 0
// boundary column is written by extra waves of the same launch (one per
// instance and SW_FZ planes, placed with that instance's row strips).
constexpr int SW_TY = 5;      // output rows per wave
constexpr int SW_PD = 3;      // planes in flight (register sets)
constexpr int SW_FZ = 8;      // planes per x = 0 copy wave
constexpr int SW_NMAX = 129;  // lane l <-> columns l + 1, l + 65

__device__ __forceinline__ float lane_from_left(float v) {  // value of lane l - 1 (0 for lane 0)
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_from_right(float v) {  // value of lane l + 1 (0 for lane 63)
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ double lane_from_left(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), 0x138, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_from_right(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), 0x130, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {  // v of lane l, in every lane
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane((int)__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane((int)__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// The coupling M = B^T W B + R in factored form (eq. "mainsys": every Gauss
// point q contributes W_q (Pi_q u - Phi_q u1)(Pi_q v - Phi_q v1)).  First
// pass: t[q] = W_q B_q x over the Gauss points (W_q folded into the stored
// entries); for A00 the 3D-column entries only, W_q Pi_q x (on x + x2 when x2
// is given).  It runs in workgroups appended to the stencil sweep's grid.
struct CgArgs {
  const int32_t* gp = nullptr;      // [points + 1] entry offsets
  const int32_t* gsplit = nullptr;  // [points] end of each point's 3D-column entries
  const int32_t* gcol = nullptr;    // global x indices
  const void* gval = nullptr;       // W_q B_q entries (the vector type)
  void* t = nullptr;                // [points] out
  const int32_t* binst = nullptr;   // Gauss-point lists
  const int64_t* bstart = nullptr;
  const int64_t* bend = nullptr;
  int nblk = 0;
};

constexpr int CG_G = 4;  // lanes per Gauss point
constexpr int CS_G = 4;  // lanes per listed row of the second pass

// Logical block of physical workgroup p (as xcd_logical_block, for a range of
// the grid that starts at a multiple of 8).
__device__ __forceinline__ int xcd_logical_block_at(int nlog, int p) {
  const int per = (nlog + 7) / 8;
  const int b = (p % 8) * per + p / 8;
  return b < nlog ? b : -1;
}

// G lanes per Gauss point, U = 16 / G entries per lane per pass with the
// loads of a pass in flight together (indices clamped into the point's range).
template <typename T, int G, int A00>
__device__ __forceinline__ void cgather_block(const CgArgs& a, int b, const T* __restrict__ x,
                                              const T* __restrict__ x2, const InstState* st, int mask) {
  const int i = a.binst[b];
  if (mask == 1 && !st[i].active) return;
  const int32_t* __restrict__ gcol = a.gcol;
  const T* __restrict__ gval = (const T*)a.gval;
  const int grp = threadIdx.x / G, lane = threadIdx.x % G, ng = 256 / G;
  constexpr int U = 16 / G;
  for (int64_t q = a.bstart[b] + grp; q < a.bend[b]; q += ng) {
    T acc = 0;
    const int e = A00 ? a.gsplit[q] : a.gp[q + 1];
    for (int k0 = a.gp[q] + lane; k0 < e; k0 += U * G) {
      int c[U];
      T v[U], xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = min(k0 + u * G, e - 1);
        c[u] = gcol[k];
        v[u] = gval[k];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
      if (A00 && x2) {
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] += x2[c[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k0 + u * G < e) acc += v[u] * xv[u];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (lane == 0) ((T*)a.t)[q] = acc;
  }
}

// CG = 1 or 2: workgroups past the sweep's (a multiple of 8) run the first
// pass of the factored coupling, t = W B x (1) or W Pi x (2, A00).
template <typename Tv, typename Tacc, int SUM = 0, int NX = 1, int CG = 0>
__global__ void __launch_bounds__(256) k_stencil_sweep(const double* __restrict__ stencil, const Tv* __restrict__ x,
                                                       Tv* __restrict__ y, const int64_t* __restrict__ off, int n,
                                                       int ytiles, int zc, int nfz, int ntile, const InstState* st,
                                                       int mask, const Tv* __restrict__ x2 = nullptr,
                                                       CgArgs cg = CgArgs()) {
  constexpr int NR = SW_TY + 2;
  if (CG) {
    const int nsw = (int)(8 * ((((ntile + 3) >> 2) + 7) / 8));
    if ((int)blockIdx.x >= nsw) {
      const int b = xcd_logical_block_at(cg.nblk, (int)blockIdx.x - nsw);
      if (b >= 0) cgather_block<Tv, CG_G, CG == 2>(cg, b, x, x2, st, mask);
      return;
    }
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int lb = xcd_logical_block((ntile + 3) >> 2);
  if (lb < 0) return;
  const int tid = lb * 4 + wave;
  if (tid >= ntile) return;
  const int64_t nn = (int64_t)n * n;
  // tiles of an instance: nfz x = 0 column tiles, then its row strips, so that
  // both kinds of an instance run on the XCD that holds its vector in L2
  const int nz = (n + zc - 1) / zc;
  const int per = nfz + ytiles * nz;
  const int i = tid / per, t0 = tid - i * per;
  if (mask && !st[i].active) return;
  if (t0 < nfz) {  // x = 0 column of planes zf .. zf + SW_FZ - 1, rows lane + 64 h
    constexpr int RG = NX + 1;  // row groups of 64: n <= 64 NX + 1
    const int zf = t0 * SW_FZ;
    const Tv* X = x + off[i];
    const Tv* X2 = SUM ? x2 + off[i] : nullptr;
    Tv* Y = y + off[i];
    // every load first (clamped to a valid address), then the stores: one
    // memory round trip per wave instead of one per row group and plane
    const Tacc wb = (Tacc)stencil[kStencilStride * i + 4];
    Tv cv[SW_FZ][RG];
#pragma unroll
    for (int zz = 0; zz < SW_FZ; ++zz)
#pragma unroll
      for (int h = 0; h < RG; ++h) {
        const int z = zf + zz, gy = lane + 64 * h;
        const int64_t v = z < n && gy < n ? z * nn + (int64_t)gy * n : 0;
        cv[zz][h] = (Tv)(wb * (SUM ? (Tacc)X[v] + (Tacc)X2[v] : (Tacc)X[v]));
      }
#pragma unroll
    for (int zz = 0; zz < SW_FZ; ++zz)
#pragma unroll
      for (int h = 0; h < RG; ++h) {
        const int z = zf + zz, gy = lane + 64 * h;
        if (z < n && gy < n) Y[z * nn + (int64_t)gy * n] = cv[zz][h];
      }
    return;
  }
  const int rem = t0 - nfz;
  const int y0 = (rem % ytiles) * SW_TY, z0 = (rem / ytiles) * zc;
  const int zend = min(n, z0 + zc);
  const Tv* X = x + off[i];
  const Tv* X2 = SUM ? x2 + off[i] : nullptr;  // SUM = 1: S (x + x2)
  Tv* Y = y + off[i];
  const double* st5 = stencil + kStencilStride * i;
  const Tacc w0 = (Tacc)st5[0], w1 = (Tacc)st5[1], w2 = (Tacc)st5[2], w3 = (Tacc)st5[3];
  const Tacc wb = (Tacc)st5[4];  // boundary rows: wb x (unit rows, or zero rows whose entries M holds)
  int xx[NX];
  bool xact[NX], xin[NX];
#pragma unroll
  for (int k = 0; k < NX; ++k) {
    xx[k] = lane + 1 + 64 * k;
    xact[k] = xx[k] <= n - 1;
    xin[k] = xx[k] <= n - 2;
  }
  // byte offsets of this lane's nodes in the rows y0 - 1 .. y0 + SW_TY of a
  // plane (clamped into the grid; 32-bit, so the loads take a scalar base)
  unsigned roff[NX][NR];
  bool rin[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int gy = y0 - 1 + r;
    rin[r] = gy >= 1 && gy <= n - 2;
#pragma unroll
    for (int k = 0; k < NX; ++k)
      roff[k][r] = (unsigned)(min(max(gy, 0), n - 1) * n + min(xx[k], n - 1)) * (unsigned)sizeof(Tv);
  }
  Tv v[SW_PD][NX][NR], v2[SUM ? SW_PD : 1][NX][NR];
  auto load = [&](int zp, int K) {
    const int64_t zb = (int64_t)min(max(zp, 0), n - 1) * nn;
    const char* P = (const char*)(X + zb);
#pragma unroll
    for (int k = 0; k < NX; ++k)
#pragma unroll
      for (int r = 0; r < NR; ++r) v[K][k][r] = *(const Tv*)(P + roff[k][r]);
    if (SUM) {
      const char* P2 = (const char*)(X2 + zb);
#pragma unroll
      for (int k = 0; k < NX; ++k)
#pragma unroll
        for (int r = 0; r < NR; ++r) v2[SUM ? K : 0][k][r] = *(const Tv*)(P2 + roff[k][r]);
    }
  };
  // partial outputs of planes zp - 1 and zp, raw plane zp - 1 (Dirichlet copies)
  Tacc accp[NX][SW_TY], accc[NX][SW_TY], prev[NX][SW_TY];
#pragma unroll
  for (int k = 0; k < NX; ++k)
#pragma unroll
    for (int t = 0; t < SW_TY; ++t) accp[k][t] = accc[k][t] = prev[k][t] = 0;
  const int nsteps = zend - z0 + 2;  // step s reduces input plane zp = z0 - 1 + s
#pragma unroll
  for (int K = 0; K < SW_PD; ++K) load(z0 - 1 + K, K);
  for (int s0 = 0; s0 < nsteps; s0 += SW_PD) {
#pragma unroll
    for (int K = 0; K < SW_PD; ++K) {
      const int s = s0 + K;
      const int zp = z0 - 1 + s;
      const bool zin = zp >= 1 && zp <= n - 2;
      Tacc raw[NX][NR], u[NX][NR], sx[NX][NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int k = 0; k < NX; ++k) {
          raw[k][r] = (Tacc)v[K][k][r];
          if (SUM) raw[k][r] += (Tacc)v2[SUM ? K : 0][k][r];
          u[k][r] = zin && rin[r] && xin[k] ? raw[k][r] : (Tacc)0;  // interior nodes only
        }
        // across the two column blocks (x = 64 <-> x = 65), read in every lane
        const Tacc x64 = NX == 2 ? lane_value(u[0][r], 63) : (Tacc)0;
        const Tacc x65 = NX == 2 ? lane_value(u[NX - 1][r], 0) : (Tacc)0;
#pragma unroll
        for (int k = 0; k < NX; ++k) {
          Tacc lft = lane_from_left(u[k][r]), rgt = lane_from_right(u[k][r]);
          if (NX == 2 && k == 1) lft = lane == 0 ? x64 : lft;
          if (NX == 2 && k == 0) rgt = lane == 63 ? x65 : rgt;
          sx[k][r] = lft + rgt;
        }
      }
      const int zo = zp - 1;  // output plane completed in this step
      const bool st_ok = s < nsteps && zo >= z0;
      const bool bz = zo == 0 || zo == n - 1;
#pragma unroll
      for (int k = 0; k < NX; ++k)
#pragma unroll
        for (int t = 0; t < SW_TY; ++t) {
          const int r = t + 1;
          const Tacc c = u[k][r], f = u[k][r - 1] + u[k][r + 1] + sx[k][r], e = sx[k][r - 1] + sx[k][r + 1];
          const Tacc up = w1 * c + w2 * f + w3 * e;   // contribution to the planes zp - 1 and zp + 1
          const Tacc mid = w0 * c + w1 * f + w2 * e;  // contribution to plane zp
          const int gy = y0 + t;
          if (st_ok && gy < n && xact[k]) {
            const bool bnd = bz || gy == 0 || gy == n - 1 || !xin[k];  // boundary row: wb x
            Y[zo * nn + (int64_t)gy * n + xx[k]] = (Tv)(bnd ? wb * prev[k][t] : accp[k][t] + up);
          }
          accp[k][t] = accc[k][t] + mid;  // output plane zp: planes zp - 1 and zp so far
          accc[k][t] = up;                // output plane zp + 1: plane zp so far
          prev[k][t] = raw[k][r];
        }
      load(zp + SW_PD, K);
    }
  }
}

// y = S x over whole concatenated vectors (one thread per row; 1D rows get 0).
// RES = 1: r = b - S x, with partial sums of r^2 over the rows that have no
// coupling entries (the coupling-row kernel completes and sums the others).
template <typename Tv, typename Tacc, int RES>
__global__ void __launch_bounds__(BS) k_stencil(const double* __restrict__ stencil, const int32_t* __restrict__ mptr,
                                                const Tv* __restrict__ x, const double* __restrict__ bvec,
                                                Tv* __restrict__ y, const int64_t* off, int n, int n3d,
                                                const int32_t* binst, const int64_t* bstart, const int64_t* bend,
                                                const InstState* st, int mask, double* part) {
  __shared__ double sh[BS / 64];
  const int b = blockIdx.x;
  const int i = binst[b];
  if (mask == 1 && !st[i].active) return;
  if (mask == 2 && st[i].done) {
    if (RES && threadIdx.x == 0) part[b] = 0.0;
    return;
  }
  const int64_t base = off[i];
  const double* st4 = stencil + kStencilStride * i;
  double loc = 0.0;
  for (int64_t row = bstart[b] + threadIdx.x; row < bend[b]; row += BS) {
    const int r = (int)(row - base);
    const Tacc sx = r < n3d ? stencil_row<Tv, Tacc>(x, base, r, n, st4) : (Tacc)0;
    if (RES) {
      const double rv = bvec[row] - (double)sx;
      y[row] = (Tv)rv;
      if (mptr[row + 1] == mptr[row]) loc += rv * rv;
    } else {
      y[row] = (Tv)sx;
    }
  }
  if (RES) {
    const double t = block_sum(loc, sh);
    if (threadIdx.x == 0) part[b] = t;
  }
}

// Coupling rows (3D rows touched by the averaging operator and all 1D rows),
// G lanes per row: y[row] += (M x)[row] (RES = 0), the same with the 1D rows
// overwritten instead (RES = 2: y holds only the 3D stencil part),
// r[row] -= (M x)[row] with partial sums of r^2 (RES = 1), or, over the 3D
// rows only, y[row] += (M00 x)[row] leaving out the A01 entries (RES = 3;
// with x2, M00 (x + x2)).
template <typename Tv, typename Tm, typename Tacc, int G, int RES>
__global__ void __launch_bounds__(BS) k_mrows(const int32_t* __restrict__ mrows, const int32_t* __restrict__ mlp,
                                              const int32_t* __restrict__ mcol, const Tm* __restrict__ mval,
                                              const Tv* __restrict__ x, Tv* __restrict__ y, const int32_t* binst,
                                              const int64_t* bstart, const int64_t* bend, const InstState* st,
                                              int mask, double* part, int nblk, const int64_t* off = nullptr, int n3d = 0,
                                              const int32_t* __restrict__ ap = nullptr,
                                              const Tv* __restrict__ x2 = nullptr) {
  __shared__ double sh[BS / 64];
  const int b = xcd_logical_block(nblk);
  if (b < 0) return;
  const int i = binst[b];
  if (mask == 1 && !st[i].active) return;
  if (mask == 2 && st[i].done) {
    if (RES == 1 && threadIdx.x == 0) part[b] = 0.0;
    return;
  }
  const int grp = threadIdx.x / G, lane = threadIdx.x % G, ng = BS / G;
  double loc = 0.0;
  for (int64_t q = bstart[b] + grp; q < bend[b]; q += ng) {
    const int row = mrows[q];
    Tacc acc = 0;
    // RES = 3 (A00 only): the row's entries end before its A01 entries (ap)
    const int e = RES == 3 ? ap[q] : mlp[q + 1];
    // U entries per lane per pass, all loads of a pass in flight together
    // (indices clamped into the row: every listed row has entries)
    constexpr int U = 32 / G;
    for (int k0 = mlp[q] + lane; k0 < e; k0 += U * G) {
      int cidx[U];
      Tm mv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = min(k0 + u * G, e - 1);
        cidx[u] = mcol[k];
        mv[u] = mval[k];
      }
      Tacc xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = (Tacc)x[cidx[u]];
      if (RES == 3 && x2) {  // M00 (x + x2)
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] += (Tacc)x2[cidx[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k0 + u * G < e) acc += (Tacc)mv[u] * (Tacc)xv[u];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (lane == 0) {
      if (RES == 1) {
        const double rv = (double)y[row] - (double)acc;
        y[row] = (Tv)rv;
        loc += rv * rv;
      } else if (RES == 2 && row - off[i] >= n3d) {
        y[row] = (Tv)acc;  // 1D row: no stencil part
      } else {
        y[row] = (Tv)((Tacc)y[row] + acc);
      }
    }
  }
  if (RES == 1) {
    const double t = block_sum(loc, sh);
    if (threadIdx.x == 0) part[b] = t;
  }
}

// Second pass over the listed coupling rows, G lanes per row: the row's
// entries of B^T (column >= 0: a Gauss point, read from t) and of R (column
// < 0: ~index into x; x + x2 when x2 is given).  RES = 2: the sum overwrites
// a 1D row and is added to a 3D row (y holds its stencil part); RES = 3 (3D
// rows only): added.
template <typename T, int G, int RES>
__global__ void __launch_bounds__(BS) k_cscatter(const int32_t* __restrict__ mrows, const int32_t* __restrict__ sp,
                                                 const int32_t* __restrict__ scol, const T* __restrict__ sval,
                                                 const T* __restrict__ t, const T* __restrict__ x,
                                                 const T* __restrict__ x2, T* __restrict__ y, const int32_t* binst,
                                                 const int64_t* bstart, const int64_t* bend, const InstState* st,
                                                 int mask, int nblk, const int64_t* off, int n3d) {
  const int b = xcd_logical_block(nblk);
  if (b < 0) return;
  const int i = binst[b];
  if (mask == 1 && !st[i].active) return;
  const int grp = threadIdx.x / G, lane = threadIdx.x % G, ng = BS / G;
  constexpr int U = 8 / G;
  for (int64_t q = bstart[b] + grp; q < bend[b]; q += ng) {
    const int row = mrows[q];
    T acc = 0;
    const int e = sp[q + 1];
    for (int k0 = sp[q] + lane; k0 < e; k0 += U * G) {
      int c[U];
      T v[U], xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = min(k0 + u * G, e - 1);
        c[u] = scol[k];
        v[u] = sval[k];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const T* src = c[u] >= 0 ? t + c[u] : x + ~c[u];
        xv[u] = *src;
      }
      if (x2) {
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (c[u] < 0) xv[u] += x2[~c[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k0 + u * G < e) acc += v[u] * xv[u];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (lane == 0) {
      if (RES == 2 && row - off[i] >= n3d) y[row] = acc;
      else y[row] += acc;
    }
  }
}

// y = A00 x for the 3D unknowns of instance inst[slot], vectors [slot][n3d].
template <typename T, typename Tm>
__global__ void __launch_bounds__(BS) k_apply_a00(const double* __restrict__ stencil, const int32_t* __restrict__ mptr,
                                                  const int32_t* __restrict__ mcol, const Tm* __restrict__ mval,
                                                  const int64_t* off, const int32_t* ma01, const int32_t* inst,
                                                  int n, int n3d, const T* __restrict__ x, T* __restrict__ y) {
  const int slot = blockIdx.y;
  const int i = inst ? inst[slot] : slot;
  const int64_t base = off[i];
  const T* xs = x + (int64_t)slot * n3d;
  const int r = blockIdx.x * BS + threadIdx.x;
  if (r >= n3d) return;
  double acc = stencil_row<T, double>(xs, 0, r, n, stencil + kStencilStride * i);
  const int e = ma01[(int64_t)i * n3d + r];  // 3D columns end where the 1D ones start
  for (int k = mptr[base + r]; k < e; ++k) acc += (double)mval[k] * (double)xs[mcol[k] - base];
  y[(int64_t)slot * n3d + r] = (T)acc;
}

__global__ void __launch_bounds__(BS) k_norm2_part(const double* __restrict__ x, const int64_t* bstart,
                                                   const int64_t* bend, double* part) {
  __shared__ double sh[BS / 64];
  const int b = blockIdx.x;
  double loc = 0.0;
  for (int64_t e = bstart[b] + threadIdx.x; e < bend[b]; e += blockDim.x) loc += x[e] * x[e];
  double t = block_sum(loc, sh);
  if (threadIdx.x == 0) part[b] = t;
}

// r = b - r over whole vectors (r holding A x), with the partial sums of r^2
// per block; instances already done (mask 2) are skipped with a zero partial.
// The partials of the coupling-row blocks (partm, nm of them), which this form
// of the residual does not use, are cleared by the same launch.
__global__ void __launch_bounds__(BS) k_residual_part(const double* __restrict__ b, double* __restrict__ r,
                                                      const int32_t* binst, const int64_t* bstart,
                                                      const int64_t* bend, const InstState* st, int mask,
                                                      double* part, double* partm, int nm) {
  __shared__ double sh[BS / 64];
  const int blk = blockIdx.x;
  for (int k = blk * BS + threadIdx.x; k < nm; k += gridDim.x * BS) partm[k] = 0.0;
  const int i = binst[blk];
  if (mask == 2 && st[i].done) {
    if (threadIdx.x == 0) part[blk] = 0.0;
    return;
  }
  double loc = 0.0;
  for (int64_t e = bstart[blk] + threadIdx.x; e < bend[blk]; e += blockDim.x) {
    const double v = b[e] - r[e];
    r[e] = v;
    loc += v * v;
  }
  const double t = block_sum(loc, sh);
  if (threadIdx.x == 0) part[blk] = t;
}

// ---------------------------------------------------------------- cycle control

// One wavefront per instance (grid = n_inst, 64 threads).
// part holds the per-chunk squares of b, partx those of x0: a non-finite norm
// of either marks the instance as bad input (the host refuses the solve); a
// zero b has the exact solution x = 0.
__global__ void k_init_state(InstState* st, const double* part, const double* partx, const int32_t* first,
                             int n_inst, double tol, int max_iters) {
  const int i = blockIdx.x;
  if (i >= n_inst) return;
  const double s = wave_inst_sum(part, first, i);
  const double sx = wave_inst_sum(partx, first, i);
  if (threadIdx.x != 0) return;
  InstState z{};
  z.bnorm = sqrt(s);
  z.tol = tol;
  z.max_iters = max_iters;
  z.rel = 1.0;
  z.prev_rel = 1.0;
  if (!isfinite(z.bnorm) || !isfinite(sx)) {
    z.bad_input = 1;
    z.done = 1;
    z.rel = NAN;
  } else if (z.bnorm == 0.0) {
    z.done = 1;
    z.converged = 1;
    z.rel = 0.0;
  }
  st[i] = z;
}

// Start of a restart cycle: beta = ||r||, convergence and stall tests.
// One wavefront per instance (grid = n_inst, 64 threads).
__global__ void k_cycle_start(InstState* st, const double* part, const int32_t* first, const double* part2,
                              const int32_t* first2, int n_inst, double* g, double* hist, int hist_cap, int m) {
  const int i = blockIdx.x;
  if (i >= n_inst) return;
  const double s = wave_inst_sum(part, first, i) + wave_inst_sum(part2, first2, i);
  if (threadIdx.x != 0) return;
  InstState z = st[i];
  z.active = 0;
  z.jend = 0;
  if (z.done) {
    st[i] = z;
    return;
  }
  const double beta = sqrt(s);
  const double rel = beta / z.bnorm;
  if (z.nhist < hist_cap) hist[(int64_t)i * hist_cap + z.nhist++] = -rel;
  z.prev_rel = z.cycles > 0 ? z.rel : 1.0;
  z.rel = rel;
  z.beta = beta;
  z.stalled = 0;
  if (rel <= z.tol) {
    z.done = 1;
    z.converged = 1;
  } else if (!isfinite(rel)) {
    z.stalled = 2;
  } else {
    const int used = z.mode ? z.fb_iters : z.iters;
    if (used >= z.max_iters) z.stalled = 3;
    else if (z.cycles > 0 && !(rel <= 0.9 * z.prev_rel)) z.stalled = 1;
    z.active = 1;
  }
  g[(int64_t)i * (m + 1)] = beta;
  z.cycles++;
  st[i] = z;
}

template <typename T>
__global__ void __launch_bounds__(BS) k_scale_to(const double* __restrict__ r, T* __restrict__ v,
                                                 const int32_t* binst, const int64_t* bstart,
                                                 const int64_t* bend, const InstState* st) {
  const int b = blockIdx.x;
  const InstState& z = st[binst[b]];
  if (!z.active) return;
  const double inv = 1.0 / z.beta;
  for (int64_t e = bstart[b] + threadIdx.x; e < bend[b]; e += blockDim.x) v[e] = from_d<T>(r[e] * inv);
}

// ---------------------------------------------------------------- preconditioner

__device__ __forceinline__ bool mode_ok(const InstState& z, int want_mode) {
  return z.active && (want_mode < 0 || z.mode == want_mode);
}

template <typename T>
__global__ void __launch_bounds__(BS) k_prec_copy(const T* __restrict__ v, T* __restrict__ z,
                                                  const int32_t* binst, const int64_t* bstart,
                                                  const int64_t* bend, const InstState* st) {
  const int b = blockIdx.x;
  if (st && !mode_ok(st[binst[b]], 0)) return;
  for (int64_t e = bstart[b] + threadIdx.x; e < bend[b]; e += blockDim.x) z[e] = v[e];
}

template <typename T>
__global__ void __launch_bounds__(BS) k_prec_jacobi(const T* __restrict__ v, T* __restrict__ z,
                                                    const double* __restrict__ dinv, const int32_t* binst,
                                                    const int64_t* bstart, const int64_t* bend,
                                                    const InstState* st, int want_mode) {
  const int b = blockIdx.x;
  if (st && !mode_ok(st[binst[b]], want_mode)) return;
  for (int64_t e = bstart[b] + threadIdx.x; e < bend[b]; e += blockDim.x)
    z[e] = from_d<T>(to_d(v[e]) * dinv[e]);
}

// Exact 1D solve z1 = A11^-1 v1 of one instance per block: forward elimination
// level by level from the leaves (each node gathers its children), diagonal
// scaling, back substitution from the root.  Values live in LDS in FP64.
template <typename T>
__global__ void __launch_bounds__(BS) k_tree_solve(const T* __restrict__ v, T* __restrict__ z,
                                                   const int64_t* off, int n3d, const int32_t* t_off,
                                                   const int32_t* lvloff, const int32_t* lvlptr,
                                                   const int32_t* lvlnodes, const int32_t* parent,
                                                   const int32_t* childptr, const int32_t* childidx,
                                                   const double* lval, const double* tdinv,
                                                   const InstState* st, int want_mode) {
  extern __shared__ double ys[];
  const int i = blockIdx.x;
  if (st && !mode_ok(st[i], want_mode)) return;
  const int nb = t_off[i];
  const int n1d = t_off[i + 1] - nb;
  const int64_t g0 = off[i] + n3d;
  for (int c = threadIdx.x; c < n1d; c += blockDim.x) ys[c] = to_d(v[g0 + c]);
  __syncthreads();
  const int l0 = lvloff[i], nlev = lvloff[i + 1] - l0 - 1;
  for (int L = 0; L < nlev; ++L) {
    const int a = lvlptr[l0 + L], e = lvlptr[l0 + L + 1];
    for (int k = a + threadIdx.x; k < e; k += blockDim.x) {
      const int c = lvlnodes[nb + k];
      double acc = ys[c];
      const int cp0 = childptr[nb + i + c], cp1 = childptr[nb + i + c + 1];
      for (int q = cp0; q < cp1; ++q) {
        const int kid = childidx[q];
        acc -= lval[nb + kid] * ys[kid];
      }
      ys[c] = acc;
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < n1d; c += blockDim.x) ys[c] *= tdinv[nb + c];
  __syncthreads();
  for (int L = nlev - 1; L >= 0; --L) {
    const int a = lvlptr[l0 + L], e = lvlptr[l0 + L + 1];
    for (int k = a + threadIdx.x; k < e; k += blockDim.x) {
      const int c = lvlnodes[nb + k];
      const int p = parent[nb + c];
      if (p >= 0) ys[c] -= lval[nb + c] * ys[p];
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < n1d; c += blockDim.x) z[g0 + c] = from_d<T>(ys[c]);
}

// Chain-compressed solve z1 = A11^-1 v1 (same matrix as the leaves-first
// LDL^T above, elimination grouped by segment), three launches:
//  (a) k_chain_fwd, one thread per segment: y = T^-1 v_c for its tridiagonal
//      block (FP64 in registers), leaving the couplings a_p y_0, a_q y_{m-1};
//  (b) k_chain_vertex, one block per instance: the right-hand side of the
//      Schur complement on the vertices (a tree over the segments), solved
//      level by level with the vertex tree staged in LDS;
//  (c) k_chain_back, one thread per segment: recompute y, write
//      z_c = y - g_p z_p - g_q z_q.
struct ChainArgs {
  const int32_t* meta;
  const int64_t* soff;
  const double *fmul, *eup, *pinv, *gp, *gq, *ap, *aq;
  const int32_t *sp, *sq, *vparent, *vseg, *vchild_ptr, *vchild_idx, *vlvl_ptr, *vlvl_nodes;
  const double *vlval, *vdinv;
  double* t01;  // [segments][2]: a_p y_0, a_q y_{m-1}
  double* zv;   // [vertices]: FP64 vertex values
};

// y = T_s^-1 v_c in w (w from the q end, then y from the p end).
// All loads of a segment (indices clamped into range) are issued before the
// two recurrences, which then run from registers; steps beyond m are masked
// by selects.  MM >= m >= 1.
template <typename T, int MM>
__device__ __forceinline__ void chain_seg_solve(const T* __restrict__ vc, const double* fmul, const double* eup,
                                                const double* pinv, int m, int S, int s, double (&w)[MM]) {
  const int mm1 = m > 1 ? m - 2 : 0;  // last index of the [m - 1][S] arrays (clamped)
  double vr[MM], fm[MM], eu[MM], pv[MM];
#pragma unroll
  for (int k = 0; k < MM; ++k) {
    vr[k] = to_d(vc[min(k, m - 1)]);
    fm[k] = fmul[(int64_t)min(k, mm1) * S + s];
    eu[k] = eup[(int64_t)min(k > 0 ? k - 1 : 0, mm1) * S + s];
    pv[k] = pinv[(int64_t)min(k, m - 1) * S + s];
  }
  __builtin_amdgcn_sched_barrier(0);
  double wn = 0.0;
#pragma unroll
  for (int k = MM - 1; k >= 0; --k) {
    const double wk = vr[k] - (k + 1 < m ? fm[k] * wn : 0.0);
    w[k] = k < m ? wk : 0.0;
    wn = k < m ? wk : wn;
  }
  double yp = 0.0;
#pragma unroll
  for (int k = 0; k < MM; ++k) {
    const double yk = (k == 0 ? w[0] : w[k] - eu[k] * yp) * pv[k];
    w[k] = k < m ? yk : w[k];
    yp = yk;
  }
}

template <typename T, int MM>
__global__ void __launch_bounds__(64) k_chain_fwd(const T* __restrict__ v, const int64_t* off, int n3d, ChainArgs c,
                                                  const InstState* st, int want_mode) {
  const int i = blockIdx.y;
  if (st && !mode_ok(st[i], want_mode)) return;
  const int32_t* mt = c.meta + 8 * i;
  const int m = mt[0], S = mt[1], V = mt[2], so = mt[4];
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= S) return;
  double t0 = 0.0, t1 = 0.0;
  if (m > 0) {
    const int64_t o1 = c.soff[2 * i], o2 = c.soff[2 * i + 1];
    double w[MM];
    chain_seg_solve<T, MM>(v + off[i] + n3d + V + (int64_t)s * m, c.fmul + o1, c.eup + o1, c.pinv + o2, m, S, s, w);
    double last = 0.0;
#pragma unroll
    for (int k = 0; k < MM; ++k)
      if (k == m - 1) last = w[k];
    t0 = c.ap[so + s] * w[0];
    t1 = c.aq[so + s] * last;
  }
  c.t01[2 * (int64_t)(so + s)] = t0;
  c.t01[2 * (int64_t)(so + s) + 1] = t1;
}

template <typename T>
__global__ void __launch_bounds__(512) k_chain_vertex(const T* __restrict__ v, T* __restrict__ z, const int64_t* off,
                                                      int n3d, ChainArgs c, const InstState* st, int want_mode) {
  extern __shared__ double cs[];
  const int i = blockIdx.x;
  if (st && !mode_ok(st[i], want_mode)) return;
  const int32_t* mt = c.meta + 8 * i;
  const int V = mt[2], nlev = mt[3];
  const int so = mt[4], vo = mt[5], lo = mt[6], co = mt[7];
  double* rv = cs;
  double* vl = rv + V;
  double* vd = vl + V;
  int32_t* vp = (int32_t*)(vd + V);
  int32_t* vsg = vp + V;
  int32_t* vcp = vsg + V;        // V + 1
  int32_t* vci = vcp + V + 1;    // V - 1 (one parent per non-root vertex)
  int32_t* ln = vci + (V - 1);   // V
  int32_t* lp = ln + V;          // nlev + 1
  for (int u = threadIdx.x; u < V; u += blockDim.x) {
    vl[u] = c.vlval[vo + u];
    vd[u] = c.vdinv[vo + u];
    vp[u] = c.vparent[vo + u];
    vsg[u] = c.vseg[vo + u];
    ln[u] = c.vlvl_nodes[vo + u];
    if (u < V - 1) vci[u] = c.vchild_idx[co + u];
  }
  for (int u = threadIdx.x; u <= V; u += blockDim.x) vcp[u] = c.vchild_ptr[vo + i + u];
  for (int u = threadIdx.x; u <= nlev; u += blockDim.x) lp[u] = c.vlvl_ptr[lo + u];
  __syncthreads();
  const T* vv = v + off[i] + n3d;
  const double* t01 = c.t01 + 2 * (int64_t)so;
  for (int u = threadIdx.x; u < V; u += blockDim.x) {
    double r = to_d(vv[u]);
    const int ps = vsg[u];
    if (ps >= 0) r -= t01[2 * ps + 1];
    for (int q = vcp[u]; q < vcp[u + 1]; ++q) r -= t01[2 * vsg[vci[q]]];
    rv[u] = r;
  }
  __syncthreads();
  for (int L = 0; L < nlev; ++L) {
    for (int k = lp[L] + threadIdx.x; k < lp[L + 1]; k += blockDim.x) {
      const int u = ln[k];
      double acc = rv[u];
      for (int q = vcp[u]; q < vcp[u + 1]; ++q) {
        const int kid = vci[q];
        acc -= vl[kid] * rv[kid];
      }
      rv[u] = acc;
    }
    __syncthreads();
  }
  for (int u = threadIdx.x; u < V; u += blockDim.x) rv[u] *= vd[u];
  __syncthreads();
  for (int L = nlev - 1; L >= 0; --L) {
    for (int k = lp[L] + threadIdx.x; k < lp[L + 1]; k += blockDim.x) {
      const int u = ln[k];
      const int pu = vp[u];
      if (pu >= 0) rv[u] -= vl[u] * rv[pu];
    }
    __syncthreads();
  }
  T* zz = z + off[i] + n3d;
  for (int u = threadIdx.x; u < V; u += blockDim.x) {
    zz[u] = from_d<T>(rv[u]);
    c.zv[vo + u] = rv[u];
  }
}

template <typename T, int MM>
__global__ void __launch_bounds__(64) k_chain_back(const T* __restrict__ v, T* __restrict__ z, const int64_t* off,
                                                   int n3d, ChainArgs c, const InstState* st, int want_mode) {
  const int i = blockIdx.y;
  if (st && !mode_ok(st[i], want_mode)) return;
  const int32_t* mt = c.meta + 8 * i;
  const int m = mt[0], S = mt[1], V = mt[2], so = mt[4], vo = mt[5];
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= S || m == 0) return;
  const int64_t o1 = c.soff[2 * i], o2 = c.soff[2 * i + 1];
  const int64_t g0 = off[i] + n3d + V + (int64_t)s * m;
  double w[MM];
  chain_seg_solve<T, MM>(v + g0, c.fmul + o1, c.eup + o1, c.pinv + o2, m, S, s, w);
  const double zp = c.zv[vo + c.sp[so + s]], zq = c.zv[vo + c.sq[so + s]];
  const double* gp = c.gp + o2;
  const double* gq = c.gq + o2;
  double gpr[MM], gqr[MM];
#pragma unroll
  for (int k = 0; k < MM; ++k) {
    gpr[k] = gp[(int64_t)min(k, m - 1) * S + s];
    gqr[k] = gq[(int64_t)min(k, m - 1) * S + s];
  }
  T* zc = z + g0;
#pragma unroll
  for (int k = 0; k < MM; ++k)
    if (k < m) zc[k] = from_d<T>(w[k] - gpr[k] * zp - gqr[k] * zq);
}

// Extension b0 = v0 - A01 z1 (z1 already in z), one launch with two kinds of
// blocks (with sb: the first smoothing step, b0 into sb and z = omega D^-1 b0).  Blocks [0, ncopy) take chunks of 3D rows: the rows without
// coupling copy v0 and add to the partial sums of b0^2 (part3).  The other
// blocks take chunks of coupling rows, G lanes per row: b0 = v0 - A01 z1 with
// A01 in a compact CSR of its own, partial sums in part3m.  Each 3D row is
// written by exactly one block.
template <typename T, typename Tm, int G>
__global__ void __launch_bounds__(BS) k_ext(const T* __restrict__ v, T* __restrict__ z,
                                            const uint8_t* __restrict__ mfree, const int64_t* off,
                                            const int32_t* cinst, const int64_t* cstart, const int64_t* cend, int ncopy,
                                            const int32_t* __restrict__ mrows, const int32_t* __restrict__ ap,
                                            const int32_t* __restrict__ ac, const Tm* __restrict__ av,
                                            const int32_t* rinst, const int64_t* rstart, const int64_t* rend,
                                            const InstState* st, int want_mode, double* part3, double* part3m,
                                            T* __restrict__ sb, const float* __restrict__ dinv, double omega) {
  __shared__ double sh[BS / 64];
  double loc = 0.0;
  if ((int)blockIdx.x < ncopy) {
    const int b = blockIdx.x;
    const int i = cinst[b];
    if (st && !mode_ok(st[i], want_mode)) {
      if (threadIdx.x == 0) part3[b] = 0.0;
      return;
    }
    const int64_t base = off[i];
    constexpr int U = 8;
    const int64_t r1 = cend[b];
    for (int64_t r0 = cstart[b] + threadIdx.x; r0 < r1; r0 += (int64_t)U * BS) {
      T vl[U];
      bool free_row[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t g = base + min(r0 + (int64_t)u * BS, r1 - 1);
        vl[u] = v[g];
        free_row[u] = mfree[g] != 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = r0 + (int64_t)u * BS;
        if (r >= r1) break;
        if (free_row[u]) {
          if (sb) {  // first smoothing step from zero
            sb[base + r] = vl[u];
            z[base + r] = from_d<T>(omega * (double)dinv[base + r] * to_d(vl[u]));
          } else {
            z[base + r] = vl[u];
          }
          loc += to_d(vl[u]) * to_d(vl[u]);
        }
      }
    }
    const double t = block_sum(loc, sh);
    if (threadIdx.x == 0) part3[b] = t;
    return;
  }
  const int b = blockIdx.x - ncopy;
  const int i = rinst[b];
  if (st && !mode_ok(st[i], want_mode)) {
    if (threadIdx.x == 0) part3m[b] = 0.0;
    return;
  }
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  constexpr int NG = BS / G, U = 2;
  for (int64_t q = rstart[b] + grp; q < rend[b]; q += NG) {
    const int row = mrows[q];
    const int e0 = ap[q], e1 = ap[q + 1];
    const T vr = v[row];
    double acc = 0.0;
    for (int k0 = e0 + lane; k0 < e1; k0 += U * G) {
      int cidx[U];
      Tm mv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = min(k0 + u * G, e1 - 1);
        cidx[u] = ac[k];
        mv[u] = av[k];
      }
      T zv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) zv[u] = z[cidx[u]];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k0 + u * G < e1) acc += (double)mv[u] * to_d(zv[u]);
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (lane == 0) {
      const T stored = from_d<T>(to_d(vr) - acc);
      if (sb) {
        sb[row] = stored;
        z[row] = from_d<T>(omega * (double)dinv[row] * to_d(stored));
      } else {
        z[row] = stored;
      }
      loc += to_d(stored) * to_d(stored);
    }
  }
  const double t = block_sum(loc, sh);
  if (threadIdx.x == 0) part3m[b] = t;
}

template <typename T>
__global__ void __launch_bounds__(BS) k_block_jacobi3d(T* __restrict__ z, const double* __restrict__ dinv,
                                                       const int64_t* off, const int32_t* binst,
                                                       const int64_t* bstart, const int64_t* bend,
                                                       const InstState* st, int want_mode) {
  const int b = blockIdx.x;
  const int i = binst[b];
  if (st && !mode_ok(st[i], want_mode)) return;
  const int64_t base = off[i];
  for (int64_t r = bstart[b] + threadIdx.x; r < bend[b]; r += blockDim.x)
    z[base + r] = from_d<T>(to_d(z[base + r]) * dinv[base + r]);
}

// One wavefront per instance (grid = n_inst, 64 threads).
__global__ void k_inv_scale(const double* part3, const int32_t* first, const double* part4, const int32_t* first4,
                            int n_inst, double* inv_s, InstState* st, int want_mode) {
  const int i = blockIdx.x;
  if (i >= n_inst) return;
  if (st && !mode_ok(st[i], want_mode)) return;
  double s = wave_inst_sum(part3, first, i) + (part4 ? wave_inst_sum(part4, first4, i) : 0.0);
  if (threadIdx.x != 0) return;
  s = sqrt(s);
  inv_s[i] = s > 0.0 ? 1.0 / s : 0.0;
  inv_s[n_inst + i] = s;
  if (st) st[i].scale3d = s;
}

// ---------------------------------------------------------------- Jacobi smoothing of the 3D solve
// Damped Jacobi relaxation z <- z + omega D^-1 (b0 - A00 z) around the network
// (Section 5, pre- and post-smoothing), over the 3D rows of the instances on
// the configured preconditioner.  D = diag(A00) (unit on Dirichlet rows).  The
// first step from z = 0 (z = omega D^-1 b0, b0 kept in sb) is taken by the
// extension kernel.

// z += x over the 3D rows.
template <typename T>
__global__ void __launch_bounds__(BS) k_vec_add3d(T* __restrict__ z, const T* __restrict__ x, const int64_t* off,
                                                  const int32_t* binst, const int64_t* bstart, const int64_t* bend,
                                                  const InstState* st) {
  const int b = blockIdx.x;
  const int i = binst[b];
  if (st && !mode_ok(st[i], 0)) return;
  const int64_t base = off[i];
  for (int64_t r = bstart[b] + threadIdx.x; r < bend[b]; r += BS)
    z[base + r] = from_d<T>(to_d(z[base + r]) + to_d(x[base + r]));
}

// One relaxation step z <- (z + x2) + omega D^-1 (sb - t) with t = A00 (z + x2)
// (x2 = the network's correction, or null).
template <typename T>
__global__ void __launch_bounds__(BS) k_smooth_sweep(T* __restrict__ z, const T* __restrict__ x2,
                                                     const T* __restrict__ sb, const T* __restrict__ t,
                                                     const float* __restrict__ dinv, double omega, const int64_t* off,
                                                     const int32_t* binst, const int64_t* bstart, const int64_t* bend,
                                                     const InstState* st) {
  const int b = blockIdx.x;
  const int i = binst[b];
  if (st && !mode_ok(st[i], 0)) return;
  const int64_t base = off[i];
  constexpr int U = 4;
  const int64_t r1 = bend[b];
  for (int64_t r0 = bstart[b] + threadIdx.x; r0 < r1; r0 += (int64_t)U * BS) {
    T zl[U], xl[U], bl[U], tl[U];
    float dl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t g = base + min(r0 + (int64_t)u * BS, r1 - 1);
      zl[u] = z[g];
      xl[u] = x2 ? x2[g] : (T)0;
      bl[u] = sb[g];
      tl[u] = t[g];
      dl[u] = dinv[g];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + (int64_t)u * BS;
      if (r >= r1) break;
      z[base + r] = from_d<T>(to_d(zl[u]) + to_d(xl[u]) + omega * (double)dl[u] * (to_d(bl[u]) - to_d(tl[u])));
    }
  }
}

// Residual of the pre-smoothed z: sr = sb - t (t = A00 z), the network input,
// with per-block partial sums of sr^2 for its normalisation.  The network
// overwrites sr on the free nodes with its correction; on the Dirichlet rows
// the 3D solver returns its input, so sr is already the correction there.
template <typename T>
__global__ void __launch_bounds__(BS) k_smooth_res(const T* __restrict__ sb, const T* __restrict__ t,
                                                   T* __restrict__ sr, const int64_t* off, const int32_t* binst,
                                                   const int64_t* bstart, const int64_t* bend, const InstState* st,
                                                   double* part) {
  __shared__ double sh[BS / 64];
  const int b = blockIdx.x;
  const int i = binst[b];
  if (st && !mode_ok(st[i], 0)) {
    if (threadIdx.x == 0) part[b] = 0.0;
    return;
  }
  const int64_t base = off[i];
  double loc = 0.0;
  constexpr int U = 4;
  const int64_t r1 = bend[b];
  for (int64_t r0 = bstart[b] + threadIdx.x; r0 < r1; r0 += (int64_t)U * BS) {
    T bl[U], tl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t g = base + min(r0 + (int64_t)u * BS, r1 - 1);
      bl[u] = sb[g];
      tl[u] = t[g];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + (int64_t)u * BS;
      if (r >= r1) break;
      const T rv = from_d<T>(to_d(bl[u]) - to_d(tl[u]));
      sr[base + r] = rv;
      loc += to_d(rv) * to_d(rv);
    }
  }
  const double tt = block_sum(loc, sh);
  if (threadIdx.x == 0) part[b] = tt;
}

// ---------------------------------------------------------------- inner FGMRES on the 3D block
// The 3D solve of Section 6: K FGMRES steps on A00 z0 = b0 from z0 = 0 with
// the network as right preconditioner.  Basis vectors IV[0..K] and directions
// IZ[0..K-1] are full-length vectors whose 1D parts stay zero.

// IV[0] = b0 / ||b0|| (b0 in z, inv_s from its partials).
template <typename T>
__global__ void __launch_bounds__(BS) k_inner_start(const T* __restrict__ z, T* __restrict__ v0,
                                                    const double* __restrict__ inv_s, const int64_t* off,
                                                    const int32_t* binst, const int64_t* bstart, const int64_t* bend,
                                                    const InstState* st) {
  const int b = blockIdx.x;
  const int i = binst[b];
  if (st && !mode_ok(st[i], 0)) return;
  const int64_t base = off[i];
  const double sc = inv_s[i];
  for (int64_t r = bstart[b] + threadIdx.x; r < bend[b]; r += BS)
    v0[base + r] = from_d<T>(to_d(z[base + r]) * sc);
}

// dst = src over the 3D rows (the network's value on the Dirichlet rows is its input).
template <typename T>
__global__ void __launch_bounds__(BS) k_copy3d(const T* __restrict__ src, T* __restrict__ dst, const int64_t* off,
                                               const int32_t* binst, const int64_t* bstart, const int64_t* bend,
                                               const InstState* st) {
  const int b = blockIdx.x;
  const int i = binst[b];
  if (st && !mode_ok(st[i], 0)) return;
  const int64_t base = off[i];
  for (int64_t r = bstart[b] + threadIdx.x; r < bend[b]; r += BS) dst[base + r] = src[base + r];
}

// End of inner step j: h = ||w|| from the last Gram-Schmidt pass, stored with
// ||w|| before orthogonalisation (breakdown test); w /= h unless this is the
// last step (h = 0 leaves a zero vector).
template <typename T>
__global__ void __launch_bounds__(BS) k_inner_finish(T* __restrict__ w, const double* __restrict__ part_last,
                                                     const double* __restrict__ part_w0, double* __restrict__ IH,
                                                     double* __restrict__ IH0, int j, int K, int scale,
                                                     const int32_t* binst, const int64_t* bstart,
                                                     const int64_t* bend, const int32_t* first,
                                                     const InstState* st) {
  const int b = blockIdx.x;
  const int i = binst[b];
  if (st && !mode_ok(st[i], 0)) return;
  const double hn = sqrt(wave_inst_sum(part_last, first, i));
  if (b == first[i] && threadIdx.x == 0) {
    IH[((int64_t)i * (K + 1) + (j + 1)) * K + j] = hn;
    IH0[(int64_t)i * K + j] = sqrt(wave_inst_sum(part_w0, first, i));
  }
  if (!scale) return;
  const double sc = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int64_t e = bstart[b] + threadIdx.x; e < bend[b]; e += BS) w[e] = from_d<T>(to_d(w[e]) * sc);
}

// Least squares of the inner solve, one thread per instance: Givens rotations
// on the (K+1) x K Hessenberg matrix with g = ||b0|| e1, steps up to the first
// breakdown (h_{j+1,j} <= 1e-14 ||A00 z_j||), back substitution into y.
__global__ void k_inner_lsq(const double* __restrict__ IH, const double* __restrict__ IH0,
                            const double* __restrict__ inv_s, double* __restrict__ y, int* __restrict__ jend_out,
                            int K, int n_inst, const InstState* st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  if (st && !mode_ok(st[i], 0)) return;
  constexpr int KM = 8;
  double H[KM + 1][KM], g[KM + 1], c[KM], s[KM];
  const double* Hi = IH + (int64_t)i * (K + 1) * K;
  for (int r = 0; r <= K; ++r)
    for (int q = 0; q < K; ++q) H[r][q] = Hi[r * K + q];
  for (int r = 0; r <= K; ++r) g[r] = 0.0;
  g[0] = inv_s[n_inst + i];  // ||b0||
  int jend = 0;
  for (int j = 0; j < K; ++j) {
    for (int q = 0; q < j; ++q) {
      const double t = c[q] * H[q][j] + s[q] * H[q + 1][j];
      H[q + 1][j] = -s[q] * H[q][j] + c[q] * H[q + 1][j];
      H[q][j] = t;
    }
    const double a = H[j][j], bb = H[j + 1][j];
    const double den = hypot(a, bb);
    c[j] = den == 0.0 ? 1.0 : a / den;
    s[j] = den == 0.0 ? 0.0 : bb / den;
    H[j][j] = c[j] * a + s[j] * bb;
    g[j + 1] = -s[j] * g[j];
    g[j] = c[j] * g[j];
    jend = j + 1;
    if (bb <= 1e-14 * IH0[(int64_t)i * K + j]) break;
  }
  double* yi = y + (int64_t)i * K;
  for (int q = 0; q < K; ++q) yi[q] = 0.0;
  for (int q = jend - 1; q >= 0; --q) {
    double acc = g[q];
    for (int p = q + 1; p < jend; ++p) acc -= H[q][p] * yi[p];
    yi[q] = H[q][q] != 0.0 ? acc / H[q][q] : 0.0;
  }
  jend_out[i] = jend;
}

// z0 = sum_j y_j IZ[j] over the 3D rows.
template <typename T>
__global__ void __launch_bounds__(BS) k_inner_combine(T* __restrict__ z, const T* __restrict__ IZ, int64_t ld,
                                                      const double* __restrict__ y, const int* __restrict__ jend,
                                                      int K, const int64_t* off, const int32_t* binst,
                                                      const int64_t* bstart, const int64_t* bend,
                                                      const InstState* st) {
  const int b = blockIdx.x;
  const int i = binst[b];
  if (st && !mode_ok(st[i], 0)) return;
  const int64_t base = off[i];
  const int je = jend[i];
  const double* yi = y + (int64_t)i * K;
  for (int64_t r = bstart[b] + threadIdx.x; r < bend[b]; r += BS) {
    double acc = 0.0;
    for (int q = 0; q < je; ++q) acc += yi[q] * to_d(IZ[(int64_t)q * ld + base + r]);
    z[base + r] = from_d<T>(acc);
  }
}

// ---------------------------------------------------------------- Arnoldi (modified Gram-Schmidt)

// Modified Gram-Schmidt for the new vector w = V[j+1], taken kMgsGroup basis
// vectors per pass.  Within a group the sequential MGS coefficients follow from
// inner products taken with the group's input w:
//   h_b = <w - sum_{a<b} h_a v_a, v_b> = <w, v_b> - sum_{a<b} h_a <v_a, v_b>,
// an identity of exact arithmetic (the <v_a, v_b> are kept, not assumed zero),
// so one pass over w serves a whole group.  A pass
//   - forms the coefficients of the previous group (NPD vectors from p0) from
//     that pass's partial sums and subtracts them from w, which is stored back
//     rounded once to the vector type;
//   - takes the partials of <w, v_c> and <v_a, v_b> for the NCU vectors of the
//     current group (from c0), or of <w, w> when the group is empty (last pass);
//   - on the first pass, also those of <w, w> before orthogonalisation.
// Partial q of block b sits at part[q * nblk + b]; dots first, then the pairs
// a < b at NCU + b (b - 1) / 2 + a.  FP64 arithmetic throughout.
template <typename T, int NPD, int NCU>
__global__ void __launch_bounds__(BS) k_mgs(T* __restrict__ V, int64_t ld, int j, int p0, int c0,
                                            const double* __restrict__ part_prev, double* __restrict__ part_cur,
                                            double* __restrict__ part_w0, double* __restrict__ H, int m,
                                            const int32_t* binst, const int64_t* bstart, const int64_t* bend,
                                            const int32_t* first, const InstState* st, int nblk) {
  constexpr int NPV = NPD + NPD * (NPD - 1) / 2;              // partial sums read
  constexpr int NCV = NCU > 0 ? NCU + NCU * (NCU - 1) / 2 : 1;  // partial sums written
  constexpr int NSH = (NPV > NCV ? NPV : NCV) + 1;
  constexpr int NVEC = 1 + NPD + NCU;
  constexpr int U = NVEC <= 3 ? 8 : 4;  // elements per thread per pass
  __shared__ double sh[NSH * (BS / 64)];
  const int b = blockIdx.x;
  const int i = binst[b];
  if (st && !st[i].active) return;
  T* w = V + (int64_t)(j + 1) * ld;
  const int f0 = first[i], f1 = first[i + 1];
  const int t = (int)threadIdx.x;
  // previous pass's partials: the first BS blocks of the instance in flight
  // before the element loads, the rest (large instances) summed up front
  double hp[NPV > 0 ? NPV : 1];
  double hq[NPV > 0 ? NPV : 1];
#pragma unroll
  for (int q = 0; q < NPV; ++q) hp[q] = 0.0;
  for (int r = f0 + t + BS; r < f1; r += BS) {
#pragma unroll
    for (int q = 0; q < NPV; ++q) hp[q] += part_prev[(int64_t)q * nblk + r];
  }
#pragma unroll
  for (int q = 0; q < NPV; ++q) hq[q] = part_prev[(int64_t)q * nblk + min(f0 + t, f1 - 1)];
  // uniform base pointers at the block's first element and 32-bit byte
  // offsets shared by all vectors (SGPR base + VGPR offset addressing)
  const int64_t es = bstart[b];
  const int len = (int)(bend[b] - es);
  T* wb = w + es;
  const char* pbase[NPD > 0 ? NPD : 1];
  const char* cbase[NCU > 0 ? NCU : 1];
#pragma unroll
  for (int a = 0; a < NPD; ++a) pbase[a] = (const char*)(V + (int64_t)(p0 + a) * ld + es);
#pragma unroll
  for (int c = 0; c < NCU; ++c) cbase[c] = (const char*)(V + (int64_t)(c0 + c) * ld + es);
  int e0 = t;
  T wl[U], pl[NPD > 0 ? NPD : 1][U], cl[NCU > 0 ? NCU : 1][U];
  auto load_pass = [&](int ea, T (&wa)[U], T (&pa)[NPD > 0 ? NPD : 1][U], T (&ca)[NCU > 0 ? NCU : 1][U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t off = (uint32_t)min(ea + u * BS, len - 1) * (uint32_t)sizeof(T);
      wa[u] = *(const T*)((const char*)wb + off);
#pragma unroll
      for (int a = 0; a < NPD; ++a) pa[a][u] = *(const T*)(pbase[a] + off);
#pragma unroll
      for (int c = 0; c < NCU; ++c) ca[c][u] = *(const T*)(cbase[c] + off);
    }
  };
  __builtin_amdgcn_sched_barrier(0);
  if (e0 < len) load_pass(e0, wl, pl, cl);
  __builtin_amdgcn_sched_barrier(0);
  double h[NPD > 0 ? NPD : 1];
  if constexpr (NPD > 0) {
#pragma unroll
    for (int q = 0; q < NPV; ++q)
      if (f0 + t < f1) hp[q] += hq[q];
    block_sums_lds<NPV>(hp, sh);
    // sequential MGS coefficients of the previous group
#pragma unroll
    for (int bb = 0; bb < NPD; ++bb) {
      double v = hp[bb];
#pragma unroll
      for (int a = 0; a < bb; ++a) v -= h[a] * hp[NPD + bb * (bb - 1) / 2 + a];
      h[bb] = v;
    }
    if (b == f0 && t < NPD) {
      double ht = h[0];
#pragma unroll
      for (int a = 1; a < NPD; ++a)
        if (t == a) ht = h[a];
      H[((int64_t)i * (m + 1) + (p0 + t)) * m + j] = ht;
    }
  }
  double acc[NCV], acc0 = 0.0;
#pragma unroll
  for (int q = 0; q < NCV; ++q) acc[q] = 0.0;
  T wn[U], pn[NPD > 0 ? NPD : 1][U], cn[NCU > 0 ? NCU : 1][U];
  for (; e0 < len; e0 += U * BS) {
    const bool more = e0 + U * BS < len;
    if (more) load_pass(e0 + U * BS, wn, pn, cn);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * BS;
      if (e >= len) break;
      double wv = to_d(wl[u]);
      if constexpr (NPD == 0) acc0 += wv * wv;
      if constexpr (NPD > 0) {
#pragma unroll
        for (int a = 0; a < NPD; ++a) wv -= h[a] * to_d(pl[a][u]);
        const T ws = from_d<T>(wv);
        wb[e] = ws;
        wv = to_d(ws);
      }
      if constexpr (NCU > 0) {
#pragma unroll
        for (int c = 0; c < NCU; ++c) acc[c] += wv * to_d(cl[c][u]);
#pragma unroll
        for (int bb = 1; bb < NCU; ++bb)
#pragma unroll
          for (int a = 0; a < bb; ++a) acc[NCU + bb * (bb - 1) / 2 + a] += to_d(cl[a][u]) * to_d(cl[bb][u]);
      } else {
        acc[0] += wv * wv;
      }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        wl[u] = wn[u];
#pragma unroll
        for (int a = 0; a < NPD; ++a) pl[a][u] = pn[a][u];
#pragma unroll
        for (int c = 0; c < NCU; ++c) cl[c][u] = cn[c][u];
      }
    }
  }
  if constexpr (NPD == 0) {
    double all[NCV + 1];
#pragma unroll
    for (int q = 0; q < NCV; ++q) all[q] = acc[q];
    all[NCV] = acc0;
    block_sums_lds<NCV + 1>(all, sh);
    if (t < NCV) {
      double o = all[0];
#pragma unroll
      for (int q = 1; q < NCV; ++q)
        if (t == q) o = all[q];
      part_cur[(int64_t)t * nblk + b] = o;
    }
    if (t == 0) part_w0[b] = all[NCV];
  } else {
    block_sums_lds<NCV>(acc, sh);
    if (t < NCV) {
      double o = acc[0];
#pragma unroll
      for (int q = 1; q < NCV; ++q)
        if (t == q) o = acc[q];
      part_cur[(int64_t)t * nblk + b] = o;
    }
  }
}

// End of Arnoldi step j: h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}; the first
// block of each instance applies the previous Givens rotations to column j,
// forms rotation j, updates g and the residual estimate rho = |g_{j+1}|, and
// retires the instance on convergence, happy breakdown or the step cap.
template <typename T>
__global__ void __launch_bounds__(BS) k_mgs_finish(T* __restrict__ V, int64_t ld, int j,
                                                   const double* __restrict__ part_last,
                                                   const double* __restrict__ part_w0, double* __restrict__ H,
                                                   double* __restrict__ cs, double* __restrict__ sn,
                                                   double* __restrict__ g, double* __restrict__ hist, int hist_cap,
                                                   int m, const int32_t* binst, const int64_t* bstart,
                                                   const int64_t* bend, const int32_t* first, InstState* st) {
  __shared__ double sh[BS / 64];
  const int b = blockIdx.x;
  const int i = binst[b];
  if (!st[i].active) return;
  T* w = V + (int64_t)(j + 1) * ld;
  // partials of both norms and the first pass of w are all in flight before
  // the block reductions
  constexpr int U = 8, NP = 4;
  const int f0 = first[i], f1 = first[i + 1];
  double pa = 0.0, pb = 0.0;
  for (int q = f0 + (int)threadIdx.x + NP * BS; q < f1; q += BS) {  // instances of more than NP BS blocks
    pa += part_last[q];
    pb += part_w0[q];
  }
  double qa[NP], qb[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int q = min(f0 + (int)threadIdx.x + u * BS, f1 - 1);
    qa[u] = part_last[q];
    qb[u] = part_w0[q];
  }
  const int64_t e1 = bend[b];
  int64_t e0 = bstart[b] + threadIdx.x;
  T wl[U];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < U; ++u) wl[u] = w[min(e0 + (int64_t)u * BS, e1 - 1)];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < NP; ++u)
    if (f0 + (int)threadIdx.x + u * BS < f1) {
      pa += qa[u];
      pb += qb[u];
    }
  const double hn = sqrt(block_sum_lds(pa, sh));
  const double w0 = sqrt(block_sum_lds(pb, sh));
  const double sc = hn > 0.0 ? 1.0 / hn : 0.0;
  for (; e0 < e1; e0 += (int64_t)U * BS) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * BS;
      if (e < e1) w[e] = from_d<T>(to_d(wl[u]) * sc);
    }
    const int64_t en = e0 + (int64_t)U * BS;
    if (en < e1) {
#pragma unroll
      for (int u = 0; u < U; ++u) wl[u] = w[min(en + (int64_t)u * BS, e1 - 1)];
    }
  }
  if (b != first[i]) return;
  double* Hc = H + (int64_t)i * (m + 1) * m;  // Hc[row * m + col]
  double* c = cs + (int64_t)i * m;
  double* s = sn + (int64_t)i * m;
  double* gi = g + (int64_t)i * (m + 1);
  // column j and the previous rotations staged in LDS by the whole block, so
  // that the sequential rotation sweep below reads no global memory
  constexpr int MR = 128;
  __shared__ double hcol[MR + 1], csh[MR], snh[MR];
  const bool staged = j < MR;
  if (staged) {
    for (int q = threadIdx.x; q <= j; q += blockDim.x) {
      hcol[q] = Hc[q * m + j];
      if (q < j) {
        csh[q] = c[q];
        snh[q] = s[q];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double a;
  if (staged) {
    double carry = hcol[0];  // rotated entry q of the column
    for (int q = 0; q < j; ++q) {
      const double x0 = carry, x1 = hcol[q + 1];
      Hc[q * m + j] = csh[q] * x0 + snh[q] * x1;
      carry = -snh[q] * x0 + csh[q] * x1;
    }
    a = carry;
  } else {
    for (int q = 0; q < j; ++q) {
      const double x0 = Hc[q * m + j], x1 = Hc[(q + 1) * m + j];
      Hc[q * m + j] = c[q] * x0 + s[q] * x1;
      Hc[(q + 1) * m + j] = -s[q] * x0 + c[q] * x1;
    }
    a = Hc[j * m + j];
  }
  const double bb = hn;
  const double den = hypot(a, bb);
  const double cj = den == 0.0 ? 1.0 : a / den, sj = den == 0.0 ? 0.0 : bb / den;
  c[j] = cj;
  s[j] = sj;
  Hc[j * m + j] = cj * a + sj * bb;
  Hc[(j + 1) * m + j] = 0.0;
  gi[j + 1] = -sj * gi[j];
  gi[j] = cj * gi[j];
  const double rho = fabs(gi[j + 1]);
  InstState z = st[i];
  if (z.mode) z.fb_iters++; else z.iters++;
  z.jend = j + 1;
  if (z.nhist < hist_cap) hist[(int64_t)i * hist_cap + z.nhist++] = rho / z.bnorm;
  const int used = z.mode ? z.fb_iters : z.iters;
  if (rho <= z.tol * z.bnorm || hn <= 1e-14 * w0 || used >= z.max_iters || !isfinite(rho)) z.active = 0;
  st[i] = z;
}

// y = R^-1 g (upper triangular, FP64), one thread per instance.
__global__ void k_solve_y(const double* H, const double* g, double* y, int m, int n_inst, const InstState* st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  const int je = st[i].jend;
  const double* Hc = H + (int64_t)i * (m + 1) * m;
  const double* gi = g + (int64_t)i * (m + 1);
  double* yi = y + (int64_t)i * m;
  for (int q = je - 1; q >= 0; --q) {
    double acc = gi[q];
    for (int p = q + 1; p < je; ++p) acc -= Hc[q * m + p] * yi[p];
    const double d = Hc[q * m + q];
    yi[q] = d != 0.0 ? acc / d : 0.0;
  }
}

// x += Z y over the Arnoldi steps taken in this cycle.
template <typename T>
__global__ void __launch_bounds__(BS) k_update_x(const T* __restrict__ Z, int64_t ld, const double* __restrict__ y,
                                                 double* __restrict__ x, int m, const int32_t* binst,
                                                 const int64_t* bstart, const int64_t* bend,
                                                 const InstState* st) {
  const int b = blockIdx.x;
  const int i = binst[b];
  const int je = st[i].jend;
  if (je == 0) return;
  const double* yi = y + (int64_t)i * m;
  // four basis vectors per pass, loads issued before use (same summation order)
  constexpr int QU = 4;
  for (int64_t e = bstart[b] + threadIdx.x; e < bend[b]; e += blockDim.x) {
    double acc = x[e];
    for (int q0 = 0; q0 < je; q0 += QU) {
      T zl[QU];
#pragma unroll
      for (int u = 0; u < QU; ++u) zl[u] = Z[(int64_t)min(q0 + u, je - 1) * ld + e];
#pragma unroll
      for (int u = 0; u < QU; ++u)
        if (q0 + u < je) acc += yi[q0 + u] * to_d(zl[u]);
    }
    x[e] = acc;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers

#define BLK(s) (s)->blk.inst, (s)->blk.start, (s)->blk.end
#define BLK3(s) (s)->blk3.inst, (s)->blk3.start, (s)->blk3.end

#define MBLK(s) (s)->mblk.inst, (s)->mblk.start, (s)->mblk.end
#define MBLK3(s) (s)->mblk3.inst, (s)->mblk3.start, (s)->mblk3.end

// The stencil sweep over the batch: waves of SW_TY rows x a z range, the z
// split aimed at s->sweep_target waves (default 2048), plus the x = 0 copy
// waves.  Only for n <= SW_NMAX.
template <typename T, int SUM, int CG = 0>
void launch_sweep(mdnp_sys* s, const T* x, T* y, const T* x2, const InstState* st, int mk, hipStream_t stream) {
  const int n = s->n;
  const int ytiles = (n + SW_TY - 1) / SW_TY;
  const int target = s->sweep_target > 0 ? s->sweep_target : 2048;
  int nz = (target + ytiles * s->n_inst - 1) / (ytiles * s->n_inst);
  nz = std::max(1, std::min(nz, n));
  const int zc = (n + nz - 1) / nz;
  nz = (n + zc - 1) / zc;
  const int nfz = (n + SW_FZ - 1) / SW_FZ;
  const int ntile = (nfz + ytiles * nz) * s->n_inst;
  CgArgs cg;
  if (CG) {
    cg.gp = s->d_gp;
    cg.gsplit = s->d_gsplit;
    cg.gcol = s->d_gcol;
    cg.gval = sizeof(T) == 8 ? (const void*)s->d_gval64 : (const void*)s->d_gval32;
    cg.t = s->d_ct;
    cg.binst = s->gblk.inst;
    cg.bstart = s->gblk.start;
    cg.bend = s->gblk.end;
    cg.nblk = s->gblk.nblk;
  }
  const dim3 grid(xcd_grid((ntile + 3) / 4) + (CG ? xcd_grid(cg.nblk) : 0u));
  if (n <= 65)
    hipLaunchKernelGGL((k_stencil_sweep<T, T, SUM, 1, CG>), grid, dim3(256), 0, stream, s->d_stencil, x, y, s->d_off,
                       n, ytiles, zc, nfz, ntile, st, mk, x2, cg);
  else
    hipLaunchKernelGGL((k_stencil_sweep<T, T, SUM, 2, CG>), grid, dim3(256), 0, stream, s->d_stencil, x, y, s->d_off,
                       n, ytiles, zc, nfz, ntile, st, mk, x2, cg);
}

// Second pass of the factored coupling over the listed rows (all, or the 3D
// rows for A00).  Its input t is one buffer per system: calls on one system
// are serialised on its stream.
template <typename T>
void launch_coupling_rows(mdnp_sys* s, const T* x, T* y, const InstState* st, int mk, bool a00, hipStream_t stream,
                          const T* x2 = nullptr) {
  const T* sv = sizeof(T) == 8 ? (const T*)s->d_sval64 : (const T*)s->d_sval32;
  if (a00)
    hipLaunchKernelGGL((k_cscatter<T, CS_G, 3>), dim3(xcd_grid(s->mblk3.nblk)), dim3(BS), 0, stream, s->d_mrows,
                       s->d_sp, s->d_scol, sv, (const T*)s->d_ct, x, x2, y, MBLK3(s), st, mk, s->mblk3.nblk, s->d_off,
                       s->n3d);
  else
    hipLaunchKernelGGL((k_cscatter<T, CS_G, 2>), dim3(xcd_grid(s->mblk.nblk)), dim3(BS), 0, stream, s->d_mrows,
                       s->d_sp, s->d_scol, sv, (const T*)s->d_ct, x, (const T*)nullptr, y, MBLK(s), st, mk,
                       s->mblk.nblk, s->d_off, s->n3d);
}

template <typename T>
void launch_spmv(mdnp_sys* s, const T* x, T* y, const InstState* st, bool mask, hipStream_t stream) {
  const int mk = mask ? 1 : 0;
  const int n = s->n;
  if (n > SW_NMAX) {  // one thread per row
    if (sizeof(T) == 8) {
      hipLaunchKernelGGL((k_stencil<T, double, 0>), dim3(s->blk.nblk), dim3(BS), 0, stream, s->d_stencil, s->d_mptr,
                         x, (const double*)nullptr, y, s->d_off, s->n, s->n3d, BLK(s), st, mk, (double*)nullptr);
      hipLaunchKernelGGL((k_mrows<T, double, double, 8, 0>), dim3(xcd_grid(s->mblk.nblk)), dim3(BS), 0, stream, s->d_mrows,
                         s->d_mlp, s->d_mcol, s->d_mval64, x, y, MBLK(s), st, mk, (double*)nullptr, s->mblk.nblk);
    } else {
      hipLaunchKernelGGL((k_stencil<T, float, 0>), dim3(s->blk.nblk), dim3(BS), 0, stream, s->d_stencil, s->d_mptr,
                         x, (const double*)nullptr, y, s->d_off, s->n, s->n3d, BLK(s), st, mk, (double*)nullptr);
      hipLaunchKernelGGL((k_mrows<T, float, float, 8, 0>), dim3(xcd_grid(s->mblk.nblk)), dim3(BS), 0, stream, s->d_mrows,
                         s->d_mlp, s->d_mcol, s->d_mval32, x, y, MBLK(s), st, mk, (double*)nullptr, s->mblk.nblk);
    }
    return;
  }
  launch_sweep<T, 0, 1>(s, x, y, (const T*)nullptr, st, mk, stream);
  launch_coupling_rows<T>(s, x, y, st, mk, false, stream);
}
template void launch_spmv<float>(mdnp_sys*, const float*, float*, const InstState*, bool, hipStream_t);
template void launch_spmv<double>(mdnp_sys*, const double*, double*, const InstState*, bool, hipStream_t);

// Chooses s->sweep_target (the wave count the stencil sweep's z split aims at)
// by timing batches of back-to-back SpMV launches on the system itself with
// HIP events (best of three batches of 20 per candidate).  The split only
// moves output planes between waves: y is the same for every choice.
template <typename T>
static bool spmv_autotune_t(mdnp_sys* s, hipStream_t stream) {
  static const int kTargets[] = {1024, 1536, 2048, 3072, 4096, 6144};
  T* buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t nt = (size_t)s->ntot;
  bool ok = hipMalloc(&buf, sizeof(T) * 2 * nt) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
            hipEventCreate(&e1) == hipSuccess &&
            hipMemsetAsync(buf, 0, sizeof(T) * 2 * nt, stream) == hipSuccess;
  if (ok) {
    int best_t = s->sweep_target;
    float best = 1e30f;
    for (int target : kTargets) {
      s->sweep_target = target;
      launch_spmv<T>(s, buf, buf + nt, nullptr, false, stream);  // warm-up
      for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, stream);
        for (int k = 0; k < 20; ++k) launch_spmv<T>(s, buf, buf + nt, nullptr, false, stream);
        (void)hipEventRecord(e1, stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          best_t = target;
        }
      }
    }
    s->sweep_target = best_t;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) (void)hipFree(buf);
  return ok;
}

bool spmv_autotune(mdnp_sys* s, hipStream_t stream) {
  if (s->n > SW_NMAX) return true;  // no sweep at this size
  return s->vec_dtype == MDNP_F64 ? spmv_autotune_t<double>(s, stream) : spmv_autotune_t<float>(s, stream);
}

// y = A00 x (or A00 (x + x2)) on the 3D rows of the instances on the configured
// preconditioner (full-length vectors, 1D parts of y left at zero or
// untouched): the stencil, then the 3D coupling rows without their A01
// entries.  x2 only where the stencil sweep applies (n <= SW_NMAX).
template <typename T>
void launch_a00(mdnp_sys* s, const T* x, T* y, const InstState* st, hipStream_t stream, const T* x2) {
  const int n = s->n;
  const int mk = st ? 1 : 0;
  typedef typename std::conditional<sizeof(T) == 8, double, float>::type Tm;
  const Tm* mv = sizeof(T) == 8 ? (const Tm*)s->d_mval64 : (const Tm*)s->d_mval32;
  if (n > SW_NMAX) {  // one thread per row (1D rows of y get 0); x2 not taken here
    hipLaunchKernelGGL((k_stencil<T, Tm, 0>), dim3(s->blk.nblk), dim3(BS), 0, stream, s->d_stencil, s->d_mptr, x,
                       (const double*)nullptr, y, s->d_off, s->n, s->n3d, BLK(s), st, mk, (double*)nullptr);
    hipLaunchKernelGGL((k_mrows<T, Tm, Tm, 4, 3>), dim3(xcd_grid(s->mblk3.nblk)), dim3(BS), 0, stream, s->d_mrows,
                       s->d_mlp, s->d_mcol, mv, x, y, MBLK3(s), st, mk, (double*)nullptr, s->mblk3.nblk, s->d_off,
                       s->n3d, s->d_m3e, (const T*)nullptr);
    return;
  }
  if (x2) launch_sweep<T, 1, 2>(s, x, y, x2, st, mk, stream);
  else launch_sweep<T, 0, 2>(s, x, y, (const T*)nullptr, st, mk, stream);
  launch_coupling_rows<T>(s, x, y, st, mk, true, stream, x2);
}

template void launch_a00<float>(mdnp_sys*, const float*, float*, const InstState*, hipStream_t, const float*);
template void launch_a00<double>(mdnp_sys*, const double*, double*, const InstState*, hipStream_t, const double*);

// The smoothed 3D solve of the neural preconditioner.  After the extension
// (which took the first relaxation step): the remaining pre-smoothing steps,
// then the network input sr = b0 - A00 z (its norm partials in part3).
template <typename T>
void launch_smooth_pre(mdnp_sys* s, T* z, const InstState* st, double* part3, hipStream_t stream) {
  const SmoothState& m = s->smooth;
  const T* sb = (const T*)m.sb;
  T* sr = (T*)m.sr;
  T* t = (T*)m.t;
  for (int k = 1; k < m.sweeps; ++k) {
    launch_a00<T>(s, z, t, st, stream);
    hipLaunchKernelGGL((k_smooth_sweep<T>), dim3(s->blk3.nblk), dim3(BS), 0, stream, z, (const T*)nullptr, sb,
                       (const T*)t, s->d_dinv32, m.omega, s->d_off, BLK3(s), st);
  }
  launch_a00<T>(s, z, t, st, stream);
  hipLaunchKernelGGL((k_smooth_res<T>), dim3(s->blk3.nblk), dim3(BS), 0, stream, sb, (const T*)t, sr, s->d_off,
                     BLK3(s), st, part3);
}
template void launch_smooth_pre<float>(mdnp_sys*, float*, const InstState*, double*, hipStream_t);
template void launch_smooth_pre<double>(mdnp_sys*, double*, const InstState*, double*, hipStream_t);

// After the network has left its correction in sr: z += sr folded into the
// first post-smoothing step (t = A00 (z + sr), z = z + sr + omega D^-1 (b0 - t)),
// then the remaining steps.
template <typename T>
void launch_smooth_post(mdnp_sys* s, T* z, const InstState* st, hipStream_t stream) {
  const SmoothState& m = s->smooth;
  const T* sb = (const T*)m.sb;
  const T* sr = (const T*)m.sr;
  T* t = (T*)m.t;
  if (s->n > SW_NMAX) {  // without the sweep: z += sr first
    hipLaunchKernelGGL((k_vec_add3d<T>), dim3(s->blk3.nblk), dim3(BS), 0, stream, z, sr, s->d_off, BLK3(s), st);
    sr = nullptr;
  }
  launch_a00<T>(s, z, t, st, stream, sr);
  hipLaunchKernelGGL((k_smooth_sweep<T>), dim3(s->blk3.nblk), dim3(BS), 0, stream, z, sr, sb, (const T*)t,
                     s->d_dinv32, m.omega, s->d_off, BLK3(s), st);
  for (int k = 1; k < m.sweeps; ++k) {
    launch_a00<T>(s, z, t, st, stream);
    hipLaunchKernelGGL((k_smooth_sweep<T>), dim3(s->blk3.nblk), dim3(BS), 0, stream, z, (const T*)nullptr, sb,
                       (const T*)t, s->d_dinv32, m.omega, s->d_off, BLK3(s), st);
  }
}
template void launch_smooth_post<float>(mdnp_sys*, float*, const InstState*, hipStream_t);
template void launch_smooth_post<double>(mdnp_sys*, double*, const InstState*, hipStream_t);

// The inner FGMRES 3D solve (Section 6) after the extension left b0 in z and
// launch_inv_scale its norm: K steps, each a network application with unit
// scaling (the basis vectors are unit vectors), an A00 application and
// Gram-Schmidt against the previous basis vectors (partials in pA / pB / pW),
// then the small least-squares problem and z0 = sum_j y_j IZ[j].
template <typename T>
void launch_inner_fgmres(mdnp_sys* s, T* z, const InstState* st, double* pA, double* pB, double* pW,
                         hipStream_t stream) {
  InnerState& q = s->inner;
  const int K = q.steps;
  const int64_t ld = s->ntot;
  T* IV = (T*)q.IV;
  T* IZ = (T*)q.IZ;
  hipLaunchKernelGGL((k_inner_start<T>), dim3(s->blk3.nblk), dim3(BS), 0, stream, (const T*)z, IV, s->cnn.inv_s,
                     s->d_off, BLK3(s), st);
  for (int j = 0; j < K; ++j) {
    T* vj = IV + (int64_t)j * ld;
    T* zj = IZ + (int64_t)j * ld;
    hipLaunchKernelGGL((k_copy3d<T>), dim3(s->blk3.nblk), dim3(BS), 0, stream, (const T*)vj, zj, s->d_off, BLK3(s),
                       st);
    cnn_apply_in_solver<T>(s, vj, zj, st, stream, q.ones);
    launch_a00<T>(s, zj, IV + (int64_t)(j + 1) * ld, st, stream);
    const int np = mgs_passes(j);
    for (int g = 0; g < np; ++g) {
      double* cur = (g % 2 == 0) ? pA : pB;
      double* prev = (g % 2 == 0) ? pB : pA;
      launch_mgs<T>(s, IV, j, g, prev, cur, pW, q.IH, K, st, stream);
    }
    const double* last = ((np - 1) % 2 == 0) ? pA : pB;
    hipLaunchKernelGGL((k_inner_finish<T>), dim3(s->blk.nblk), dim3(BS), 0, stream, IV + (int64_t)(j + 1) * ld, last,
                       (const double*)pW, q.IH, q.IH0, j, K, j + 1 < K ? 1 : 0, BLK(s), s->blk.first, st);
  }
  hipLaunchKernelGGL(k_inner_lsq, dim3((s->n_inst + 63) / 64), dim3(64), 0, stream, (const double*)q.IH,
                     (const double*)q.IH0, (const double*)s->cnn.inv_s, q.y, q.jend, K, s->n_inst, st);
  hipLaunchKernelGGL((k_inner_combine<T>), dim3(s->blk3.nblk), dim3(BS), 0, stream, z, (const T*)IZ, ld,
                     (const double*)q.y, (const int*)q.jend, K, s->d_off, BLK3(s), st);
}
template void launch_inner_fgmres<float>(mdnp_sys*, float*, const InstState*, double*, double*, double*, hipStream_t);
template void launch_inner_fgmres<double>(mdnp_sys*, double*, const InstState*, double*, double*, double*,
                                          hipStream_t);

void launch_spmv_a00_slots(mdnp_sys* s, const int32_t* inst, int n_slots, const float* x, float* y,
                           hipStream_t stream) {
  dim3 grid((s->n3d + BS - 1) / BS, n_slots);
  hipLaunchKernelGGL((k_apply_a00<float, float>), grid, dim3(BS), 0, stream, s->d_stencil, s->d_mptr, s->d_mcol,
                     s->d_mval32, s->d_off, s->d_ma01, inst, s->n, s->n3d, x, y);
}

template <typename T>
void launch_spmv_a00_all(mdnp_sys* s, const T* x, T* y, hipStream_t stream) {
  dim3 grid((s->n3d + BS - 1) / BS, s->n_inst);
  if (sizeof(T) == 8)
    hipLaunchKernelGGL((k_apply_a00<T, double>), grid, dim3(BS), 0, stream, s->d_stencil, s->d_mptr, s->d_mcol,
                       s->d_mval64, s->d_off, s->d_ma01, (const int32_t*)nullptr, s->n, s->n3d, x, y);
  else
    hipLaunchKernelGGL((k_apply_a00<T, float>), grid, dim3(BS), 0, stream, s->d_stencil, s->d_mptr, s->d_mcol,
                       s->d_mval32, s->d_off, s->d_ma01, (const int32_t*)nullptr, s->n, s->n3d, x, y);
}
template void launch_spmv_a00_all<float>(mdnp_sys*, const float*, float*, hipStream_t);
template void launch_spmv_a00_all<double>(mdnp_sys*, const double*, double*, hipStream_t);

void launch_residual(mdnp_sys* s, const double* b, const double* x, double* r, double* part, double* partm,
                     const InstState* st, hipStream_t stream) {
  const int mk = st ? 2 : 0;
  if (s->n <= SW_NMAX) {
    // the FP64 operator in its split form (stencil sweep, factored coupling)
    // over every instance, then r = b - A x and its squares
    launch_spmv<double>(s, x, r, nullptr, false, stream);
    hipLaunchKernelGGL(k_residual_part, dim3(s->blk.nblk), dim3(BS), 0, stream, b, r, BLK(s), st, mk, part, partm,
                       s->mblk.nblk);
    return;
  }
  hipLaunchKernelGGL((k_stencil<double, double, 1>), dim3(s->blk.nblk), dim3(BS), 0, stream, s->d_stencil, s->d_mptr,
                     x, b, r, s->d_off, s->n, s->n3d, BLK(s), st, mk, part);
  hipLaunchKernelGGL((k_mrows<double, double, double, 8, 1>), dim3(xcd_grid(s->mblk.nblk)), dim3(BS), 0, stream, s->d_mrows,
                     s->d_mlp, s->d_mcol, s->d_mval64, x, r, MBLK(s), st, mk, partm, s->mblk.nblk);
}

void launch_norm2_partials(mdnp_sys* s, const double* x, double* part, hipStream_t stream) {
  hipLaunchKernelGGL(k_norm2_part, dim3(s->blk.nblk), dim3(BS), 0, stream, x, s->blk.start, s->blk.end, part);
}

void launch_init_state(mdnp_sys* s, InstState* st, const double* part, const double* partx, double tol,
                       int max_iters, hipStream_t stream) {
  hipLaunchKernelGGL(k_init_state, dim3(s->n_inst), dim3(64), 0, stream, st, part, partx, s->blk.first,
                     s->n_inst, tol, max_iters);
}

void launch_cycle_start(mdnp_sys* s, InstState* st, const double* part, const double* partm, double* g, double* hist,
                        int hist_cap, int m, hipStream_t stream) {
  hipLaunchKernelGGL(k_cycle_start, dim3(s->n_inst), dim3(64), 0, stream, st, part, s->blk.first, partm,
                     s->mblk.first, s->n_inst, g, hist, hist_cap, m);
}

template <typename T>
void launch_scale_to(mdnp_sys* s, const double* r, T* v0, const InstState* st, hipStream_t stream) {
  hipLaunchKernelGGL((k_scale_to<T>), dim3(s->blk.nblk), dim3(BS), 0, stream, r, v0, BLK(s), st);
}
template void launch_scale_to<float>(mdnp_sys*, const double*, float*, const InstState*, hipStream_t);
template void launch_scale_to<double>(mdnp_sys*, const double*, double*, const InstState*, hipStream_t);

template <typename T>
void launch_prec_copy(mdnp_sys* s, const T* v, T* z, const InstState* st, hipStream_t stream) {
  hipLaunchKernelGGL((k_prec_copy<T>), dim3(s->blk.nblk), dim3(BS), 0, stream, v, z, BLK(s), st);
}
template void launch_prec_copy<float>(mdnp_sys*, const float*, float*, const InstState*, hipStream_t);
template void launch_prec_copy<double>(mdnp_sys*, const double*, double*, const InstState*, hipStream_t);

template <typename T>
void launch_prec_jacobi(mdnp_sys* s, const T* v, T* z, const InstState* st, int want_mode, hipStream_t stream) {
  hipLaunchKernelGGL((k_prec_jacobi<T>), dim3(s->blk.nblk), dim3(BS), 0, stream, v, z, s->d_dinv, BLK(s), st,
                     want_mode);
}
template void launch_prec_jacobi<float>(mdnp_sys*, const float*, float*, const InstState*, int, hipStream_t);
template void launch_prec_jacobi<double>(mdnp_sys*, const double*, double*, const InstState*, int, hipStream_t);

void tree_solve_setup(size_t shm_bytes) {
  if (shm_bytes > 65536) {
    hipFuncSetAttribute((const void*)k_tree_solve<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm_bytes);
    hipFuncSetAttribute((const void*)k_tree_solve<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm_bytes);
  }
}

void chain_solve_setup(size_t shm_bytes) {
  if (shm_bytes > 65536) {
    hipFuncSetAttribute((const void*)k_chain_vertex<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm_bytes);
    hipFuncSetAttribute((const void*)k_chain_vertex<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm_bytes);
  }
}

template <typename T>
void launch_tree_solve(mdnp_sys* s, const T* v, T* z, const InstState* st, int want_mode, hipStream_t stream) {
  const auto& cd = s->chain;
  if (cd.enabled) {
    const ChainArgs a{cd.meta, cd.soff, cd.fmul, cd.eup, cd.pinv, cd.gp, cd.gq, cd.ap, cd.aq, cd.sp, cd.sq,
                      cd.vparent, cd.vseg, cd.vchild_ptr, cd.vchild_idx, cd.vlvl_ptr, cd.vlvl_nodes, cd.vlval,
                      cd.vdinv, cd.t01, cd.zv};
    const dim3 sgrid((unsigned)((cd.max_s + 63) / 64), (unsigned)s->n_inst);
    const bool m16 = cd.max_m <= 16;
    if (m16) hipLaunchKernelGGL((k_chain_fwd<T, 16>), sgrid, dim3(64), 0, stream, v, s->d_off, s->n3d, a, st, want_mode);
    else hipLaunchKernelGGL((k_chain_fwd<T, kChainMaxM>), sgrid, dim3(64), 0, stream, v, s->d_off, s->n3d, a, st,
                            want_mode);
    const int threads = std::min(512, std::max(64, (cd.max_v + 63) / 64 * 64));
    hipLaunchKernelGGL((k_chain_vertex<T>), dim3(s->n_inst), dim3(threads), cd.lds_bytes, stream, v, z, s->d_off,
                       s->n3d, a, st, want_mode);
    if (m16) hipLaunchKernelGGL((k_chain_back<T, 16>), sgrid, dim3(64), 0, stream, v, z, s->d_off, s->n3d, a, st,
                                want_mode);
    else hipLaunchKernelGGL((k_chain_back<T, kChainMaxM>), sgrid, dim3(64), 0, stream, v, z, s->d_off, s->n3d, a, st,
                            want_mode);
    return;
  }
  const size_t shm = sizeof(double) * (size_t)s->max_n1d;
  hipLaunchKernelGGL((k_tree_solve<T>), dim3(s->n_inst), dim3(BS), shm, stream, v, z, s->d_off, s->n3d,
                     s->d_t_off, s->d_t_lvloff, s->d_t_lvlptr, s->d_t_lvlnodes, s->d_t_parent, s->d_t_childptr,
                     s->d_t_childidx, s->d_t_lval, s->d_t_dinv, st, want_mode);
}
template void launch_tree_solve<float>(mdnp_sys*, const float*, float*, const InstState*, int, hipStream_t);
template void launch_tree_solve<double>(mdnp_sys*, const double*, double*, const InstState*, int, hipStream_t);

template <typename T>
void launch_extension(mdnp_sys* s, const T* v, T* z, double* part3, double* part3m, const InstState* st,
                      int want_mode, hipStream_t stream, bool smooth_first) {
  const int nb = s->blk3.nblk + s->mblk3.nblk;
  T* sb = smooth_first ? (T*)s->smooth.sb : nullptr;
  const double om = s->smooth.omega;
  if (sizeof(T) == 8)
    hipLaunchKernelGGL((k_ext<T, double, 4>), dim3(nb), dim3(BS), 0, stream, v, z, s->d_mfree, s->d_off, BLK3(s),
                       s->blk3.nblk, s->d_mrows, s->d_a01p, s->d_a01c, s->d_a01v64, MBLK3(s), st, want_mode, part3,
                       part3m, sb, s->d_dinv32, om);
  else
    hipLaunchKernelGGL((k_ext<T, float, 4>), dim3(nb), dim3(BS), 0, stream, v, z, s->d_mfree, s->d_off, BLK3(s),
                       s->blk3.nblk, s->d_mrows, s->d_a01p, s->d_a01c, s->d_a01v32, MBLK3(s), st, want_mode, part3,
                       part3m, sb, s->d_dinv32, om);
}
template void launch_extension<float>(mdnp_sys*, const float*, float*, double*, double*, const InstState*, int,
                                      hipStream_t, bool);
template void launch_extension<double>(mdnp_sys*, const double*, double*, double*, double*, const InstState*, int,
                                       hipStream_t, bool);

template <typename T>
void launch_block_jacobi3d(mdnp_sys* s, T* z, const InstState* st, int want_mode, hipStream_t stream) {
  hipLaunchKernelGGL((k_block_jacobi3d<T>), dim3(s->blk3.nblk), dim3(BS), 0, stream, z, s->d_dinv, s->d_off,
                     BLK3(s), st, want_mode);
}
template void launch_block_jacobi3d<float>(mdnp_sys*, float*, const InstState*, int, hipStream_t);
template void launch_block_jacobi3d<double>(mdnp_sys*, double*, const InstState*, int, hipStream_t);

void launch_inv_scale(mdnp_sys* s, const double* part3, const double* part3m, double* inv_s, InstState* st,
                      int want_mode, hipStream_t stream) {
  hipLaunchKernelGGL(k_inv_scale, dim3(s->n_inst), dim3(64), 0, stream, part3, s->blk3.first, part3m,
                     s->mblk3.first, s->n_inst, inv_s, st, want_mode);
}

template <typename T, int NPD, int NCU>
void launch_mgs_pass(mdnp_sys* s, T* V, int j, int p0, int c0, const double* part_prev, double* part_cur,
                     double* part_w0, double* H, int m, const InstState* st, hipStream_t stream) {
  hipLaunchKernelGGL((k_mgs<T, NPD, NCU>), dim3(s->blk.nblk), dim3(BS), 0, stream, V, (int64_t)s->ntot, j, p0, c0,
                     part_prev, part_cur, part_w0, H, m, BLK(s), s->blk.first, st, s->blk.nblk);
}

template <typename T>
void launch_mgs(mdnp_sys* s, T* V, int j, int g, const double* part_prev, double* part_cur, double* part_w0,
                double* H, int m, const InstState* st, hipStream_t stream) {
  static_assert(kMgsGroup == 4, "pass dispatch below is written for groups of 4");
  const int nvec = j + 1;
  const int npd = g >= 1 ? std::min(kMgsGroup, nvec - (g - 1) * kMgsGroup) : 0;
  const int ncu = std::max(0, std::min(kMgsGroup, nvec - g * kMgsGroup));
  const int p0 = (g - 1) * kMgsGroup, c0 = g * kMgsGroup;
#define MGS_PASS(A, B) launch_mgs_pass<T, A, B>(s, V, j, p0, c0, part_prev, part_cur, part_w0, H, m, st, stream)
  switch (npd * 8 + ncu) {
    case 0 * 8 + 1: MGS_PASS(0, 1); break;
    case 0 * 8 + 2: MGS_PASS(0, 2); break;
    case 0 * 8 + 3: MGS_PASS(0, 3); break;
    case 0 * 8 + 4: MGS_PASS(0, 4); break;
    case 4 * 8 + 1: MGS_PASS(4, 1); break;
    case 4 * 8 + 2: MGS_PASS(4, 2); break;
    case 4 * 8 + 3: MGS_PASS(4, 3); break;
    case 4 * 8 + 4: MGS_PASS(4, 4); break;
    case 1 * 8 + 0: MGS_PASS(1, 0); break;
    case 2 * 8 + 0: MGS_PASS(2, 0); break;
    case 3 * 8 + 0: MGS_PASS(3, 0); break;
    case 4 * 8 + 0: MGS_PASS(4, 0); break;
    default: break;  // not reached: j >= 0, 0 <= g <= mgs_passes(j) - 1
  }
#undef MGS_PASS
}
template void launch_mgs<float>(mdnp_sys*, float*, int, int, const double*, double*, double*, double*, int,
                                const InstState*, hipStream_t);
template void launch_mgs<double>(mdnp_sys*, double*, int, int, const double*, double*, double*, double*, int,
                                 const InstState*, hipStream_t);

template <typename T>
void launch_mgs_finish(mdnp_sys* s, T* V, int j, const double* part_last, const double* part_w0, double* H,
                       double* cs, double* sn, double* g, double* hist, int hist_cap, int m, InstState* st,
                       hipStream_t stream) {
  hipLaunchKernelGGL((k_mgs_finish<T>), dim3(s->blk.nblk), dim3(BS), 0, stream, V, (int64_t)s->ntot, j, part_last,
                     part_w0, H, cs, sn, g, hist, hist_cap, m, BLK(s), s->blk.first, st);
}
template void launch_mgs_finish<float>(mdnp_sys*, float*, int, const double*, const double*, double*, double*,
                                       double*, double*, double*, int, int, InstState*, hipStream_t);
template void launch_mgs_finish<double>(mdnp_sys*, double*, int, const double*, const double*, double*, double*,
                                        double*, double*, double*, int, int, InstState*, hipStream_t);

void launch_solve_y(mdnp_sys* s, const double* H, const double* g, double* y, int m, const InstState* st,
                    hipStream_t stream) {
  hipLaunchKernelGGL(k_solve_y, dim3((s->n_inst + 63) / 64), dim3(64), 0, stream, H, g, y, m, s->n_inst, st);
}

template <typename T>
void launch_update_x(mdnp_sys* s, const T* Z, const double* y, double* x, int m, const InstState* st,
                     hipStream_t stream) {
  hipLaunchKernelGGL((k_update_x<T>), dim3(s->blk.nblk), dim3(BS), 0, stream, Z, (int64_t)s->ntot, y, x, m,
                     BLK(s), st);
}
template void launch_update_x<float>(mdnp_sys*, const float*, const double*, double*, int, const InstState*,
                                     hipStream_t);
template void launch_update_x<double>(mdnp_sys*, const double*, const double*, double*, int, const InstState*,
                                      hipStream_t);

}  // namespace mdnp
