// C ABI of the library: contexts, systems (upload of assembled instances),
// preconditioner selection, the restarted FGMRES driver and the entry points of
// the individual steps of the path.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <thread>
#include <atomic>

#include "conv_common.hpp"
#include "kernels.hpp"

using namespace mdnp;

namespace {

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIPCHK(call)                                   \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) throw HipError{_e, #call};   \
  } while (0)

struct ArgError {
  mdnp_status st;
  std::string msg;
};

[[noreturn]] void fail(mdnp_status st, const std::string& msg) { throw ArgError{st, msg}; }

template <typename F>
mdnp_status guarded(mdnp_ctx* ctx, F&& f) {
  try {
    f();
    if (ctx) ctx->err.clear();
    return MDNP_OK;
  } catch (const ArgError& a) {
    if (ctx) ctx->err = a.msg;
    return a.st;
  } catch (const HipError& h) {
    if (ctx) ctx->err = std::string("HIP error: ") + hipGetErrorString(h.e) + " in " + h.what;
    return h.e == hipErrorOutOfMemory ? MDNP_E_OOM : MDNP_E_HIP;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return MDNP_E_OOM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return MDNP_E_ARG;
  } catch (...) {
    if (ctx) ctx->err = "unknown error";
    return MDNP_E_ARG;
  }
}

template <typename T>
T* dalloc(size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw HipError{e, "hipMalloc"};
  return (T*)p;
}

template <typename T>
T* dupload(const std::vector<T>& v, hipStream_t s) {
  T* p = dalloc<T>(v.size());
  if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return p;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

hipStream_t pick(mdnp_ctx* ctx, void* s) { return s ? (hipStream_t)s : ctx->stream; }

void build_blocks(Blocks& B, const std::vector<int64_t>& start_i, const std::vector<int64_t>& len_i,
                  int64_t total_len, hipStream_t s, int min_chunk = 256, int64_t target_blocks = 2048) {
  const int n_inst = (int)start_i.size();
  int chunk = min_chunk;
  while (chunk < 8192 && total_len / chunk > target_blocks) chunk *= 2;
  B.chunk = chunk;
  std::vector<int32_t> bi;
  std::vector<int64_t> bs, be;
  B.h_first.assign(n_inst + 1, 0);
  for (int i = 0; i < n_inst; ++i) {
    B.h_first[i] = (int32_t)bi.size();
    for (int64_t a = 0; a < len_i[i]; a += chunk) {
      bi.push_back(i);
      bs.push_back(start_i[i] + a);
      be.push_back(start_i[i] + std::min(len_i[i], a + chunk));
    }
  }
  B.h_first[n_inst] = (int32_t)bi.size();
  B.nblk = (int)bi.size();
  B.inst = dupload(bi, s);
  B.start = dupload(bs, s);
  B.end = dupload(be, s);
  B.first = dupload(B.h_first, s);
}

void free_blocks(Blocks& B) {
  dfree(B.inst); dfree(B.start); dfree(B.end); dfree(B.first);
  B = Blocks();
}

// Captured graphs hold the launch shapes and buffers of the time they were
// taken: dropped whenever either changes.
void drop_graphs(SolveWork& w) {
  for (hipGraphExec_t g : w.graphs) (void)hipGraphExecDestroy(g);
  w.graphs.clear();
  w.graph_m = -1;
  w.graph_fb = -1;
}

void free_work(SolveWork& w) {
  dfree(w.V); dfree(w.Z); dfree(w.r); dfree(w.H); dfree(w.cs); dfree(w.sn); dfree(w.g); dfree(w.y);
  dfree(w.part); dfree(w.hist); dfree(w.st); dfree(w.xs);
  drop_graphs(w);
  if (w.h_st) (void)hipHostFree(w.h_st);
  w = SolveWork();
}

void free_smooth(SmoothState& m) {
  dfree(m.sb); dfree(m.sr); dfree(m.t);
  m = SmoothState();
}

void free_inner(InnerState& q) {
  dfree(q.IV); dfree(q.IZ); dfree(q.IH); dfree(q.IH0); dfree(q.y); dfree(q.jend); dfree(q.ones);
  q = InnerState();
}

void free_sys(mdnp_sys* s) {
  free_smooth(s->smooth);
  free_inner(s->inner);
  void* ptrs[] = {s->d_off, s->d_stencil, s->d_mptr, s->d_mfree, s->d_mcol, s->d_mval64, s->d_mval32, s->d_ma01, s->d_mrows, s->d_mlp,
                  s->d_a01p, s->d_a01c, s->d_a01v64, s->d_a01v32, s->d_m3e, s->d_gp, s->d_gsplit, s->d_gcol,
                  s->d_gval64, s->d_gval32, s->d_sp, s->d_scol, s->d_sval64, s->d_sval32, s->d_ct,
                  s->d_dinv, s->d_dinv32, s->d_dist,
                  s->d_alpha, s->d_t_off, s->d_t_lvloff, s->d_t_lvlptr, s->d_t_lvlnodes, s->d_t_parent,
                  s->d_t_childptr, s->d_t_childidx, s->d_t_lval, s->d_t_dinv};
  for (void* p : ptrs) dfree(p);
  {
    auto& c = s->chain;
    void* cp[] = {c.meta, c.soff, c.fmul, c.eup, c.pinv, c.gp, c.gq, c.ap, c.aq, c.sp, c.sq, c.vparent, c.vseg,
                  c.vchild_ptr, c.vchild_idx, c.vlvl_ptr, c.vlvl_nodes, c.vlval, c.vdinv, c.t01, c.zv};
    for (void* p : cp) dfree(p);
  }
  free_blocks(s->blk);
  free_blocks(s->blk3);
  free_blocks(s->mblk);
  free_blocks(s->mblk3);
  free_blocks(s->gblk);
  free_work(s->work);
  cnn_release(s->cnn);
  delete s;
}

size_t vsize(mdnp_dtype d) { return d == MDNP_F64 ? 8 : 4; }

// Partial-sum areas: ping-pong A/B and w0 over the whole-vector blocks, the
// 3D-part blocks, and the coupling-row blocks (all rows, 3D rows).
struct Parts {
  double *pA, *pB, *pW, *p3, *pM, *pM3;
};

// pA, pB: ping-pong partials of the Gram-Schmidt passes (kMgsVals values per
// block; the other vector reductions use their first blk.nblk entries)
size_t parts_size(const mdnp_sys* s) {
  return (2 * (size_t)kMgsVals + 1) * (size_t)s->blk.nblk + (size_t)s->blk3.nblk + (size_t)s->mblk.nblk +
         (size_t)s->mblk3.nblk;
}

Parts parts(const mdnp_sys* s, double* base) {
  Parts p;
  p.pA = base;
  p.pB = p.pA + (size_t)kMgsVals * s->blk.nblk;
  p.pW = p.pB + (size_t)kMgsVals * s->blk.nblk;
  p.p3 = p.pW + s->blk.nblk;
  p.pM = p.p3 + s->blk3.nblk;
  p.pM3 = p.pM + s->mblk.nblk;
  return p;
}

}  // namespace

// ============================================================================ context

extern "C" mdnp_status mdnp_create(mdnp_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return MDNP_E_ARG;
  *out = nullptr;
  mdnp_ctx* ctx = new (std::nothrow) mdnp_ctx();
  if (!ctx) return MDNP_E_OOM;
  mdnp_status st = guarded(ctx, [&] {
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev) fail(MDNP_E_ARG, "no such HIP device");
    HIPCHK(hipSetDevice(hip_device));
    ctx->device = hip_device;
    if (!loss_scratch_resolve(hip_device, &ctx->loss_scratch))
      fail(MDNP_E_HIP, "could not resolve the device address of the fixed loss workspace");
    if (hip_stream) {
      ctx->stream = (hipStream_t)hip_stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
      ctx->own_stream = true;
    }
  });
  if (st != MDNP_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_destroy(mdnp_ctx* ctx) {
  if (!ctx) return MDNP_E_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (mdnp_sys* s : ctx->systems) free_sys(s);
  cnn_release(ctx->cnn);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return MDNP_OK;
}

extern "C" const char* mdnp_last_error(const mdnp_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

// ============================================================================ host assembly

struct mdnp_host_sys {
  HostInstance h;
};

extern "C" mdnp_status mdnp_host_assemble(const mdnp_instance_desc* desc, mdnp_host_sys** out, char* err,
                                          int32_t err_len) {
  auto seterr = [&](const std::string& m) {
    if (err && err_len > 0) {
      std::snprintf(err, (size_t)err_len, "%s", m.c_str());
    }
  };
  if (!desc || !out) {
    seterr("null argument");
    return MDNP_E_ARG;
  }
  *out = nullptr;
  try {
    mdnp_host_sys* hs = new mdnp_host_sys();
    bool geom = false;
    std::string e = assemble_instance(*desc, hs->h, geom);
    if (!e.empty()) {
      delete hs;
      seterr(e);
      return geom ? MDNP_E_GEOM : MDNP_E_ARG;
    }
    *out = hs;
    seterr("");
    return MDNP_OK;
  } catch (const std::bad_alloc&) {
    seterr("host allocation failed");
    return MDNP_E_OOM;
  }
}

extern "C" mdnp_status mdnp_host_sizes(const mdnp_host_sys* hs, int32_t* n3d, int32_t* n1d, int64_t* nnz,
                                       int32_t* n_levels) {
  if (!hs) return MDNP_E_ARG;
  if (n3d) *n3d = hs->h.n3d;
  if (n1d) *n1d = hs->h.n1d;
  if (nnz) *nnz = (int64_t)hs->h.col.size();
  if (n_levels) *n_levels = (int32_t)hs->h.tree.lvl_ptr.size() - 1;
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_host_export(const mdnp_host_sys* hs, int32_t* row_ptr, int32_t* col, double* val,
                                        double* F, float* dist, double* alpha) {
  if (!hs) return MDNP_E_ARG;
  const HostInstance& h = hs->h;
  if (row_ptr) std::memcpy(row_ptr, h.row_ptr.data(), h.row_ptr.size() * sizeof(int32_t));
  if (col) std::memcpy(col, h.col.data(), h.col.size() * sizeof(int32_t));
  if (val) std::memcpy(val, h.val.data(), h.val.size() * sizeof(double));
  if (F) std::memcpy(F, h.F.data(), h.F.size() * sizeof(double));
  if (dist) std::memcpy(dist, h.dist.data(), h.dist.size() * sizeof(float));
  if (alpha) *alpha = h.alpha;
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_host_coupling_sizes(const mdnp_host_sys* hs, int32_t* n_gauss, int64_t* b_nnz,
                                                int64_t* r_nnz) {
  if (!hs) return MDNP_E_ARG;
  const HostInstance& h = hs->h;
  if (n_gauss) *n_gauss = (int32_t)h.b_w.size();
  if (b_nnz) *b_nnz = (int64_t)h.b_col.size();
  if (r_nnz) *r_nnz = (int64_t)h.r_col.size();
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_host_coupling(const mdnp_host_sys* hs, int32_t* b_ptr, int32_t* b_split, int32_t* b_col,
                                          double* b_val, double* w, int32_t* r_ptr, int32_t* r_col, double* r_val) {
  if (!hs) return MDNP_E_ARG;
  const HostInstance& h = hs->h;
  auto put = [](auto* dst, const auto& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  put(b_ptr, h.b_ptr);
  put(b_split, h.b_split);
  put(b_col, h.b_col);
  put(b_val, h.b_val);
  put(w, h.b_w);
  put(r_ptr, h.r_ptr);
  put(r_col, h.r_col);
  put(r_val, h.r_val);
  return MDNP_OK;
}

// Host form of the chain-compressed 1D solve (the steps of k_chain_solve).
static void host_chain_solve(const ChainFactor& C, const double* v1, double* z1) {
  const int m = C.m, S = (int)C.sp.size(), V = (int)C.vparent.size();
  std::vector<double> t0(S, 0.0), t1(S, 0.0), w(std::max(m, 1)), rv(V);
  auto seg_solve = [&](int s) {
    const double* vc = v1 + V + (size_t)s * m;
    for (int k = m - 1; k >= 0; --k) w[k] = vc[k] - (k + 1 < m ? C.fmul[(size_t)k * S + s] * w[k + 1] : 0.0);
    for (int k = 0; k < m; ++k)
      w[k] = (k == 0 ? w[0] : w[k] - C.eup[(size_t)(k - 1) * S + s] * w[k - 1]) * C.pinv[(size_t)k * S + s];
  };
  for (int s = 0; s < S && m > 0; ++s) {
    seg_solve(s);
    t0[s] = C.ap[s] * w[0];
    t1[s] = C.aq[s] * w[m - 1];
  }
  for (int u = 0; u < V; ++u) {
    double r = v1[u];
    if (C.vseg[u] >= 0) r -= t1[C.vseg[u]];
    for (int q = C.vchild_ptr[u]; q < C.vchild_ptr[u + 1]; ++q) r -= t0[C.vseg[C.vchild_idx[q]]];
    rv[u] = r;
  }
  const int nlev = (int)C.vlvl_ptr.size() - 1;
  for (int L = 0; L < nlev; ++L)
    for (int k = C.vlvl_ptr[L]; k < C.vlvl_ptr[L + 1]; ++k) {
      const int u = C.vlvl_nodes[k];
      for (int q = C.vchild_ptr[u]; q < C.vchild_ptr[u + 1]; ++q) rv[u] -= C.vlval[C.vchild_idx[q]] * rv[C.vchild_idx[q]];
    }
  for (int u = 0; u < V; ++u) rv[u] *= C.vdinv[u];
  for (int L = nlev - 1; L >= 0; --L)
    for (int k = C.vlvl_ptr[L]; k < C.vlvl_ptr[L + 1]; ++k) {
      const int u = C.vlvl_nodes[k];
      if (C.vparent[u] >= 0) rv[u] -= C.vlval[u] * rv[C.vparent[u]];
    }
  for (int u = 0; u < V; ++u) z1[u] = rv[u];
  for (int s = 0; s < S && m > 0; ++s) {
    seg_solve(s);
    for (int k = 0; k < m; ++k)
      z1[V + (size_t)s * m + k] =
          w[k] - C.gp[(size_t)k * S + s] * rv[C.sp[s]] - C.gq[(size_t)k * S + s] * rv[C.sq[s]];
  }
}

extern "C" mdnp_status mdnp_host_tree_solve(const mdnp_host_sys* hs, const double* v1, double* z1) {
  if (!hs || !v1 || !z1) return MDNP_E_ARG;
  if (hs->h.chain.m <= kChainMaxM) {
    host_chain_solve(hs->h.chain, v1, z1);
    return MDNP_OK;
  }
  const TreeFactor& T = hs->h.tree;
  const int n1d = hs->h.n1d;
  std::vector<double> y(v1, v1 + n1d);
  const int nlev = (int)T.lvl_ptr.size() - 1;
  for (int L = 0; L < nlev; ++L)
    for (int k = T.lvl_ptr[L]; k < T.lvl_ptr[L + 1]; ++k) {
      const int c = T.lvl_nodes[k];
      for (int q = T.child_ptr[c]; q < T.child_ptr[c + 1]; ++q) y[c] -= T.lval[T.child_idx[q]] * y[T.child_idx[q]];
    }
  for (int c = 0; c < n1d; ++c) y[c] *= T.dinv[c];
  for (int L = nlev - 1; L >= 0; --L)
    for (int k = T.lvl_ptr[L]; k < T.lvl_ptr[L + 1]; ++k) {
      const int c = T.lvl_nodes[k];
      if (T.parent[c] >= 0) y[c] -= T.lval[c] * y[T.parent[c]];
    }
  std::memcpy(z1, y.data(), sizeof(double) * n1d);
  return MDNP_OK;
}

extern "C" void mdnp_host_free(mdnp_host_sys* hs) { delete hs; }

// ============================================================================ upload

extern "C" mdnp_status mdnp_upload(mdnp_ctx* ctx, const mdnp_instance_desc* descs, int32_t n_inst,
                                   mdnp_dtype vec_dtype, mdnp_sys** out) {
  if (!ctx) return MDNP_E_ARG;
  mdnp_sys* s = nullptr;
  mdnp_status st = guarded(ctx, [&] {
    if (!descs || !out || n_inst < 1) fail(MDNP_E_ARG, "mdnp_upload: null argument or n_inst < 1");
    if (vec_dtype != MDNP_F64 && vec_dtype != MDNP_F32) fail(MDNP_E_ARG, "vec_dtype must be MDNP_F64 or MDNP_F32");
    for (int i = 1; i < n_inst; ++i) {
      if (descs[i].n_cells != descs[0].n_cells) fail(MDNP_E_ARG, "all instances of a system must share n_cells");
      if (descs[i].boundary != descs[0].boundary)
        fail(MDNP_E_ARG, "all instances of a system must share the boundary condition");
    }
    HIPCHK(hipSetDevice(ctx->device));
    s = new mdnp_sys();
    s->ctx = ctx;
    s->n_inst = n_inst;
    s->vec_dtype = vec_dtype;
    s->host.resize(n_inst);
    // assemble on the host in parallel
    std::vector<std::string> errs(n_inst);
    std::vector<char> geoms(n_inst, 0);
    int nth = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
    nth = std::min(nth, n_inst);
    std::vector<std::thread> pool;
    std::atomic<int> next{0};
    for (int t = 0; t < nth; ++t)
      pool.emplace_back([&] {
        for (int i = next++; i < n_inst; i = next++) {
          bool g = false;
          try {
            errs[i] = assemble_instance(descs[i], s->host[i], g);
          } catch (const std::bad_alloc&) {
            errs[i] = "host allocation failed";
          }
          geoms[i] = g;
        }
      });
    for (auto& th : pool) th.join();
    for (int i = 0; i < n_inst; ++i)
      if (!errs[i].empty()) fail(geoms[i] ? MDNP_E_GEOM : MDNP_E_ARG, "instance " + std::to_string(i) + ": " + errs[i]);
    const HostInstance& h0 = s->host[0];
    s->n_cells = h0.n_cells;
    s->neumann = h0.neumann;
    s->n = h0.n;
    s->n3d = h0.n3d;
    // offsets
    s->off.assign(n_inst + 1, 0);
    s->nnz_off.assign(n_inst + 1, 0);
    for (int i = 0; i < n_inst; ++i) {
      s->off[i + 1] = s->off[i] + s->host[i].n3d + s->host[i].n1d;
      s->nnz_off[i + 1] = s->nnz_off[i] + (int64_t)s->host[i].col.size();
      s->max_n1d = std::max(s->max_n1d, s->host[i].n1d);
    }
    s->ntot = s->off[n_inst];
    s->nnz_tot = s->nnz_off[n_inst];
    if (s->ntot >= INT32_MAX || s->nnz_tot >= INT32_MAX) fail(MDNP_E_ARG, "system too large for 32-bit indices");
    if ((size_t)s->max_n1d * 8 > 160 * 1024) fail(MDNP_E_ARG, "1D block too large for the on-chip tree solve");
    hipStream_t stream = ctx->stream;
    // concatenated operator in split form (stencil + coupling CSR), global indices
    s->mnz_tot = 0;
    for (int i = 0; i < n_inst; ++i) s->mnz_tot += (int64_t)s->host[i].m_col.size();
    if (s->mnz_tot >= INT32_MAX) fail(MDNP_E_ARG, "coupling block too large for 32-bit indices");
    std::vector<int32_t> mp(s->ntot + 1), mc(s->mnz_tot), ma01((size_t)n_inst * s->n3d);
    std::vector<double> mv64(s->mnz_tot), dinv(s->ntot), alpha(n_inst), stn((size_t)n_inst * kStencilStride);
    std::vector<float> mv32(s->mnz_tot), dist((size_t)n_inst * s->n3d);
    int64_t mo = 0;
    for (int i = 0; i < n_inst; ++i) {
      const HostInstance& h = s->host[i];
      const int64_t o = s->off[i];
      const int nr = h.n3d + h.n1d;
      for (int r = 0; r <= nr; ++r) mp[o + r] = (int32_t)(mo + h.m_ptr[r]);
      for (size_t k = 0; k < h.m_col.size(); ++k) {
        mc[mo + k] = (int32_t)(o + h.m_col[k]);
        mv64[mo + k] = h.m_val[k];
        mv32[mo + k] = (float)h.m_val[k];
      }
      for (int r = 0; r < h.n3d; ++r) ma01[(size_t)i * s->n3d + r] = (int32_t)(mo + h.m_a01[r]);
      mo += (int64_t)h.m_col.size();
      for (int r = 0; r < nr; ++r) dinv[o + r] = 1.0 / h.diag[r];
      {
        // the network's distance channel is the distance field scaled to unit
        // norm, like the residual channel it is stacked with
        double nd = 0.0;
        for (int r = 0; r < h.n3d; ++r) nd += (double)h.dist[r] * (double)h.dist[r];
        const double sc = nd > 0.0 ? 1.0 / std::sqrt(nd) : 0.0;
        for (int r = 0; r < h.n3d; ++r) dist[(size_t)i * s->n3d + r] = (float)((double)h.dist[r] * sc);
      }
      alpha[i] = h.alpha;
      for (int q = 0; q < 4; ++q) stn[(size_t)i * kStencilStride + q] = h.stencil[q];
      stn[(size_t)i * kStencilStride + 4] = h.neumann ? 0.0 : 1.0;  // a boundary row of S
    }
    s->d_off = dupload(s->off, stream);
    s->d_stencil = dupload(stn, stream);
    s->d_mptr = dupload(mp, stream);
    {
      std::vector<uint8_t> mf(mp.size() - 1);
      for (size_t r = 0; r + 1 < mp.size(); ++r) mf[r] = mp[r + 1] == mp[r] ? 1 : 0;
      s->d_mfree = dupload(mf, stream);
    }
    s->d_mcol = dupload(mc, stream);
    s->d_mval64 = dupload(mv64, stream);
    s->d_mval32 = dupload(mv32, stream);
    s->d_ma01 = dupload(ma01, stream);
    s->d_dinv = dupload(dinv, stream);
    {
      std::vector<float> dinv32(dinv.begin(), dinv.end());
      s->d_dinv32 = dupload(dinv32, stream);
    }
    s->d_dist = dupload(dist, stream);
    s->d_alpha = dupload(alpha, stream);
    // coupling-row lists: 3D rows with M entries, then all 1D rows
    std::vector<int32_t> mrows;
    std::vector<int64_t> ms(n_inst), ml(n_inst), ml3(n_inst);
    for (int i = 0; i < n_inst; ++i) {
      const HostInstance& h = s->host[i];
      ms[i] = (int64_t)mrows.size();
      for (int r = 0; r < h.n3d; ++r)
        if (h.m_ptr[r + 1] > h.m_ptr[r]) mrows.push_back((int32_t)(s->off[i] + r));
      ml3[i] = (int64_t)mrows.size() - ms[i];
      for (int r = h.n3d; r < h.n3d + h.n1d; ++r) mrows.push_back((int32_t)(s->off[i] + r));
      ml[i] = (int64_t)mrows.size() - ms[i];
      s->m_rows.push_back(ml[i]);
      s->m_nnz.push_back((int64_t)h.m_col.size());
    }
    s->d_mrows = dupload(mrows, stream);
    {
      // entries of listed row q are [mlp[q], mlp[q + 1]): rows left out of the
      // list have no M entries, so consecutive listed rows are contiguous in M
      std::vector<int32_t> mlp(mrows.size() + 1);
      for (size_t q = 0; q < mrows.size(); ++q) mlp[q] = mp[mrows[q]];
      mlp[mrows.size()] = mrows.empty() ? 0 : mp[mrows.back() + 1];
      for (size_t q = 0; q < mrows.size(); ++q)
        if (mp[mrows[q] + 1] != mlp[q + 1]) fail(MDNP_E_ARG, "internal error: coupling rows are not contiguous");
      s->d_mlp = dupload(mlp, stream);
    }
    {
      // A01 (3D rows x 1D columns) as a compact CSR over the listed rows
      // (empty for the 1D rows): the extension reads only these entries
      std::vector<int32_t> ap(mrows.size() + 1, 0), ac;
      std::vector<double> av64;
      std::vector<float> av32;
      for (int i = 0; i < n_inst; ++i)
        for (int64_t q = ms[i]; q < ms[i] + ml[i]; ++q) {
          ap[q] = (int32_t)ac.size();
          if (q >= ms[i] + ml3[i]) continue;
          const int32_t row = mrows[q];
          const int64_t r = row - s->off[i];
          for (int32_t k = ma01[(size_t)i * s->n3d + r]; k < mp[row + 1]; ++k) {
            ac.push_back(mc[k]);
            av64.push_back(mv64[k]);
            av32.push_back(mv32[k]);
          }
        }
      ap[mrows.size()] = (int32_t)ac.size();
      s->d_a01p = dupload(ap, stream);
      // end of the 3D-column entries of each listed row (its A01 entries come last)
      std::vector<int32_t> m3e(mrows.size());
      for (size_t q = 0; q < mrows.size(); ++q) m3e[q] = mp[mrows[q] + 1] - (ap[q + 1] - ap[q]);
      s->d_m3e = dupload(m3e, stream);
      s->d_a01c = dupload(ac, stream);
      s->d_a01v64 = dupload(av64, stream);
      s->d_a01v32 = dupload(av32, stream);
    }
    // coupling rows: short chunks (a few rows per lane group) for latency hiding
    build_blocks(s->mblk, ms, ml, (int64_t)mrows.size(), stream, 64, 8192);
    build_blocks(s->mblk3, ms, ml3, (int64_t)mrows.size(), stream, 64, 8192);
    // M in factored form: W B by Gauss point, and over the listed rows (in
    // their order) each row's B^T entries, Gauss points ascending, then its R
    // entries
    {
      std::vector<int32_t> gp(1, 0), gsplit, gcol, sp(mrows.size() + 1, 0), scol;
      std::vector<double> gv, sv;
      std::vector<int64_t> gs(n_inst), gl(n_inst);
      int64_t nq = 0;
      for (int i = 0; i < n_inst; ++i) {
        const HostInstance& h = s->host[i];
        const int nqi = (int)h.b_w.size();
        const int nr = h.n3d + h.n1d;
        const int64_t o = s->off[i];
        if (nq + nqi >= INT32_MAX || (int64_t)gcol.size() + h.b_ptr[nqi] >= INT32_MAX)
          fail(MDNP_E_ARG, "too many coupling entries for 32-bit indices");
        gs[i] = nq;
        gl[i] = nqi;
        for (int q = 0; q < nqi; ++q) {
          gsplit.push_back(gp.back() + (h.b_split[q] - h.b_ptr[q]));
          for (int32_t e = h.b_ptr[q]; e < h.b_ptr[q + 1]; ++e) {
            gcol.push_back((int32_t)(o + h.b_col[e]));
            gv.push_back(h.b_w[q] * h.b_val[e]);
          }
          gp.push_back((int32_t)gcol.size());
        }
        std::vector<int32_t> tp((size_t)nr + 1, 0);
        for (int32_t e = 0; e < h.b_ptr[nqi]; ++e) ++tp[h.b_col[e] + 1];
        for (int r = 0; r < nr; ++r) tp[r + 1] += tp[r];
        std::vector<int32_t> tq(tp[nr]);
        std::vector<double> tv(tp[nr]);
        {
          std::vector<int32_t> fill(tp.begin(), tp.end() - 1);
          for (int q = 0; q < nqi; ++q)
            for (int32_t e = h.b_ptr[q]; e < h.b_ptr[q + 1]; ++e) {
              const int r = h.b_col[e];
              tq[fill[r]] = q;
              tv[fill[r]++] = h.b_val[e];
            }
        }
        const size_t s0 = scol.size();
        for (int64_t k = ms[i]; k < ms[i] + ml[i]; ++k) {
          const int r = (int)(mrows[k] - o);
          sp[k] = (int32_t)scol.size();
          for (int32_t e = tp[r]; e < tp[r + 1]; ++e) {
            scol.push_back((int32_t)(nq + tq[e]));
            sv.push_back(tv[e]);
          }
          for (int32_t e = h.r_ptr[r]; e < h.r_ptr[r + 1]; ++e) {
            scol.push_back(~(int32_t)(o + h.r_col[e]));
            sv.push_back(h.r_val[e]);
          }
          if (scol.size() >= (size_t)INT32_MAX) fail(MDNP_E_ARG, "too many coupling entries for 32-bit indices");
        }
        // every row with an entry of B^T or R is listed
        if ((int64_t)(scol.size() - s0) != (int64_t)tp[nr] + h.r_ptr[nr])
          fail(MDNP_E_ARG, "internal error: a row of the factored coupling is not listed");
        s->c_gauss.push_back(nqi);
        s->c_bnnz.push_back(h.b_ptr[nqi]);
        s->c_snnz.push_back((int64_t)(scol.size() - s0));
        nq += nqi;
      }
      sp[mrows.size()] = (int32_t)scol.size();
      s->d_gp = dupload(gp, stream);
      s->d_gsplit = dupload(gsplit, stream);
      s->d_gcol = dupload(gcol, stream);
      s->d_gval64 = dupload(gv, stream);
      s->d_gval32 = dupload(std::vector<float>(gv.begin(), gv.end()), stream);
      s->d_sp = dupload(sp, stream);
      s->d_scol = dupload(scol, stream);
      s->d_sval64 = dupload(sv, stream);
      s->d_sval32 = dupload(std::vector<float>(sv.begin(), sv.end()), stream);
      s->d_ct = dalloc<double>((size_t)nq);
      build_blocks(s->gblk, gs, gl, nq, stream, 64, 8192);
    }
    // tree factorisation
    std::vector<int32_t> toff(n_inst + 1, 0), lvloff(n_inst + 1, 0), lvlptr, lvlnodes, parent, childptr, childidx;
    std::vector<double> lval, tdinv;
    for (int i = 0; i < n_inst; ++i) {
      const TreeFactor& T = s->host[i].tree;
      const int n1d = s->host[i].n1d;
      toff[i + 1] = toff[i] + n1d;
      lvloff[i + 1] = lvloff[i] + (int32_t)T.lvl_ptr.size();
      lvlptr.insert(lvlptr.end(), T.lvl_ptr.begin(), T.lvl_ptr.end());
      lvlnodes.insert(lvlnodes.end(), T.lvl_nodes.begin(), T.lvl_nodes.end());
      parent.insert(parent.end(), T.parent.begin(), T.parent.end());
      const int32_t cbase = (int32_t)childidx.size();
      for (int c = 0; c <= n1d; ++c) childptr.push_back(cbase + T.child_ptr[c]);
      childidx.insert(childidx.end(), T.child_idx.begin(), T.child_idx.end());
      lval.insert(lval.end(), T.lval.begin(), T.lval.end());
      tdinv.insert(tdinv.end(), T.dinv.begin(), T.dinv.end());
    }
    s->d_t_off = dupload(toff, stream);
    s->d_t_lvloff = dupload(lvloff, stream);
    s->d_t_lvlptr = dupload(lvlptr, stream);
    s->d_t_lvlnodes = dupload(lvlnodes, stream);
    s->d_t_parent = dupload(parent, stream);
    s->d_t_childptr = dupload(childptr, stream);
    s->d_t_childidx = dupload(childidx, stream);
    s->d_t_lval = dupload(lval, stream);
    s->d_t_dinv = dupload(tdinv, stream);
    tree_solve_setup(sizeof(double) * (size_t)s->max_n1d);
    // chain-compressed tree solve
    {
      auto& cd = s->chain;
      std::vector<int32_t> meta, sp, sq, vparent, vseg, vcp, vci, vlp, vln;
      std::vector<int64_t> soff;
      std::vector<double> fmul, eup, pinv, gp, gq, ap, aq, vlval, vdinv;
      bool ok = true;
      for (int i = 0; i < n_inst; ++i) {
        const ChainFactor& C = s->host[i].chain;
        const int S = (int)C.sp.size(), V = (int)C.vparent.size();
        ok = ok && C.m <= kChainMaxM;
        cd.max_v = std::max(cd.max_v, V);
        cd.max_s = std::max(cd.max_s, S);
        cd.max_m = std::max(cd.max_m, C.m);
        const int32_t m8[8] = {C.m, S, V, (int32_t)C.vlvl_ptr.size() - 1, (int32_t)sp.size(), (int32_t)vparent.size(),
                               (int32_t)vlp.size(), (int32_t)vci.size()};
        meta.insert(meta.end(), m8, m8 + 8);
        soff.push_back((int64_t)fmul.size());
        soff.push_back((int64_t)pinv.size());
        fmul.insert(fmul.end(), C.fmul.begin(), C.fmul.end());
        eup.insert(eup.end(), C.eup.begin(), C.eup.end());
        pinv.insert(pinv.end(), C.pinv.begin(), C.pinv.end());
        gp.insert(gp.end(), C.gp.begin(), C.gp.end());
        gq.insert(gq.end(), C.gq.begin(), C.gq.end());
        ap.insert(ap.end(), C.ap.begin(), C.ap.end());
        aq.insert(aq.end(), C.aq.begin(), C.aq.end());
        sp.insert(sp.end(), C.sp.begin(), C.sp.end());
        sq.insert(sq.end(), C.sq.begin(), C.sq.end());
        vparent.insert(vparent.end(), C.vparent.begin(), C.vparent.end());
        vseg.insert(vseg.end(), C.vseg.begin(), C.vseg.end());
        vcp.insert(vcp.end(), C.vchild_ptr.begin(), C.vchild_ptr.end());
        vci.insert(vci.end(), C.vchild_idx.begin(), C.vchild_idx.end());
        vlp.insert(vlp.end(), C.vlvl_ptr.begin(), C.vlvl_ptr.end());
        vln.insert(vln.end(), C.vlvl_nodes.begin(), C.vlvl_nodes.end());
        vlval.insert(vlval.end(), C.vlval.begin(), C.vlval.end());
        vdinv.insert(vdinv.end(), C.vdinv.begin(), C.vdinv.end());
      }
      // vertex values, two coupling terms per segment and the vertex tree in LDS
      for (int i = 0; i < n_inst; ++i) {
        const ChainFactor& C = s->host[i].chain;
        cd.lds_bytes = std::max(cd.lds_bytes, chain_lds_bytes((int)C.vparent.size(), (int)C.sp.size(),
                                                             (int)C.vlvl_ptr.size() - 1));
      }
      ok = ok && cd.lds_bytes <= 160 * 1024;
      cd.enabled = ok ? 1 : 0;
      if (ok) {
        // keep every array non-empty so that each pointer is valid
        for (auto* v : {&fmul, &eup, &pinv, &gp, &gq}) if (v->empty()) v->push_back(0.0);
        if (vci.empty()) vci.push_back(0);
        cd.meta = dupload(meta, stream);
        cd.soff = dupload(soff, stream);
        cd.fmul = dupload(fmul, stream);
        cd.eup = dupload(eup, stream);
        cd.pinv = dupload(pinv, stream);
        cd.gp = dupload(gp, stream);
        cd.gq = dupload(gq, stream);
        cd.ap = dupload(ap, stream);
        cd.aq = dupload(aq, stream);
        cd.sp = dupload(sp, stream);
        cd.sq = dupload(sq, stream);
        cd.vparent = dupload(vparent, stream);
        cd.vseg = dupload(vseg, stream);
        cd.vchild_ptr = dupload(vcp, stream);
        cd.vchild_idx = dupload(vci, stream);
        cd.vlvl_ptr = dupload(vlp, stream);
        cd.vlvl_nodes = dupload(vln, stream);
        cd.vlval = dupload(vlval, stream);
        cd.vdinv = dupload(vdinv, stream);
        cd.t01 = dalloc<double>(2 * sp.size());
        cd.zv = dalloc<double>(vparent.size());
        chain_solve_setup(cd.lds_bytes);
      }
    }
    // reduction tilings
    std::vector<int64_t> st_all(n_inst), len_all(n_inst), st3(n_inst), len3(n_inst);
    for (int i = 0; i < n_inst; ++i) {
      st_all[i] = s->off[i];
      len_all[i] = s->off[i + 1] - s->off[i];
      st3[i] = 0;  // 3D blocks use local row indices
      len3[i] = s->n3d;
    }
    build_blocks(s->blk, st_all, len_all, s->ntot, stream);
    build_blocks(s->blk3, st3, len3, (int64_t)n_inst * s->n3d, stream);
    HIPCHK(hipStreamSynchronize(stream));
    // drop the host copies that are not needed any more (keep CSR, F, dist for export)
    for (auto& h : s->host) {
      std::vector<int32_t>().swap(h.a01_start);
      std::vector<int32_t>().swap(h.m_ptr);
      std::vector<int32_t>().swap(h.m_col);
      std::vector<double>().swap(h.m_val);
      std::vector<int32_t>().swap(h.m_a01);
      h.tree = TreeFactor();
      h.chain = ChainFactor();
    }
    ctx->systems.push_back(s);
    *out = s;
  });
  if (st != MDNP_OK && s) {
    auto it = std::find(ctx->systems.begin(), ctx->systems.end(), s);
    if (it == ctx->systems.end()) free_sys(s);
  }
  return st;
}

extern "C" mdnp_status mdnp_sys_free(mdnp_ctx* ctx, mdnp_sys* s) {
  if (!ctx || !s) return MDNP_E_ARG;
  auto it = std::find(ctx->systems.begin(), ctx->systems.end(), s);
  if (it == ctx->systems.end()) return MDNP_E_ARG;
  (void)hipStreamSynchronize(ctx->stream);
  ctx->systems.erase(it);
  free_sys(s);
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_sys_sizes(const mdnp_sys* s, int32_t inst, int32_t* n3d, int32_t* n1d, int64_t* nnz,
                                      int64_t* offset) {
  if (!s || inst < 0 || inst >= s->n_inst) return MDNP_E_ARG;
  if (n3d) *n3d = s->host[inst].n3d;
  if (n1d) *n1d = s->host[inst].n1d;
  if (nnz) *nnz = (int64_t)s->host[inst].col.size();
  if (offset) *offset = s->off[inst];
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_sys_split_sizes(const mdnp_sys* s, int32_t inst, int64_t* m_nnz, int64_t* m_rows) {
  if (!s || inst < 0 || inst >= s->n_inst) return MDNP_E_ARG;
  if (m_nnz) *m_nnz = s->m_nnz[inst];
  if (m_rows) *m_rows = s->m_rows[inst];
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_sys_coupling_sizes(const mdnp_sys* s, int32_t inst, int64_t* n_gauss, int64_t* b_nnz,
                                               int64_t* s_nnz) {
  if (!s || inst < 0 || inst >= s->n_inst) return MDNP_E_ARG;
  if (n_gauss) *n_gauss = s->c_gauss[inst];
  if (b_nnz) *b_nnz = s->c_bnnz[inst];
  if (s_nnz) *s_nnz = s->c_snnz[inst];
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_export_csr(const mdnp_sys* s, int32_t inst, int32_t* row_ptr, int32_t* col, double* val) {
  if (!s || inst < 0 || inst >= s->n_inst) return MDNP_E_ARG;
  const HostInstance& h = s->host[inst];
  if (row_ptr) std::memcpy(row_ptr, h.row_ptr.data(), h.row_ptr.size() * sizeof(int32_t));
  if (col) std::memcpy(col, h.col.data(), h.col.size() * sizeof(int32_t));
  if (val) std::memcpy(val, h.val.data(), h.val.size() * sizeof(double));
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_export_rhs(const mdnp_sys* s, int32_t inst, double* F, double* dist, double* alpha) {
  if (!s || inst < 0 || inst >= s->n_inst) return MDNP_E_ARG;
  const HostInstance& h = s->host[inst];
  if (F) std::memcpy(F, h.F.data(), h.F.size() * sizeof(double));
  if (dist)
    for (int r = 0; r < h.n3d; ++r) dist[r] = (double)h.dist[r];
  if (alpha) *alpha = h.alpha;
  return MDNP_OK;
}

// ============================================================================ preconditioner

extern "C" mdnp_status mdnp_set_preconditioner(mdnp_ctx* ctx, mdnp_sys* s, mdnp_prec_kind kind, const float* weights,
                                               int64_t n_weights, double alpha, mdnp_dtype cnn_dtype) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s) fail(MDNP_E_ARG, "null system");
    if (kind < MDNP_PREC_NONE || kind > MDNP_PREC_BLOCK_JACOBI) fail(MDNP_E_ARG, "unknown preconditioner kind");
    HIPCHK(hipSetDevice(ctx->device));
    s->kind = kind;
    s->alpha_override = alpha > 0.0 ? alpha : 0.0;
    s->prec_set = true;
    drop_graphs(s->work);
    if (kind != MDNP_PREC_NEURAL) return;
    s->prec_set = false;
    if (!weights) fail(MDNP_E_ARG, "neural preconditioner needs weights");
    int64_t np = 0;
    for (int l = 0; l < kNumLayers; ++l) {
      const int taps = kLayers[l].kind == KIND_PT ? 1 : 27;
      np += (int64_t)kLayers[l].cout * taps * kLayers[l].cin + kLayers[l].cout;
    }
    if (n_weights != np) fail(MDNP_E_ARG, "expected " + std::to_string(np) + " weights");
    if (cnn_dtype != MDNP_F32 && cnn_dtype != MDNP_BF16 && cnn_dtype != MDNP_FP8E4M3 &&
        cnn_dtype != MDNP_FP8E4M3_ACT)
      fail(MDNP_E_ARG, "cnn_dtype must be MDNP_F32, MDNP_BF16, MDNP_FP8E4M3 or MDNP_FP8E4M3_ACT");
    if (s->n_cells % 4 != 0 || s->n_cells < 4) fail(MDNP_E_ARG, "the network needs n_cells divisible by 4");
    for (int64_t k = 0; k < n_weights; ++k)
      if (!std::isfinite(weights[k])) fail(MDNP_E_NONFINITE, "non-finite network weight");
    CnnState& c = s->cnn;
    if (!c.w_own) c.w_own = dalloc<float>((size_t)np);
    HIPCHK(hipMemcpyAsync(c.w_own, weights, sizeof(float) * np, hipMemcpyHostToDevice, ctx->stream));
    c.w = c.w_own;
    // FP8: the weights become E4M3 codes x per-channel powers of two, exact in
    // BF16; MDNP_FP8E4M3 runs the network with them on the BF16 kernels,
    // MDNP_FP8E4M3_ACT on the FP8 kernels with E4M3 activations
    c.fp8_weights = cnn_dtype == MDNP_FP8E4M3 || cnn_dtype == MDNP_FP8E4M3_ACT;
    if (c.fp8_weights) cnn_quantize_e4m3(c.w_own, ctx->stream);
    if (cnn_dtype == MDNP_FP8E4M3) cnn_dtype = MDNP_BF16;
    c.dtype = cnn_dtype;
    if (!c.inv_s) c.inv_s = dalloc<double>(2 * (size_t)s->n_inst);
    cnn_prepare_weights(c, c.w, ctx->stream);
    if (cnn_dtype == MDNP_FP8E4M3_ACT) {
      // packed E4M3 fragments; the activation scales are set by
      // mdnp_fp8_calibrate or mdnp_set_fp8_scales before the network runs
      if (!fp8_prepare_weights(c, ctx->stream)) fail(MDNP_E_OOM, "FP8 weight fragments");
      for (float& v : c.act8_scale) v = 0.0f;
    }
    if (!cnn_reserve(c, s->n_inst, s->n, cnn_dtype)) fail(MDNP_E_OOM, "network activation buffers");
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    c.ready = true;
    s->prec_set = true;
  });
}

extern "C" mdnp_status mdnp_autotune(mdnp_ctx* ctx, mdnp_sys* s, int32_t* chosen) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s) fail(MDNP_E_ARG, "null system");
    HIPCHK(hipSetDevice(ctx->device));
    drop_graphs(s->work);  // captured with the old launch shapes
    if (!spmv_autotune(s, ctx->stream)) fail(MDNP_E_OOM, "autotune: could not allocate its timing buffers");
    const bool net = s->kind == MDNP_PREC_NEURAL && s->prec_set && s->cnn.dtype == MDNP_BF16;
    if (net && !cnn_autotune(s, ctx->stream, 5))
      fail(MDNP_E_OOM, "autotune: could not allocate its timing buffers");
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (chosen) {
      for (int l = 0; l < 11; ++l) chosen[l] = s->cnn.sweep_blocks[l];
      chosen[11] = s->sweep_target;
      chosen[12] = s->cnn.tile_mb[3];
      chosen[13] = s->cnn.tile_mb[7];
      chosen[14] = s->cnn.tile_mb[1];
      chosen[15] = s->cnn.tile_mb[9];
      chosen[16] = s->cnn.tile_mb[6];
      chosen[17] = s->cnn.tile_mb[8];
      const int xl[5] = {0, 1, 3, 7, 9};
      for (int k = 0; k < 5; ++k) chosen[18 + k] = s->cnn.tile_xb[xl[k]];
    }
  });
}

extern "C" mdnp_status mdnp_set_tuning(mdnp_ctx* ctx, mdnp_sys* s, const int32_t* chosen) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !chosen) fail(MDNP_E_ARG, "null argument");
    for (int k = 0; k < 23; ++k)
      if (chosen[k] < 0) fail(MDNP_E_ARG, "launch-shape codes are >= 0");
    HIPCHK(hipSetDevice(ctx->device));
    drop_graphs(s->work);  // captured with the old launch shapes
    for (int l = 0; l < 11; ++l) s->cnn.sweep_blocks[l] = chosen[l];
    s->sweep_target = chosen[11];
    s->cnn.tile_mb[3] = chosen[12];
    s->cnn.tile_mb[7] = chosen[13];
    s->cnn.tile_mb[1] = chosen[14];
    s->cnn.tile_mb[9] = chosen[15];
    s->cnn.tile_mb[6] = chosen[16];
    s->cnn.tile_mb[8] = chosen[17];
    const int xl[5] = {0, 1, 3, 7, 9};
    for (int k = 0; k < 5; ++k) s->cnn.tile_xb[xl[k]] = chosen[18 + k];
  });
}

extern "C" mdnp_status mdnp_cnn_layer_times(mdnp_ctx* ctx, mdnp_sys* s, int32_t reps, float* ms) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !ms) fail(MDNP_E_ARG, "null argument");
    if (reps < 1) fail(MDNP_E_ARG, "reps must be >= 1");
    if (s->kind != MDNP_PREC_NEURAL || !s->prec_set) fail(MDNP_E_STATE, "no neural preconditioner set");
    HIPCHK(hipSetDevice(ctx->device));
    if (!cnn_layer_times(s, ctx->stream, reps, ms)) fail(MDNP_E_OOM, "layer timing: buffers or events");
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

extern "C" mdnp_status mdnp_set_inner_steps(mdnp_ctx* ctx, mdnp_sys* s, int32_t steps) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s) fail(MDNP_E_ARG, "null system");
    if (steps < 0 || steps > 8) fail(MDNP_E_ARG, "steps must be in [0, 8]");
    if (steps > 0 && s->smooth.sweeps > 0) fail(MDNP_E_STATE, "switch the smoothing off first");
    if (steps > 0 && s->neumann) fail(MDNP_E_STATE, "inner FGMRES steps are built for the Dirichlet condition only");
    HIPCHK(hipSetDevice(ctx->device));
    drop_graphs(s->work);
    free_inner(s->inner);
    if (steps == 0) return;
    InnerState& q = s->inner;
    const size_t vb = vsize(s->vec_dtype) * (size_t)s->ntot;
    const size_t ni = (size_t)s->n_inst;
    q.IV = dalloc<char>(vb * (steps + 1));
    q.IZ = dalloc<char>(vb * steps);
    q.IH = dalloc<double>(ni * (steps + 1) * steps);
    q.IH0 = dalloc<double>(ni * steps);
    q.y = dalloc<double>(ni * steps);
    q.jend = dalloc<int>(ni);
    // 1D parts of the basis and directions stay zero; the Hessenberg rows
    // below the diagonal band are never written
    HIPCHK(hipMemsetAsync(q.IV, 0, vb * (steps + 1), ctx->stream));
    HIPCHK(hipMemsetAsync(q.IZ, 0, vb * steps, ctx->stream));
    HIPCHK(hipMemsetAsync(q.IH, 0, sizeof(double) * ni * (steps + 1) * steps, ctx->stream));
    std::vector<double> ones(2 * ni, 1.0);
    q.ones = dupload(ones, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    q.steps = steps;
  });
}

extern "C" mdnp_status mdnp_set_smoothing(mdnp_ctx* ctx, mdnp_sys* s, int32_t sweeps, double omega) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s) fail(MDNP_E_ARG, "null system");
    if (sweeps < 0 || sweeps > 16) fail(MDNP_E_ARG, "sweeps must be in [0, 16]");
    if (sweeps > 0 && !(omega > 0.0 && omega < 2.0)) fail(MDNP_E_ARG, "omega must be in (0, 2)");
    if (sweeps > 0 && s->inner.steps > 0) fail(MDNP_E_STATE, "switch the inner FGMRES steps off first");
    if (sweeps > 0 && s->neumann) fail(MDNP_E_STATE, "smoothing is built for the Dirichlet condition only");
    HIPCHK(hipSetDevice(ctx->device));
    drop_graphs(s->work);
    SmoothState& m = s->smooth;
    if (sweeps == 0) {
      free_smooth(m);
      return;
    }
    if (!m.sb) {
      const size_t bytes = vsize(s->vec_dtype) * (size_t)s->ntot;
      m.sb = dalloc<char>(bytes);
      m.sr = dalloc<char>(bytes);
      m.t = dalloc<char>(bytes);
      // the 1D parts are never written by the smoothing kernels: keep them finite
      HIPCHK(hipMemsetAsync(m.sb, 0, bytes, ctx->stream));
      HIPCHK(hipMemsetAsync(m.sr, 0, bytes, ctx->stream));
      HIPCHK(hipMemsetAsync(m.t, 0, bytes, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    m.sweeps = sweeps;
    m.omega = omega;
  });
}

// ============================================================================ solve

namespace {

// Arnoldi steps per captured graph of a restart cycle.
constexpr int kCycleChunk = 5;

void ensure_work(mdnp_sys* s, int m, int hist_cap) {
  SolveWork& w = s->work;
  if (w.m >= m && w.hist_cap >= hist_cap && w.V) return;
  free_work(w);
  const size_t es = vsize(s->vec_dtype);
  const size_t nt = (size_t)s->ntot, ni = (size_t)s->n_inst;
  w.V = dalloc<char>(es * nt * (m + 1));
  w.Z = dalloc<char>(es * nt * m);
  w.r = dalloc<double>(nt);
  w.H = dalloc<double>(ni * (m + 1) * m);
  w.cs = dalloc<double>(ni * m);
  w.sn = dalloc<double>(ni * m);
  w.g = dalloc<double>(ni * (m + 1));
  w.y = dalloc<double>(ni * m);
  w.part = dalloc<double>(parts_size(s));
  w.hist = dalloc<double>(ni * hist_cap);
  w.st = dalloc<InstState>(ni);
  w.xs = dalloc<double>(nt);
  if (hipHostMalloc((void**)&w.h_st, sizeof(InstState) * ni, hipHostMallocDefault) != hipSuccess) {
    w.h_st = nullptr;
    fail(MDNP_E_OOM, "pinned host copy of the instance states");
  }
  w.m = m;
  w.hist_cap = hist_cap;
  if (!s->cnn.inv_s) s->cnn.inv_s = dalloc<double>(2 * ni);
}

// Preconditioner application z = Q(v) for the Arnoldi step (mode-masked).
template <typename T>
void apply_prec(mdnp_sys* s, const T* v, T* z, const InstState* st, bool any_fb, hipStream_t stream) {
  const Parts P = parts(s, s->work.part);
  switch (s->kind) {
    case MDNP_PREC_NONE:
      launch_prec_copy<T>(s, v, z, st, stream);
      break;
    case MDNP_PREC_JACOBI:
      launch_prec_jacobi<T>(s, v, z, st, -1, stream);
      any_fb = false;
      break;
    case MDNP_PREC_BLOCK_JACOBI:
    case MDNP_PREC_NEURAL:
    {
      const bool inner = s->kind == MDNP_PREC_NEURAL && s->inner.steps > 0;
      const bool smooth = s->kind == MDNP_PREC_NEURAL && !inner && s->smooth.sweeps > 0;
      launch_tree_solve<T>(s, v, z, st, 0, stream);
      launch_extension<T>(s, v, z, P.p3, P.pM3, st, 0, stream, smooth);
      if (s->kind == MDNP_PREC_BLOCK_JACOBI) {
        launch_block_jacobi3d<T>(s, z, st, 0, stream);
      } else if (inner) {
        // z0 = inner FGMRES(K) on A00 z0 = b0 with the network as preconditioner
        launch_inv_scale(s, P.p3, P.pM3, s->cnn.inv_s, const_cast<InstState*>(st), 0, stream);
        launch_inner_fgmres<T>(s, z, st, P.pA, P.pB, P.pW, stream);
      } else if (smooth) {
        // z0 = smoothed 3D solve of b0: relaxation from zero (the first step in
        // the extension), the network on the remaining residual (its correction
        // replaces that residual in sr), relaxation from the corrected z0
        T* sr = (T*)s->smooth.sr;
        launch_smooth_pre<T>(s, z, st, P.p3, stream);
        launch_inv_scale(s, P.p3, nullptr, s->cnn.inv_s, const_cast<InstState*>(st), 0, stream);
        cnn_apply_in_solver<T>(s, sr, sr, st, stream);
        launch_smooth_post<T>(s, z, st, stream);
      } else {
        launch_inv_scale(s, P.p3, P.pM3, s->cnn.inv_s, const_cast<InstState*>(st), 0, stream);
        cnn_apply_in_solver<T>(s, z, z, st, stream);
      }
    }
      break;
  }
  if (any_fb) launch_prec_jacobi<T>(s, v, z, st, 1, stream);
}

// Arnoldi steps j0 .. j1 - 1 of a restart cycle (all instances, masked).
template <typename T>
void arnoldi_steps(mdnp_sys* s, int j0, int j1, bool any_fb, hipStream_t stream) {
  SolveWork& w = s->work;
  T* V = (T*)w.V;
  T* Z = (T*)w.Z;
  const int64_t nt = s->ntot;
  const Parts P = parts(s, w.part);
  double* pA = P.pA;
  double* pB = P.pB;
  double* pW = P.pW;
  for (int j = j0; j < j1; ++j) {
    apply_prec<T>(s, V + j * nt, Z + j * nt, w.st, any_fb, stream);
    launch_spmv<T>(s, Z + j * nt, V + (j + 1) * nt, w.st, true, stream);
    const int np = mgs_passes(j);
    for (int g = 0; g < np; ++g) {
      double* cur = (g % 2 == 0) ? pA : pB;
      double* prev = (g % 2 == 0) ? pB : pA;
      launch_mgs<T>(s, V, j, g, prev, cur, pW, w.H, w.m, w.st, stream);
    }
    double* last = ((np - 1) % 2 == 0) ? pA : pB;
    launch_mgs_finish<T>(s, V, j, last, pW, w.H, w.cs, w.sn, w.g, w.hist, w.hist_cap, w.m, w.st, stream);
  }
}

// End of a restart cycle: y from the triangular system, x += Z y.  The x of
// the cycle start (finite: its true residual was) is kept in xs first, so an
// instance whose update turns non-finite can restart from it.
template <typename T>
void cycle_end(mdnp_sys* s, double* x, hipStream_t stream) {
  SolveWork& w = s->work;
  HIPCHK(hipMemcpyAsync(w.xs, x, sizeof(double) * s->ntot, hipMemcpyDeviceToDevice, stream));
  launch_solve_y(s, w.H, w.g, w.y, w.m, w.st, stream);
  launch_update_x<T>(s, (T*)w.Z, w.y, x, w.m, w.st, stream);
}

template <typename T>
void solve_impl(mdnp_ctx* ctx, mdnp_sys* s, const double* d_b, double* d_x, const mdnp_solve_opts& o,
                mdnp_inst_stats* stats, hipStream_t stream) {
  const int m0 = o.restart;
  const int mf = o.fallback_restart > 0 ? o.fallback_restart : o.restart;
  const int mmax = std::max(m0, mf);
  const bool fb_allowed = o.fallback_max_iters > 0 && s->kind != MDNP_PREC_JACOBI;
  const int total_cap = o.max_iters + (fb_allowed ? o.fallback_max_iters : 0);
  const int hist_cap = 2 * total_cap + 8;
  ensure_work(s, mmax, hist_cap);
  SolveWork& w = s->work;
  const int ni = s->n_inst;
  {
    const Parts P = parts(s, w.part);
    launch_norm2_partials(s, d_b, P.pA, stream);
    launch_norm2_partials(s, d_x, P.pB, stream);
    launch_init_state(s, w.st, P.pA, P.pB, o.tol, o.max_iters, stream);
  }
  std::vector<InstState> hs(ni);
  HIPCHK(hipMemcpyAsync(hs.data(), w.st, sizeof(InstState) * ni, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  for (int i = 0; i < ni; ++i)
    if (hs[i].bad_input) fail(MDNP_E_NONFINITE, "non-finite entry in b or x0 of instance " + std::to_string(i));
  for (int i = 0; i < ni; ++i)  // b = 0: the solution is 0
    if (hs[i].done)
      HIPCHK(hipMemsetAsync(d_x + s->off[i], 0, sizeof(double) * (s->off[i + 1] - s->off[i]), stream));
  HIPCHK(hipMemcpyAsync(w.xs, d_x, sizeof(double) * s->ntot, hipMemcpyDeviceToDevice, stream));
  std::vector<char> used_fb(ni, 0);
  int cycles = 0;
  const int max_cycles = total_cap + 4;
  while (true) {
    const Parts P = parts(s, w.part);
    launch_residual(s, d_b, d_x, w.r, P.pA, P.pM, w.st, stream);
    launch_cycle_start(s, w.st, P.pA, P.pM, w.g, w.hist, w.hist_cap, w.m, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hs.data(), w.st, sizeof(InstState) * ni, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    bool changed = false, any_active = false, any_fb = false, all_fb = true, pending = false;
    for (int i = 0; i < ni; ++i) {
      InstState& z = hs[i];
      if (z.done) continue;
      if (z.stalled == 2) {  // (the cycle-start kernel leaves such an instance inactive)
        // the last update made x non-finite: go back to the x of the previous
        // cycle start (true relative residual prev_rel) before the fallback or
        // before giving up; the instance sits this cycle out and its residual
        // is recomputed at the next cycle start
        HIPCHK(hipMemcpyAsync(d_x + s->off[i], w.xs + s->off[i], sizeof(double) * (s->off[i + 1] - s->off[i]),
                              hipMemcpyDeviceToDevice, stream));
        z.rel = z.prev_rel;
        z.active = 0;
        changed = true;
        if (z.mode == 0 && fb_allowed) {
          z.mode = 1;
          z.max_iters = o.fallback_max_iters;
          z.stalled = 0;
          used_fb[i] = 1;
          pending = true;
        } else {
          z.done = 1;
        }
        continue;
      }
      if (!z.active) continue;
      if (z.stalled) {
        if (z.mode == 0 && fb_allowed) {
          z.mode = 1;
          z.max_iters = o.fallback_max_iters;
          z.stalled = 0;
          used_fb[i] = 1;
          changed = true;
        } else if (z.stalled == 3) {  // out of steps
          z.done = 1;
          z.active = 0;
          changed = true;
          continue;
        }
      }
      any_active = true;
      if (z.mode == 1) any_fb = true; else all_fb = false;
    }
    if (changed) HIPCHK(hipMemcpyAsync(w.st, hs.data(), sizeof(InstState) * ni, hipMemcpyHostToDevice, stream));
    if ((!any_active && !pending) || ++cycles > max_cycles) break;
    if (!any_active) continue;  // only restarted instances: recompute their residuals
    const int m = all_fb ? mf : m0;
    w.last_m = m;
    launch_scale_to<T>(s, w.r, (T*)w.V, w.st, stream);
    // the cycle in chunks of kCycleChunk steps; after each chunk the host reads
    // the instance states and stops once none takes part any more (the
    // remaining steps would only launch masked kernels)
    const int nch = (m + kCycleChunk - 1) / kCycleChunk;
    if (o.use_graph && (w.graph_m != m || w.graph_fb != (int)any_fb)) {
      drop_graphs(w);
      for (int c = 0; c < nch; ++c) {
        hipGraph_t g;
        HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
        arnoldi_steps<T>(s, c * kCycleChunk, std::min(m, (c + 1) * kCycleChunk), any_fb, stream);
        HIPCHK(hipStreamEndCapture(stream, &g));
        hipGraphExec_t ge = nullptr;
        HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        HIPCHK(hipGraphDestroy(g));
        w.graphs.push_back(ge);
      }
      w.graph_m = m;
      w.graph_fb = (int)any_fb;
    }
    for (int c = 0; c < nch; ++c) {
      if (o.use_graph) HIPCHK(hipGraphLaunch(w.graphs[c], stream));
      else arnoldi_steps<T>(s, c * kCycleChunk, std::min(m, (c + 1) * kCycleChunk), any_fb, stream);
      if (c + 1 == nch) break;
      HIPCHK(hipMemcpyAsync(w.h_st, w.st, sizeof(InstState) * ni, hipMemcpyDeviceToHost, stream));
      HIPCHK(hipStreamSynchronize(stream));
      bool any = false;
      for (int i = 0; i < ni; ++i) any = any || (w.h_st[i].active && !w.h_st[i].done);
      if (!any) break;
    }
    cycle_end<T>(s, d_x, stream);
    HIPCHK(hipGetLastError());
  }
  // history and statistics
  w.h_nhist.assign(ni, 0);
  w.h_hist.assign((size_t)ni * w.hist_cap, 0.0);
  HIPCHK(hipMemcpyAsync(w.h_hist.data(), w.hist, sizeof(double) * w.h_hist.size(), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(hs.data(), w.st, sizeof(InstState) * ni, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  for (int i = 0; i < ni; ++i) {
    w.h_nhist[i] = std::min(hs[i].nhist, w.hist_cap);
    if (stats) {
      stats[i].iters = hs[i].iters;
      stats[i].fallback_iters = hs[i].fb_iters;
      stats[i].converged = hs[i].converged;
      stats[i].used_fallback = used_fb[i];
      stats[i].final_rel_res = hs[i].rel;
    }
  }
  (void)ctx;
}

// the E4M3 network needs its activation scales
void check_fp8_scales(const mdnp_sys* s) {
  if (s->kind == MDNP_PREC_NEURAL && s->cnn.dtype == MDNP_FP8E4M3_ACT && !(s->cnn.act8_scale[0] > 0.0f))
    fail(MDNP_E_STATE, "FP8 activation scales not set (mdnp_fp8_calibrate or mdnp_set_fp8_scales)");
}

void check_opts(const mdnp_solve_opts* o) {
  if (!o) fail(MDNP_E_ARG, "null options");
  if (o->restart < 1 || o->restart > 512) fail(MDNP_E_ARG, "restart must be in [1, 512]");
  if (o->fallback_restart < 0 || o->fallback_restart > 512) fail(MDNP_E_ARG, "fallback_restart must be in [0, 512]");
  if (o->max_iters < 1 || o->fallback_max_iters < 0) fail(MDNP_E_ARG, "invalid iteration caps");
  if ((int64_t)o->max_iters + o->fallback_max_iters > 100000000) fail(MDNP_E_ARG, "iteration caps too large");
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) fail(MDNP_E_ARG, "tol must be positive");
}

}  // namespace

extern "C" mdnp_status mdnp_solve_device(mdnp_ctx* ctx, mdnp_sys* s, const double* d_b, double* d_x,
                                         const mdnp_solve_opts* opts, mdnp_inst_stats* stats, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !d_b || !d_x) fail(MDNP_E_ARG, "null argument");
    check_opts(opts);
    if (!s->prec_set) fail(MDNP_E_STATE, "no preconditioner set (mdnp_set_preconditioner)");
    check_fp8_scales(s);
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t stream = pick(ctx, hip_stream);
    if (s->vec_dtype == MDNP_F64) solve_impl<double>(ctx, s, d_b, d_x, *opts, stats, stream);
    else solve_impl<float>(ctx, s, d_b, d_x, *opts, stats, stream);
  });
}

extern "C" mdnp_status mdnp_solve(mdnp_ctx* ctx, mdnp_sys* s, const double* b, double* x, const mdnp_solve_opts* opts,
                                  mdnp_inst_stats* stats) {
  if (!ctx) return MDNP_E_ARG;
  double* db = nullptr;
  double* dx = nullptr;
  mdnp_status st = guarded(ctx, [&] {
    if (!s || !b || !x) fail(MDNP_E_ARG, "null argument");
    check_opts(opts);
    for (int64_t k = 0; k < s->ntot; ++k)
      if (!std::isfinite(b[k]) || !std::isfinite(x[k])) fail(MDNP_E_NONFINITE, "non-finite entry in b or x0");
    HIPCHK(hipSetDevice(ctx->device));
    db = dalloc<double>(s->ntot);
    dx = dalloc<double>(s->ntot);
    HIPCHK(hipMemcpyAsync(db, b, sizeof(double) * s->ntot, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(dx, x, sizeof(double) * s->ntot, hipMemcpyHostToDevice, ctx->stream));
  });
  if (st != MDNP_OK) {
    dfree(db);
    dfree(dx);
    return st;
  }
  st = mdnp_solve_device(ctx, s, db, dx, opts, stats, ctx->stream);
  if (st == MDNP_OK) {
    st = guarded(ctx, [&] {
      HIPCHK(hipMemcpyAsync(x, dx, sizeof(double) * s->ntot, hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
    });
  }
  (void)hipStreamSynchronize(ctx->stream);
  dfree(db);
  dfree(dx);
  return st;
}

extern "C" mdnp_status mdnp_history(const mdnp_sys* s, int32_t inst, double* out, int32_t cap, int32_t* n_out) {
  if (!s || inst < 0 || inst >= s->n_inst) return MDNP_E_ARG;
  const SolveWork& w = s->work;
  const int n = (int)w.h_nhist.size() > inst ? w.h_nhist[inst] : 0;
  if (n_out) *n_out = n;
  if (out)
    for (int k = 0; k < std::min(n, cap); ++k) out[k] = w.h_hist[(size_t)inst * w.hist_cap + k];
  return MDNP_OK;
}

extern "C" mdnp_status mdnp_export_basis(mdnp_ctx* ctx, const mdnp_sys* s, int32_t k, void* d_out, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !d_out) fail(MDNP_E_ARG, "null argument");
    if (!s->work.V || s->work.last_m < 0) fail(MDNP_E_STATE, "no solve has run on this system");
    if (k < 0 || k > s->work.last_m)
      fail(MDNP_E_ARG, "basis index out of range (the last cycle had restart " + std::to_string(s->work.last_m) + ")");
    HIPCHK(hipSetDevice(ctx->device));
    const size_t es = vsize(s->vec_dtype);
    HIPCHK(hipMemcpyAsync(d_out, (const char*)s->work.V + es * (size_t)s->ntot * k, es * (size_t)s->ntot,
                          hipMemcpyDeviceToDevice, pick(ctx, hip_stream)));
  });
}

// ============================================================================ path steps

extern "C" mdnp_status mdnp_spmv(mdnp_ctx* ctx, mdnp_sys* s, int32_t block, const void* d_x, void* d_y,
                                 mdnp_dtype dtype, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !d_x || !d_y) fail(MDNP_E_ARG, "null argument");
    if (block != 0 && block != 1) fail(MDNP_E_ARG, "block must be 0 (A) or 1 (A00)");
    if (dtype != MDNP_F32 && dtype != MDNP_F64) fail(MDNP_E_ARG, "dtype must be MDNP_F32 or MDNP_F64");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t stream = pick(ctx, hip_stream);
    if (block == 0) {
      if (dtype == MDNP_F64) launch_spmv<double>(s, (const double*)d_x, (double*)d_y, nullptr, false, stream);
      else launch_spmv<float>(s, (const float*)d_x, (float*)d_y, nullptr, false, stream);
    } else {
      if (dtype == MDNP_F64) launch_spmv_a00_all<double>(s, (const double*)d_x, (double*)d_y, stream);
      else launch_spmv_a00_all<float>(s, (const float*)d_x, (float*)d_y, stream);
    }
    HIPCHK(hipGetLastError());
  });
}

extern "C" mdnp_status mdnp_spmv_repeat(mdnp_ctx* ctx, mdnp_sys* s, const void* d_x, void* d_y, mdnp_dtype dtype,
                                        int32_t reps, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !d_x || !d_y) fail(MDNP_E_ARG, "null argument");
    if (dtype != MDNP_F32 && dtype != MDNP_F64) fail(MDNP_E_ARG, "dtype must be MDNP_F32 or MDNP_F64");
    if (reps < 1) fail(MDNP_E_ARG, "reps must be positive");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t stream = pick(ctx, hip_stream);
    for (int k = 0; k < reps; ++k) {
      if (dtype == MDNP_F64) launch_spmv<double>(s, (const double*)d_x, (double*)d_y, nullptr, false, stream);
      else launch_spmv<float>(s, (const float*)d_x, (float*)d_y, nullptr, false, stream);
    }
    HIPCHK(hipGetLastError());
  });
}

extern "C" mdnp_status mdnp_tree_solve(mdnp_ctx* ctx, mdnp_sys* s, const void* d_v, void* d_z, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !d_v || !d_z) fail(MDNP_E_ARG, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t stream = pick(ctx, hip_stream);
    if (s->vec_dtype == MDNP_F64) launch_tree_solve<double>(s, (const double*)d_v, (double*)d_z, nullptr, 0, stream);
    else launch_tree_solve<float>(s, (const float*)d_v, (float*)d_z, nullptr, 0, stream);
    HIPCHK(hipGetLastError());
  });
}

extern "C" mdnp_status mdnp_precond_apply(mdnp_ctx* ctx, mdnp_sys* s, const void* d_v, void* d_z, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !d_v || !d_z) fail(MDNP_E_ARG, "null argument");
    if (!s->prec_set) fail(MDNP_E_STATE, "no preconditioner set");
    check_fp8_scales(s);
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t stream = pick(ctx, hip_stream);
    if (!s->work.part) s->work.part = dalloc<double>(parts_size(s));
    if (!s->cnn.inv_s) s->cnn.inv_s = dalloc<double>(2 * (size_t)s->n_inst);
    if (s->vec_dtype == MDNP_F64) apply_prec<double>(s, (const double*)d_v, (double*)d_z, nullptr, false, stream);
    else apply_prec<float>(s, (const float*)d_v, (float*)d_z, nullptr, false, stream);
    HIPCHK(hipGetLastError());
  });
}

extern "C" mdnp_status mdnp_set_fp8_scales(mdnp_ctx* ctx, mdnp_sys* s, const float* scales, int32_t count) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !scales) fail(MDNP_E_ARG, "null argument");
    if (count != 11) fail(MDNP_E_ARG, "expected 11 scales (X, L0a, L0b, L1a, L1b, L2a, L2b, U1, D1, U0, D0)");
    if (!(s->kind == MDNP_PREC_NEURAL && s->prec_set && s->cnn.dtype == MDNP_FP8E4M3_ACT))
      fail(MDNP_E_STATE, "no neural preconditioner with MDNP_FP8E4M3_ACT set");
    for (int k = 0; k < 11; ++k) {
      int e = 0;
      if (!(scales[k] > 0.0f) || !std::isfinite(scales[k]) || std::frexp(scales[k], &e) != 0.5f)
        fail(MDNP_E_ARG, "scales must be positive powers of two");
    }
    if (scales[4] != scales[7] || scales[2] != scales[9])
      fail(MDNP_E_ARG, "the stacked pairs (L1b, U1) and (L0b, U0) need one scale each");
    for (int k = 0; k < 11; ++k) s->cnn.act8_scale[k] = scales[k];
    drop_graphs(s->work);  // captured with the old scales
  });
}

extern "C" mdnp_status mdnp_get_fp8_scales(mdnp_ctx* ctx, const mdnp_sys* s, float* scales, int32_t count) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !scales) fail(MDNP_E_ARG, "null argument");
    if (count != 11) fail(MDNP_E_ARG, "expected 11 scales");
    for (int k = 0; k < 11; ++k) scales[k] = s->cnn.act8_scale[k];
  });
}

extern "C" mdnp_status mdnp_fp8_calibrate(mdnp_ctx* ctx, mdnp_sys* s, const void* d_v, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  void* z = nullptr;
  mdnp_status st = guarded(ctx, [&] {
    if (!s || !d_v) fail(MDNP_E_ARG, "null argument");
    if (!(s->kind == MDNP_PREC_NEURAL && s->prec_set && s->cnn.dtype == MDNP_FP8E4M3_ACT))
      fail(MDNP_E_STATE, "no neural preconditioner with MDNP_FP8E4M3_ACT set");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t stream = pick(ctx, hip_stream);
    CnnState& c = s->cnn;
    if (!s->work.part) s->work.part = dalloc<double>(parts_size(s));
    if (!c.inv_s) c.inv_s = dalloc<double>(2 * (size_t)s->n_inst);
    if (!c.fp8_amax) c.fp8_amax = dalloc<unsigned>(16);
    z = dalloc<char>(vsize(s->vec_dtype) * (size_t)s->ntot);
    fp8_zero_amax(c.fp8_amax, stream);
    // the preconditioner on v with the network in FP32, recording the largest
    // magnitude of its input and of every layer output
    c.fp8_calibrating = true;
    if (s->vec_dtype == MDNP_F64) apply_prec<double>(s, (const double*)d_v, (double*)z, nullptr, false, stream);
    else apply_prec<float>(s, (const float*)d_v, (float*)z, nullptr, false, stream);
    c.fp8_calibrating = false;
    unsigned bits[11];
    HIPCHK(hipMemcpyAsync(bits, c.fp8_amax, sizeof(bits), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    float amax[11];
    for (int k = 0; k < 11; ++k) std::memcpy(&amax[k], &bits[k], 4);
    for (int k = 0; k < 11; ++k)
      if (!std::isfinite(amax[k])) fail(MDNP_E_NONFINITE, "non-finite activation in the calibration run");
    fp8_scales_from_amax(amax, c.act8_scale);
    drop_graphs(s->work);
  });
  if (s) s->cnn.fp8_calibrating = false;
  dfree(z);
  return st;
}

extern "C" int64_t mdnp_cnn_saved_bytes(int32_t batch, int32_t n, mdnp_dtype dtype) {
  return cnn_saved_bytes(batch, n, dtype);
}

extern "C" mdnp_status mdnp_cnn_forward(mdnp_ctx* ctx, const float* d_w, const float* d_x, float* d_y, void* d_saved,
                                        int32_t batch, int32_t n, mdnp_dtype dtype, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!d_w || !d_x || !d_y) fail(MDNP_E_ARG, "null argument");
    if (batch < 1 || n < 5 || (n - 1) % 4 != 0) fail(MDNP_E_ARG, "need batch >= 1 and n = 1 (mod 4), n >= 5");
    if (dtype != MDNP_F32 && dtype != MDNP_BF16) fail(MDNP_E_ARG, "dtype must be MDNP_F32 or MDNP_BF16");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t stream = pick(ctx, hip_stream);
    CnnState& c = ctx->cnn;
    c.w = d_w;
    c.dtype = dtype;
    cnn_prepare_weights(c, d_w, stream);
    if (!d_saved && !cnn_reserve(c, batch, n, dtype)) fail(MDNP_E_OOM, "network activation buffers");
    cnn_forward_batch(c, d_x, d_y, d_saved, batch, n, dtype, stream);
    HIPCHK(hipGetLastError());
  });
}

extern "C" mdnp_status mdnp_cnn_backward(mdnp_ctx* ctx, const float* d_w, const void* d_saved, const float* d_dy,
                                         float* d_dx, float* d_dw, int32_t batch, int32_t n, mdnp_dtype dtype,
                                         void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!d_w || !d_saved || !d_dy || !d_dw) fail(MDNP_E_ARG, "null argument");
    if (batch < 1 || n < 5 || (n - 1) % 4 != 0) fail(MDNP_E_ARG, "need batch >= 1 and n = 1 (mod 4), n >= 5");
    if (dtype != MDNP_F32 && dtype != MDNP_BF16) fail(MDNP_E_ARG, "dtype must be MDNP_F32 or MDNP_BF16");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t stream = pick(ctx, hip_stream);
    CnnState& c = ctx->cnn;
    c.w = d_w;
    if (c.w_off.empty()) cnn_prepare_weights(c, d_w, stream);
    cnn_backward_batch(c, d_saved, d_dy, d_dx, d_dw, batch, n, dtype, stream);
    if (!c.bwd) fail(MDNP_E_OOM, "backward scratch allocation failed");
    HIPCHK(hipGetLastError());
  });
}

extern "C" mdnp_status mdnp_loss_grad(mdnp_ctx* ctx, mdnp_sys* s, const int32_t* d_inst, int32_t n_slots,
                                      const float* d_r, const float* d_u, float* d_du, double* d_loss,
                                      void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !d_inst || !d_r || !d_u || !d_du || !d_loss || n_slots < 1) fail(MDNP_E_ARG, "bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    launch_loss_grad(s, d_inst, n_slots, d_r, d_u, d_du, d_loss, pick(ctx, hip_stream));
    if (!s->cnn.loss) fail(MDNP_E_OOM, "loss scratch allocation failed");
    HIPCHK(hipGetLastError());
  });
}

extern "C" mdnp_status mdnp_loss_grad_noalloc(mdnp_ctx* ctx, mdnp_sys* s, const int32_t* d_inst, int32_t n_slots,
                                              const float* d_r, const float* d_u, float* d_du, double* d_loss,
                                              void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !d_inst || !d_r || !d_u || !d_du || !d_loss || n_slots < 1) fail(MDNP_E_ARG, "bad argument");
    const size_t need = loss_grad_scratch_bytes(s->n3d, n_slots);
    if (need > kLossScratchBytes)
      fail(MDNP_E_ARG, "n_slots x n3d too large for the fixed workspace: needs " + std::to_string(need) +
                           " bytes, the maximum is " + std::to_string(kLossScratchBytes));
    if (!ctx->loss_scratch) fail(MDNP_E_STATE, "fixed loss workspace not resolved");
    HIPCHK(hipSetDevice(ctx->device));
    launch_loss_grad_fixed(s, d_inst, n_slots, d_r, d_u, d_du, d_loss, ctx->loss_scratch, pick(ctx, hip_stream));
    HIPCHK(hipGetLastError());
  });
}

extern "C" mdnp_status mdnp_pack_input(mdnp_ctx* ctx, mdnp_sys* s, const int32_t* d_inst, int32_t n_slots,
                                       const float* d_r, float* d_x, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!s || !d_inst || !d_r || !d_x || n_slots < 1) fail(MDNP_E_ARG, "bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    launch_pack_input(s, d_inst, n_slots, d_r, d_x, pick(ctx, hip_stream));
    HIPCHK(hipGetLastError());
  });
}

extern "C" mdnp_status mdnp_adam_step(mdnp_ctx* ctx, float* d_w, const float* d_g, float* d_m, float* d_v, int64_t n,
                                      float lr, float b1, float b2, float eps, int32_t step, void* hip_stream) {
  if (!ctx) return MDNP_E_ARG;
  return guarded(ctx, [&] {
    if (!d_w || !d_g || !d_m || !d_v || n < 1 || step < 1) fail(MDNP_E_ARG, "bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    launch_adam(d_w, d_g, d_m, d_v, n, lr, b1, b2, eps, step, pick(ctx, hip_stream));
    HIPCHK(hipGetLastError());
  });
}
