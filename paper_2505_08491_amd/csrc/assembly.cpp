// Host assembly of the coupled 3D-1D block system of one instance (Section 2.1,
// eq. "mainsys"), its right-hand side, the distance field and the tree
// factorisation of the 1D block used by the exact 1D solve of eq. "twosteps".
//
//  * 3D: trilinear elements on N^3 uniform cells of the unit cube.  The
//    assembled stiffness at an interior node is the 27-point stencil
//    k h {8/3 centre, 0 faces, -1/6 edges, -1/12 corners} (tensor products of
//    the 1D P1 stiffness and mass); the reaction term adds
//    sigma h^3 {8/27, 2/27, 1/54, 1/216}.  Face entries are kept in the pattern.
//  * 1D: P1 elements on every straight segment, stiffness k_Lambda pi R^2 / l.
//  * Coupling: 2-point Gauss per 1D element; at each Gauss point the 3D field
//    is averaged over n_circle equispaced points of the circle of radius R in
//    the plane normal to the segment (T_Lambda).  With p the averaging weights
//    and Phi the two P1 values, the point adds W (p, -Phi)(p, -Phi)^T,
//    W = 2 pi R beta (l / 2).
//  * Homogeneous Dirichlet conditions on the cube boundary by symmetric
//    elimination with unit diagonal.
#include "assembly.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>

namespace mdnp {
namespace {

constexpr double kPi = 3.14159265358979323846;

struct Trip {
  int32_t row, col;
  double v;
};

inline void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Normal frame of a unit tangent: n1 = normalise(tau x e_a), a the axis of the
// smallest |tau_k| (first one on ties), n2 = tau x n1.
void wall_frame(const double tau[3], double n1[3], double n2[3]) {
  int a = 0;
  for (int k = 1; k < 3; ++k)
    if (std::fabs(tau[k]) < std::fabs(tau[a])) a = k;
  double e[3] = {0, 0, 0};
  e[a] = 1.0;
  cross3(tau, e, n1);
  double nn = std::sqrt(n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
  for (int k = 0; k < 3; ++k) n1[k] /= nn;
  cross3(tau, n1, n2);
}

}  // namespace

static std::string factor_1d(const mdnp_instance_desc& d, HostInstance& H);

std::string assemble_instance(const mdnp_instance_desc& d, HostInstance& H, bool& geom) {
  geom = false;
  if (d.n_cells < 2 || d.n_cells > 1024) return "n_cells must be in [2, 1024]";
  if (!d.vertex_xyz || !d.seg_vertices || !d.seg_radius || !d.seg_beta) return "null geometry array";
  if (d.elems_per_segment < 1 || d.elems_per_segment > 4096) return "elems_per_segment must be in [1, 4096]";
  if (d.n_circle < 3 || d.n_circle > 4096) return "n_circle must be in [3, 4096]";
  if (d.boundary != MDNP_BC_DIRICHLET && d.boundary != MDNP_BC_NEUMANN) return "boundary must be MDNP_BC_DIRICHLET or MDNP_BC_NEUMANN";
  if (d.problem != MDNP_PROBLEM_COUPLED && d.problem != MDNP_PROBLEM_BLOCK3D) return "problem must be MDNP_PROBLEM_COUPLED or MDNP_PROBLEM_BLOCK3D";
  if (!(std::isfinite(d.k_omega) && std::isfinite(d.sigma_omega) && std::isfinite(d.k_lambda) &&
        std::isfinite(d.f_lambda)) || d.k_omega < 0 || d.sigma_omega < 0 || d.k_lambda < 0)
    return "coefficients must be finite and non-negative";
  const int V = d.n_vertices, S = d.n_segments, E = d.elems_per_segment;
  geom = true;
  if (V < 2 || S != V - 1) return "the segments must form a tree: n_segments = n_vertices - 1 >= 1";
  for (int v = 0; v < V; ++v)
    for (int k = 0; k < 3; ++k) {
      double x = d.vertex_xyz[3 * v + k];
      if (!(std::isfinite(x) && x > 0.0 && x < 1.0)) return "vertex outside the open unit cube";
    }
  std::vector<int32_t> parent_seg(V, -1);
  for (int s = 0; s < S; ++s) {
    int p = d.seg_vertices[2 * s], q = d.seg_vertices[2 * s + 1];
    if (p < 0 || p >= V || q < 0 || q >= V || p == q) return "segment vertex index out of range";
    if (q == 0 || parent_seg[q] >= 0) return "every vertex except the root 0 must be the child end of exactly one segment";
    parent_seg[q] = s;
    if (!(std::isfinite(d.seg_radius[s]) && d.seg_radius[s] > 0.0)) return "segment radius must be positive";
    if (!(std::isfinite(d.seg_beta[s]) && d.seg_beta[s] >= 0.0)) return "segment permeability must be non-negative";
    double L2 = 0;
    for (int k = 0; k < 3; ++k) {
      double dd = d.vertex_xyz[3 * q + k] - d.vertex_xyz[3 * p + k];
      L2 += dd * dd;
    }
    if (!(L2 > 0.0)) return "zero-length segment";
  }
  {  // connectivity from the root
    std::vector<std::vector<int>> kids(V);
    for (int s = 0; s < S; ++s) kids[d.seg_vertices[2 * s]].push_back(d.seg_vertices[2 * s + 1]);
    std::vector<char> seen(V, 0);
    std::vector<int> st{0};
    seen[0] = 1;
    int cnt = 1;
    while (!st.empty()) {
      int v = st.back();
      st.pop_back();
      for (int c : kids[v])
        if (!seen[c]) { seen[c] = 1; ++cnt; st.push_back(c); }
    }
    if (cnt != V) return "the segments do not connect every vertex to the root";
  }
  geom = false;

  const int N = d.n_cells, n = N + 1;
  const double h = 1.0 / N;
  const int64_t n3d64 = (int64_t)n * n * n;
  const int64_t n1d64 = (int64_t)V + (int64_t)S * (E - 1);
  if (n3d64 + n1d64 >= (int64_t)1 << 31) return "system too large for 32-bit indices";
  const int n3d = (int)n3d64, n1d = (int)n1d64, nt = n3d + n1d;
  H.n_cells = N; H.n = n; H.n3d = n3d; H.n1d = n1d;

  auto is_bnd = [&](int r) -> bool {
    if (r >= n3d) return false;
    int i = r % n, j = (r / n) % n, k = r / (n * n);
    return i == 0 || j == 0 || k == 0 || i == n - 1 || j == n - 1 || k == n - 1;
  };
  // Dirichlet: boundary nodes are eliminated; Neumann: every node is free
  const bool dir = d.boundary == MDNP_BC_DIRICHLET;
  auto elim = [&](int r) -> bool { return dir && is_bnd(r); };

  // 1D mesh: vertices, then segment interiors from the parent end
  std::vector<double> pos((size_t)n1d * 3);
  std::memcpy(pos.data(), d.vertex_xyz, sizeof(double) * 3 * V);
  std::vector<int32_t> ea, eb, es;
  ea.reserve((size_t)S * E); eb.reserve((size_t)S * E); es.reserve((size_t)S * E);
  for (int s = 0; s < S; ++s) {
    int p = d.seg_vertices[2 * s], q = d.seg_vertices[2 * s + 1];
    const double* P = d.vertex_xyz + 3 * p;
    const double* Q = d.vertex_xyz + 3 * q;
    for (int t = 1; t < E; ++t) {
      double f = (double)t / E;
      for (int k = 0; k < 3; ++k) pos[3 * ((size_t)V + (size_t)s * (E - 1) + t - 1) + k] = P[k] + f * (Q[k] - P[k]);
    }
    int prev = p;
    for (int e = 0; e < E; ++e) {
      int nxt = (e == E - 1) ? q : V + s * (E - 1) + e;
      ea.push_back(prev); eb.push_back(nxt); es.push_back(s);
      prev = nxt;
    }
  }
  const int ne = (int)ea.size();

  // coupling and 1D triplets (Dirichlet rows/columns dropped)
  std::vector<Trip> trips;
  trips.reserve((size_t)ne * 2 * 500 + (size_t)ne * 4);
  H.F.assign(nt, 0.0);
  const double g2[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  const int nc = d.n_circle;
  std::vector<double> cth(nc), sth(nc);
  for (int k = 0; k < nc; ++k) {
    double th = 2.0 * kPi * k / nc;
    cth[k] = std::cos(th);
    sth[k] = std::sin(th);
  }
  std::vector<std::pair<int32_t, double>> pis;
  std::vector<int32_t> nodes;
  std::vector<double> coef;
  std::vector<Trip> k11;  // the 1D stiffness triplets again, for R
  k11.reserve((size_t)ne * 4);
  H.b_ptr.assign(1, 0);
  H.b_col.clear();
  H.b_val.clear();
  H.b_split.clear();
  H.b_w.clear();
  for (int e = 0; e < ne; ++e) {
    const double* Pa = &pos[3 * (size_t)ea[e]];
    const double* Pb = &pos[3 * (size_t)eb[e]];
    double D[3] = {Pb[0] - Pa[0], Pb[1] - Pa[1], Pb[2] - Pa[2]};
    double ell = std::sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    double tau[3] = {D[0] / ell, D[1] / ell, D[2] / ell};
    double n1[3], n2[3];
    wall_frame(tau, n1, n2);
    const int s = es[e];
    const double R = d.seg_radius[s];
    const double W = 2.0 * kPi * R * d.seg_beta[s] * ell / 2.0;
    // 1D stiffness and load
    const double kk = d.k_lambda * kPi * R * R / ell;
    const int A1 = n3d + ea[e], B1 = n3d + eb[e];
    trips.push_back({A1, A1, kk}); trips.push_back({A1, B1, -kk});
    trips.push_back({B1, A1, -kk}); trips.push_back({B1, B1, kk});
    k11.push_back({A1, A1, kk}); k11.push_back({A1, B1, -kk});
    k11.push_back({B1, A1, -kk}); k11.push_back({B1, B1, kk});
    H.F[A1] += d.f_lambda * ell / 2;
    H.F[B1] += d.f_lambda * ell / 2;
    for (int qi = 0; qi < 2; ++qi) {
      const double t = g2[qi];
      double g[3];
      for (int k = 0; k < 3; ++k) g[k] = Pa[k] + t * D[k];
      pis.clear();
      for (int k = 0; k < nc; ++k) {
        double x[3];
        int cell[3];
        double xi[3];
        for (int c = 0; c < 3; ++c) {
          x[c] = g[c] + R * (cth[k] * n1[c] + sth[k] * n2[c]);
          double fl = std::floor(x[c] / h);
          int ci = (int)fl;
          ci = std::min(std::max(ci, 0), N - 1);
          cell[c] = ci;
          xi[c] = x[c] / h - ci;
        }
        for (int l = 0; l < 8; ++l) {
          int a = l & 1, b = (l >> 1) & 1, cc = (l >> 2) & 1;
          double fx = a ? xi[0] : 1.0 - xi[0];
          double fy = b ? xi[1] : 1.0 - xi[1];
          double fz = cc ? xi[2] : 1.0 - xi[2];
          int node = (cell[0] + a) + n * (cell[1] + b) + n * n * (cell[2] + cc);
          pis.push_back({node, fx * fy * fz / nc});
        }
      }
      std::sort(pis.begin(), pis.end(),
                [](const std::pair<int32_t, double>& u, const std::pair<int32_t, double>& v) {
                  return u.first < v.first;
                });
      nodes.clear();
      coef.clear();
      for (size_t k = 0; k < pis.size();) {
        size_t k2 = k;
        double acc = 0.0;
        while (k2 < pis.size() && pis[k2].first == pis[k].first) acc += pis[k2++].second;
        nodes.push_back(pis[k].first);
        coef.push_back(acc);
        k = k2;
      }
      nodes.push_back(A1); coef.push_back(-(1.0 - t));
      nodes.push_back(B1); coef.push_back(-t);
      const int m = (int)nodes.size();
      // row q of B: the free 3D nodes (ascending), then the two 1D nodes
      for (int u = 0; u < m; ++u) {
        if (u == m - 2) H.b_split.push_back((int32_t)H.b_col.size());
        if (elim(nodes[u])) continue;
        H.b_col.push_back(nodes[u]);
        H.b_val.push_back(coef[u]);
      }
      H.b_ptr.push_back((int32_t)H.b_col.size());
      H.b_w.push_back(W);
      for (int u = 0; u < m; ++u) {
        if (elim(nodes[u])) continue;
        for (int v = 0; v < m; ++v) {
          if (elim(nodes[v])) continue;
          trips.push_back({nodes[u], nodes[v], W * (coef[u] * coef[v])});
        }
      }
    }
  }

  // bucket the triplets by row, sort each row by column, merge duplicates
  std::vector<int64_t> tptr((size_t)nt + 1, 0);
  for (const Trip& t : trips) ++tptr[t.row + 1];
  for (int r = 0; r < nt; ++r) tptr[r + 1] += tptr[r];
  std::vector<std::pair<int32_t, double>> rowt(trips.size());
  {
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (const Trip& t : trips) rowt[fill[t.row]++] = {t.col, t.v};
  }
  std::vector<Trip>().swap(trips);
  // the 1D stiffness by row (1D rows only), for R
  std::vector<int64_t> kptr((size_t)n1d + 1, 0);
  for (const Trip& t : k11) ++kptr[t.row - n3d + 1];
  for (int r = 0; r < n1d; ++r) kptr[r + 1] += kptr[r];
  std::vector<std::pair<int32_t, double>> krow(k11.size());
  {
    std::vector<int64_t> fill(kptr.begin(), kptr.end() - 1);
    for (const Trip& t : k11) krow[fill[t.row - n3d]++] = {t.col, t.v};
  }
  std::vector<Trip>().swap(k11);
  H.r_ptr.assign((size_t)nt + 1, 0);
  H.r_col.clear();
  H.r_val.clear();

  // stencil values at an interior node (sums over its 8 cells) and one cell's
  // share (node pairs differing in 0..3 coordinates; a pair shares 2^(3 - nd)
  // cells around an interior node, fewer on the boundary)
  const double kh = d.k_omega * h, sh3 = d.sigma_omega * h * h * h;
  const double kst[4] = {kh * (8.0 / 3.0), 0.0, kh * (-1.0 / 6.0), kh * (-1.0 / 12.0)};
  const double mst[4] = {sh3 * (8.0 / 27.0), sh3 * (2.0 / 27.0), sh3 * (1.0 / 54.0), sh3 * (1.0 / 216.0)};
  const double kel[4] = {kh * (1.0 / 3.0), 0.0, kh * (-1.0 / 12.0), kh * (-1.0 / 12.0)};
  const double mel[4] = {sh3 * (1.0 / 27.0), sh3 * (1.0 / 54.0), sh3 * (1.0 / 108.0), sh3 * (1.0 / 216.0)};
  H.neumann = !dir;

  H.row_ptr.assign((size_t)nt + 1, 0);
  H.col.clear();
  H.val.clear();
  H.col.reserve((size_t)n3d * 27 + rowt.size());
  H.val.reserve((size_t)n3d * 27 + rowt.size());
  H.a01_start.assign(n3d, 0);
  H.diag.assign(nt, 0.0);
  for (int q = 0; q < 4; ++q) H.stencil[q] = kst[q] + mst[q];
  H.m_ptr.assign((size_t)nt + 1, 0);
  H.m_col.clear();
  H.m_val.clear();
  H.m_a01.assign(n3d, 0);
  typedef std::vector<std::pair<int32_t, double>> RowEntries;
  // sum of two column-sorted entry lists, columns merged
  auto merge_rows = [](const RowEntries& a, const RowEntries& b, RowEntries& out) {
    out.clear();
    out.reserve(a.size() + b.size());
    size_t i = 0, j = 0;
    while (i < a.size() || j < b.size()) {
      const int32_t ca = i < a.size() ? a[i].first : INT32_MAX;
      const int32_t cb = j < b.size() ? b[j].first : INT32_MAX;
      const int32_t cmin = std::min(ca, cb);
      double acc = 0.0;
      if (ca == cmin) acc += a[i++].second;
      if (cb == cmin) acc += b[j++].second;
      out.push_back({cmin, acc});
    }
  };
  RowEntries merged, cpl, stn, corr, mrow;
  for (int r = 0; r < nt; ++r) {
    auto b0 = rowt.begin() + tptr[r], b1 = rowt.begin() + tptr[r + 1];
    std::sort(b0, b1, [](const std::pair<int32_t, double>& u, const std::pair<int32_t, double>& v) {
      return u.first < v.first;
    });
    // coupling / 1D part of the row on its own (duplicates merged)
    cpl.clear();
    for (auto it = b0; it != b1;) {
      const int32_t cc = it->first;
      double acc = 0.0;
      while (it != b1 && it->first == cc) acc += (it++)->second;
      cpl.push_back({cc, acc});
    }
    // stencil part of a 3D row (stn), and the entries of it that the device's
    // stencil kernels leave to M (corr): with the natural boundary those
    // kernels still skip boundary nodes (a boundary row yields 0, boundary
    // columns are left out), so M carries every boundary row's stencil
    // entries and the boundary columns of the rows next to the boundary
    stn.clear();
    corr.clear();
    if (r < n3d) {
      if (elim(r)) {
        stn.push_back({r, 1.0});
      } else {
        const int ix[3] = {r % n, (r / n) % n, r / (n * n)};
        const bool rb = is_bnd(r);
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int dd[3] = {dx, dy, dz};
              bool inside = true;
              for (int a = 0; a < 3; ++a) inside = inside && ix[a] + dd[a] >= 0 && ix[a] + dd[a] <= n - 1;
              if (!inside) continue;
              const int c = r + dx + n * dy + n * n * dz;
              if (elim(c)) continue;
              const int nd = (dx != 0) + (dy != 0) + (dz != 0);
              double v;
              if (!rb) {
                v = kst[nd] + mst[nd];
              } else {  // cells shared with the neighbour: 1 or 2 along each axis where it does not move
                int cells = 1;
                for (int a = 0; a < 3; ++a)
                  if (dd[a] == 0) cells *= (ix[a] > 0) + (ix[a] < n - 1);
                v = (kel[nd] + mel[nd]) * cells;
              }
              stn.push_back({c, v});
              if (rb || is_bnd(c)) corr.push_back({c, v});
            }
      }
    }
    merge_rows(cpl, corr, mrow);
    // row r of R: the natural-boundary stencil entries of a 3D row, the 1D
    // stiffness of a 1D row (duplicates merged)
    if (r < n3d) {
      for (const auto& e : corr) {
        H.r_col.push_back(e.first);
        H.r_val.push_back(e.second);
      }
    } else {
      auto k0 = krow.begin() + kptr[r - n3d], k1 = krow.begin() + kptr[r - n3d + 1];
      std::sort(k0, k1, [](const std::pair<int32_t, double>& u, const std::pair<int32_t, double>& v) {
        return u.first < v.first;
      });
      for (auto it = k0; it != k1;) {
        const int32_t cc = it->first;
        double acc = 0.0;
        while (it != k1 && it->first == cc) acc += (it++)->second;
        H.r_col.push_back(cc);
        H.r_val.push_back(acc);
      }
    }
    H.r_ptr[r + 1] = (int32_t)H.r_col.size();
    bool m01 = false;
    for (const auto& e : mrow) {
      if (r < n3d && !m01 && e.first >= n3d) {
        H.m_a01[r] = (int32_t)H.m_col.size();
        m01 = true;
      }
      H.m_col.push_back(e.first);
      H.m_val.push_back(e.second);
    }
    if (r < n3d && !m01) H.m_a01[r] = (int32_t)H.m_col.size();
    H.m_ptr[r + 1] = (int32_t)H.m_col.size();
    if (r < n3d && elim(r)) {
      merged = stn;
    } else {
      merge_rows(stn, cpl, merged);
    }
    bool found01 = false;
    for (const auto& e : merged) {
      if (r < n3d && !found01 && e.first >= n3d) {
        H.a01_start[r] = (int32_t)H.col.size();
        found01 = true;
      }
      if (e.first == r) H.diag[r] = e.second;
      H.col.push_back(e.first);
      H.val.push_back(e.second);
    }
    if (r < n3d && !found01) H.a01_start[r] = (int32_t)H.col.size();
    H.row_ptr[r + 1] = (int32_t)H.col.size();
    if (H.col.size() >= (size_t)INT32_MAX) return "too many nonzeros for 32-bit indices";
  }

  // normalisation of the network input/output: RMS of diag(A00) on free nodes
  {
    double acc = 0.0;
    int64_t cnt = 0;
    for (int r = 0; r < n3d; ++r)
      if (!elim(r)) { acc += H.diag[r] * H.diag[r]; ++cnt; }
    H.alpha = cnt ? std::sqrt(acc / cnt) : 1.0;
  }

  // distance field d(x) = min_s |x - proj_[P,Q] x|
  H.dist.assign(n3d, 0.0f);
  for (int r = 0; r < n3d; ++r) {
    const double X[3] = {(r % n) * h, ((r / n) % n) * h, (r / (n * n)) * h};
    double best = INFINITY;
    for (int s = 0; s < S; ++s) {
      const double* P = d.vertex_xyz + 3 * d.seg_vertices[2 * s];
      const double* Q = d.vertex_xyz + 3 * d.seg_vertices[2 * s + 1];
      double Dv[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
      double t = ((X[0] - P[0]) * Dv[0] + (X[1] - P[1]) * Dv[1] + (X[2] - P[2]) * Dv[2]) /
                 (Dv[0] * Dv[0] + Dv[1] * Dv[1] + Dv[2] * Dv[2]);
      t = std::min(std::max(t, 0.0), 1.0);
      double e0 = X[0] - (P[0] + t * Dv[0]), e1 = X[1] - (P[1] + t * Dv[1]), e2 = X[2] - (P[2] + t * Dv[2]);
      best = std::min(best, e0 * e0 + e1 * e1 + e2 * e2);
    }
    H.dist[r] = (float)std::sqrt(best);
  }

  std::string err = factor_1d(d, H);
  if (!err.empty() || d.problem != MDNP_PROBLEM_BLOCK3D) return err;

  // the 3D block alone: b = -A01 x with A11 x = f1 (exact tree solve in FP64),
  // then the layout [C 0; 0 I] [u0; u1] = [b; 0]
  {
    const TreeFactor& T = H.tree;
    std::vector<double> y(H.F.begin() + n3d, H.F.end());
    std::vector<int32_t> order;  // root first (BFS)
    order.reserve(n1d);
    order.push_back(0);
    for (size_t k = 0; k < order.size(); ++k)
      for (int32_t e = T.child_ptr[order[k]]; e < T.child_ptr[order[k] + 1]; ++e) order.push_back(T.child_idx[e]);
    for (int k = n1d - 1; k >= 0; --k) {  // L y = f, leaves first
      const int c = order[k];
      if (T.parent[c] >= 0) y[T.parent[c]] -= T.lval[c] * y[c];
    }
    for (int c = 0; c < n1d; ++c) y[c] *= T.dinv[c];
    for (int k = 0; k < n1d; ++k) {  // L^T x = D^-1 y, root first
      const int c = order[k];
      if (T.parent[c] >= 0) y[c] -= T.lval[c] * y[T.parent[c]];
    }
    std::vector<double> b(n3d, 0.0);
    for (int r = 0; r < n3d; ++r)
      for (int32_t e = H.a01_start[r]; e < H.row_ptr[r + 1]; ++e) b[r] -= H.val[e] * y[H.col[e] - n3d];
    // drop the A01 / A10 entries, unit 1D rows, in A and in M
    auto strip = [&](std::vector<int32_t>& ptr, std::vector<int32_t>& col, std::vector<double>& val,
                     std::vector<int32_t>* a01) {
      std::vector<int32_t> p2(ptr.size(), 0), c2;
      std::vector<double> v2;
      c2.reserve(col.size());
      v2.reserve(val.size());
      for (int r = 0; r < nt; ++r) {
        if (r < n3d) {
          for (int32_t e = ptr[r]; e < ptr[r + 1]; ++e)
            if (col[e] < n3d) { c2.push_back(col[e]); v2.push_back(val[e]); }
          if (a01) (*a01)[r] = (int32_t)c2.size();
        } else {
          c2.push_back(r);
          v2.push_back(1.0);
        }
        p2[r + 1] = (int32_t)c2.size();
      }
      ptr.swap(p2);
      col.swap(c2);
      val.swap(v2);
    };
    strip(H.row_ptr, H.col, H.val, &H.a01_start);
    strip(H.m_ptr, H.m_col, H.m_val, &H.m_a01);
    strip(H.r_ptr, H.r_col, H.r_val, nullptr);
    {  // B keeps its 3D columns only
      std::vector<int32_t> p2(1, 0), c2;
      std::vector<double> v2;
      for (size_t q = 0; q + 1 < H.b_ptr.size(); ++q) {
        for (int32_t e = H.b_ptr[q]; e < H.b_split[q]; ++e) {
          c2.push_back(H.b_col[e]);
          v2.push_back(H.b_val[e]);
        }
        p2.push_back((int32_t)c2.size());
        H.b_split[q] = p2.back();
      }
      H.b_ptr.swap(p2);
      H.b_col.swap(c2);
      H.b_val.swap(v2);
    }
    for (int r = n3d; r < nt; ++r) H.diag[r] = 1.0;
    for (int r = 0; r < n3d; ++r) H.F[r] = b[r];
    for (int r = n3d; r < nt; ++r) H.F[r] = 0.0;
    return factor_1d(d, H);
  }
}

// Factorisations of the 1D block A11 held in H's CSR (no fill): leaves-first
// LDL^T of the whole tree and the chain-compressed form.
static std::string factor_1d(const mdnp_instance_desc& d, HostInstance& H) {
  const int V = d.n_vertices, S = d.n_segments, E = d.elems_per_segment;
  const int n3d = H.n3d, n1d = H.n1d;
  // tree factorisation of A11 (1D block incl. coupling mass), leaves first
  TreeFactor& T = H.tree;
  T.parent.assign(n1d, -1);
  for (int s = 0; s < S; ++s) {
    int p = d.seg_vertices[2 * s], q = d.seg_vertices[2 * s + 1];
    int prev = p;
    for (int t = 0; t < E - 1; ++t) {
      int node = V + s * (E - 1) + t;
      T.parent[node] = prev;
      prev = node;
    }
    T.parent[q] = prev;
  }
  std::vector<std::vector<int32_t>> kids(n1d);
  for (int c = 0; c < n1d; ++c)
    if (T.parent[c] >= 0) kids[T.parent[c]].push_back(c);
  std::vector<int32_t> bfs;
  bfs.reserve(n1d);
  bfs.push_back(0);
  for (size_t k = 0; k < bfs.size(); ++k)
    for (int c : kids[bfs[k]]) bfs.push_back(c);
  if ((int)bfs.size() != n1d) return "internal error: 1D mesh is not a tree";
  auto a11 = [&](int row, int colj) -> double {
    const int r = n3d + row, c = n3d + colj;
    const int32_t* b = H.col.data() + H.row_ptr[r];
    const int32_t* e = H.col.data() + H.row_ptr[r + 1];
    const int32_t* f = std::lower_bound(b, e, c);
    return (f != e && *f == c) ? H.val[f - H.col.data()] : 0.0;
  };
  std::vector<double> piv(n1d);
  std::vector<int32_t> level(n1d, 0);
  T.lval.assign(n1d, 0.0);
  T.dinv.assign(n1d, 0.0);
  for (int k = n1d - 1; k >= 0; --k) {
    int c = bfs[k];
    double dc = a11(c, c);
    int lv = 0;
    for (int kid : kids[c]) {
      double acl = a11(c, kid);
      dc -= acl * acl / piv[kid];
      lv = std::max(lv, level[kid] + 1);
    }
    if (!(dc > 0.0)) return "1D block is not positive definite (check R, beta and k_lambda)";
    piv[c] = dc;
    level[c] = lv;
    T.dinv[c] = 1.0 / dc;
    if (T.parent[c] >= 0) T.lval[c] = a11(T.parent[c], c) / dc;
  }
  T.child_ptr.assign(n1d + 1, 0);
  for (int c = 0; c < n1d; ++c) T.child_ptr[c + 1] = T.child_ptr[c] + (int32_t)kids[c].size();
  T.child_idx.clear();
  for (int c = 0; c < n1d; ++c) for (int kid : kids[c]) T.child_idx.push_back(kid);
  int nlev = 0;
  for (int c = 0; c < n1d; ++c) nlev = std::max(nlev, level[c] + 1);
  T.lvl_ptr.assign(nlev + 1, 0);
  for (int c = 0; c < n1d; ++c) ++T.lvl_ptr[level[c] + 1];
  for (int l = 0; l < nlev; ++l) T.lvl_ptr[l + 1] += T.lvl_ptr[l];
  T.lvl_nodes.assign(n1d, 0);
  {
    std::vector<int32_t> fill(T.lvl_ptr.begin(), T.lvl_ptr.end() - 1);
    for (int c = 0; c < n1d; ++c) T.lvl_nodes[fill[level[c]]++] = c;
  }

  // chain-compressed factorisation (same matrix, elimination grouped by segment)
  ChainFactor& C = H.chain;
  const int m = E - 1;
  C.m = m;
  C.fmul.assign((size_t)std::max(m - 1, 0) * S, 0.0);
  C.eup.assign((size_t)std::max(m - 1, 0) * S, 0.0);
  C.pinv.assign((size_t)m * S, 0.0);
  C.gp.assign((size_t)m * S, 0.0);
  C.gq.assign((size_t)m * S, 0.0);
  C.ap.assign(S, 0.0);
  C.aq.assign(S, 0.0);
  C.sp.assign(S, 0);
  C.sq.assign(S, 0);
  C.vseg.assign(V, -1);
  std::vector<double> vdiag(V), voff(V, 0.0);  // Schur complement: diagonal, entry to the parent vertex
  for (int v = 0; v < V; ++v) vdiag[v] = a11(v, v);
  std::vector<double> dd(std::max(m, 1)), ee(std::max(m, 1)), piv2(std::max(m, 1)), w(std::max(m, 1));
  auto chain_solve = [&](int s, std::vector<double>& rhs) {  // rhs <- T_s^-1 rhs
    for (int i = m - 2; i >= 0; --i) rhs[i] -= C.fmul[(size_t)i * S + s] * rhs[i + 1];
    rhs[0] *= C.pinv[s];
    for (int i = 1; i < m; ++i) rhs[i] = (rhs[i] - ee[i - 1] * rhs[i - 1]) * C.pinv[(size_t)i * S + s];
  };
  for (int s = 0; s < S; ++s) {
    const int p = d.seg_vertices[2 * s], q = d.seg_vertices[2 * s + 1];
    C.sp[s] = p;
    C.sq[s] = q;
    C.vseg[q] = s;
    if (m == 0) {
      voff[q] = a11(p, q);
      continue;
    }
    const int c0 = V + s * m;
    for (int i = 0; i < m; ++i) dd[i] = a11(c0 + i, c0 + i);
    for (int i = 0; i + 1 < m; ++i) ee[i] = a11(c0 + i, c0 + i + 1);
    piv2[m - 1] = dd[m - 1];
    for (int i = m - 2; i >= 0; --i) piv2[i] = dd[i] - ee[i] * ee[i] / piv2[i + 1];
    for (int i = 0; i < m; ++i) {
      if (!(piv2[i] > 0.0)) return "1D block is not positive definite (check R, beta and k_lambda)";
      C.pinv[(size_t)i * S + s] = 1.0 / piv2[i];
    }
    for (int i = 0; i + 1 < m; ++i) {
      C.fmul[(size_t)i * S + s] = ee[i] / piv2[i + 1];
      C.eup[(size_t)i * S + s] = ee[i];
    }
    C.ap[s] = a11(p, c0);
    C.aq[s] = a11(q, c0 + m - 1);
    std::fill(w.begin(), w.end(), 0.0);
    w[0] = C.ap[s];
    chain_solve(s, w);
    for (int i = 0; i < m; ++i) C.gp[(size_t)i * S + s] = w[i];
    const double gp0 = w[0];
    std::fill(w.begin(), w.end(), 0.0);
    w[m - 1] = C.aq[s];
    chain_solve(s, w);
    for (int i = 0; i < m; ++i) C.gq[(size_t)i * S + s] = w[i];
    vdiag[p] -= C.ap[s] * gp0;
    vdiag[q] -= C.aq[s] * w[m - 1];
    voff[q] = -C.ap[s] * w[0];
  }
  // vertex tree (parent of q = p of its segment), leaves-first LDL^T by BFS from vertex 0
  C.vparent.assign(V, -1);
  for (int s = 0; s < S; ++s) C.vparent[C.sq[s]] = C.sp[s];
  std::vector<std::vector<int32_t>> vkids(V);
  for (int v = 0; v < V; ++v)
    if (C.vparent[v] >= 0) vkids[C.vparent[v]].push_back(v);
  std::vector<int32_t> vbfs;
  vbfs.reserve(V);
  vbfs.push_back(0);
  for (size_t k = 0; k < vbfs.size(); ++k)
    for (int c : vkids[vbfs[k]]) vbfs.push_back(c);
  if ((int)vbfs.size() != V) return "internal error: vertex graph is not a tree";
  std::vector<double> vpiv(V);
  std::vector<int32_t> vlevel(V, 0);
  C.vlval.assign(V, 0.0);
  C.vdinv.assign(V, 0.0);
  for (int k = V - 1; k >= 0; --k) {
    const int v = vbfs[k];
    double dv = vdiag[v];
    int lv = 0;
    for (int u : vkids[v]) {
      dv -= voff[u] * voff[u] / vpiv[u];
      lv = std::max(lv, vlevel[u] + 1);
    }
    if (!(dv > 0.0)) return "1D block is not positive definite (check R, beta and k_lambda)";
    vpiv[v] = dv;
    vlevel[v] = lv;
    C.vdinv[v] = 1.0 / dv;
    if (C.vparent[v] >= 0) C.vlval[v] = voff[v] / dv;
  }
  C.vchild_ptr.assign(V + 1, 0);
  for (int v = 0; v < V; ++v) C.vchild_ptr[v + 1] = C.vchild_ptr[v] + (int32_t)vkids[v].size();
  C.vchild_idx.clear();
  for (int v = 0; v < V; ++v) for (int u : vkids[v]) C.vchild_idx.push_back(u);
  int vnlev = 0;
  for (int v = 0; v < V; ++v) vnlev = std::max(vnlev, vlevel[v] + 1);
  C.vlvl_ptr.assign(vnlev + 1, 0);
  for (int v = 0; v < V; ++v) ++C.vlvl_ptr[vlevel[v] + 1];
  for (int l = 0; l < vnlev; ++l) C.vlvl_ptr[l + 1] += C.vlvl_ptr[l];
  C.vlvl_nodes.assign(V, 0);
  {
    std::vector<int32_t> fill(C.vlvl_ptr.begin(), C.vlvl_ptr.end() - 1);
    for (int v = 0; v < V; ++v) C.vlvl_nodes[fill[vlevel[v]]++] = v;
  }
  return std::string();
}

}  // namespace mdnp
