// Host-side assembly of one instance of the coupled 3D-1D system (Section 2.1).
// Independent implementation used by the library at upload time.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mdnp.h"

namespace mdnp {

struct TreeFactor {
  // Leaves-first LDL^T of the tree matrix A11 (no fill).  Local 1D indices.
  std::vector<int32_t> parent;      // parent node, -1 at the root
  std::vector<double> lval;         // L[parent(c), c] = a_{p c} / d_c
  std::vector<double> dinv;         // 1 / d_c
  std::vector<int32_t> child_ptr;   // children of each node (CSR)
  std::vector<int32_t> child_idx;
  std::vector<int32_t> lvl_ptr;     // nodes grouped by level: level(c) = 1 + max level(children)
  std::vector<int32_t> lvl_nodes;
};

struct ChainFactor {
  // Chain-compressed solve of A11: the m = E - 1 interior nodes of every
  // segment form a tridiagonal block T_s between the segment's parent-side
  // vertex p and child vertex q.  Per segment: y = T_s^-1 v_c; the vertices
  // solve the Schur complement (a tree over the vertices, edges = segments)
  // with right-hand side v_v - (couplings) y; then z_c = y - g_p z_p - g_q z_q.
  // Per-step arrays are laid out [step][segment].
  int m = 0;                        // interior nodes per segment
  std::vector<double> fmul;         // [m - 1][S]: w_i = v_i - fmul_i w_{i+1}
  std::vector<double> pinv;         // [m][S]: 1 / pivot_i (elimination from the q end)
  std::vector<double> eup;          // [m - 1][S]: T[i, i + 1] (back substitution towards q)
  std::vector<double> gp, gq;       // [m][S]: T^-1 (a_p e_0), T^-1 (a_q e_{m-1})
  std::vector<double> ap, aq;       // [S]: A[p, c_0], A[q, c_{m-1}]
  std::vector<int32_t> sp, sq;      // [S]: parent-side and child vertex
  // leaves-first LDL^T of the vertex Schur complement
  std::vector<int32_t> vparent, vseg, vchild_ptr, vchild_idx, vlvl_ptr, vlvl_nodes;
  std::vector<double> vlval, vdinv;
};

struct HostInstance {
  int n_cells = 0, n = 0, n3d = 0, n1d = 0;
  std::vector<int32_t> row_ptr, col;   // CSR of A, local indices, sorted columns
  std::vector<double> val;
  std::vector<int32_t> a01_start;      // per 3D row: first entry with a 1D column
  // Split form used by the device: A = S + M with S the constant 27-point
  // stencil on the interior 3D nodes (boundary neighbours left out; identity
  // on Dirichlet nodes, zero on Neumann boundary nodes) and M the coupling
  // entries of the 3D rows, the stencil entries S leaves out under the
  // natural boundary, and the whole 1D rows (CSR, sorted).
  double stencil[4] = {0, 0, 0, 0};    // stencil value by number of differing coordinates
  bool neumann = false;                // natural boundary: the stencil kernels yield 0 on boundary
                                       // rows (M holds those rows), Dirichlet: the unit row
  std::vector<int32_t> m_ptr, m_col;
  std::vector<double> m_val;
  std::vector<int32_t> m_a01;          // per 3D row: first M entry with a 1D column
  // M in factored form (eq. "mainsys"): M = B^T W B + R with one row of B per
  // Gauss point q, B_q = [Pi_q | -Phi_q] on the free nodes (its 3D columns
  // first, the two 1D columns from b_split[q]), W_q its weight, and R the rest
  // of M: the 1D stiffness rows (unit 1D rows in the 3D-block layout, which
  // has no 1D columns in B) and the natural-boundary stencil entries.
  std::vector<int32_t> b_ptr, b_col, b_split;
  std::vector<double> b_val, b_w;
  std::vector<int32_t> r_ptr, r_col;   // R in CSR over all rows, sorted columns
  std::vector<double> r_val;
  std::vector<double> F;               // right-hand side [n3d + n1d]
  std::vector<float> dist;             // distance field at the 3D nodes
  std::vector<double> diag;            // diag(A)
  double alpha = 0.0;                  // RMS of diag(A00) over the free 3D nodes
  TreeFactor tree;
  ChainFactor chain;
};

// Validates and assembles; returns an empty string on success or an error message.
// `geom_error` is set when the failure is a geometry error.
std::string assemble_instance(const mdnp_instance_desc& d, HostInstance& out, bool& geom_error);

}  // namespace mdnp
