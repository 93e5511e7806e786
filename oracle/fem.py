"""FP64 assembly of the coupled 3D-1D finite-element system (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2.1 of the paper: the weak form a(u, v) = a_Omega + a_Lambda
+ b_Lambda(T u_Omega - u_Lambda, T v_Omega - v_Lambda) and its Galerkin block
system A = K + M with K = diag(K00, K11) and the coupling block M
(eq. "mainsys").  The restriction operator T_Lambda is the cross-section
average on the vessel wall (Section 2, definition of T_Lambda), evaluated with
an equispaced rule of `n_circle` points on the circle of radius R around each
1D quadrature point.

Readings taken where the paper leaves a choice (listed in the design notes):
  * 3D space: trilinear (Q1) elements on a uniform grid of N^3 cells of the
    unit cube (the paper allows "tetrahedrons or bricks" on a uniform mesh);
    homogeneous Dirichlet conditions by symmetric elimination, boundary rows
    and columns replaced by the identity, boundary nodes kept as unknowns;
    or (instance boundary "neumann", the setup of the paper's Section 5) the
    natural condition: every node free, nothing eliminated.
  * The 3D-block problem of Section 5 (instance problem "block3d"): C = A00
    alone with b = -A01 A11^-1 f_1 (eq. "matrixC", eq. "setB"), written as
    [C 0; 0 I] [u0; u1] = [b; 0] so that it shares the coupled layout.
  * 1D diffusion carries the cross-section area: k_Lambda * pi R^2 (weak form
    a_Lambda with the |D| weight).
  * One perimeter factor in the coupling: c = 2 pi R beta, i.e. the block
    system "K + 2 pi eps M" with eps = R and a wall permeability beta.
  * Source f_Lambda on the graph, no 3D source (right-hand side [0; f_1]).
  * The 1D mesh has `elems_per_segment` P1 elements per straight segment; its
    nodes are numbered vertices first, then the interior nodes of segment s as
    V + s (E - 1) + t, t running from the parent end to the child end.
  * Quadrature: 2-point Gauss-Legendre per 1D element for every line integral.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

GAUSS2 = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))


# --------------------------------------------------------------------------
# 3D trilinear element (a_Omega of Section 2.1, eq. "aomega")
# --------------------------------------------------------------------------

def q1_reference_matrices():
    """Stiffness and mass matrices of the trilinear element on [0, 1]^3.

    Local node l = a + 2 b + 4 c sits at corner (a, b, c).  The integrals
    int grad(phi_l) . grad(phi_m) and int phi_l phi_m are evaluated by
    2 x 2 x 2 Gauss quadrature, exact for these polynomial integrands.
    """
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    corners = [(l & 1, (l >> 1) & 1, (l >> 2) & 1) for l in range(8)]
    for gx in GAUSS2:
        for gy in GAUSS2:
            for gz in GAUSS2:
                x = (gx, gy, gz)
                phi = np.zeros(8)
                grad = np.zeros((8, 3))
                for l, c in enumerate(corners):
                    f = [x[d] if c[d] else 1.0 - x[d] for d in range(3)]
                    df = [1.0 if c[d] else -1.0 for d in range(3)]
                    phi[l] = f[0] * f[1] * f[2]
                    grad[l, 0] = df[0] * f[1] * f[2]
                    grad[l, 1] = f[0] * df[1] * f[2]
                    grad[l, 2] = f[0] * f[1] * df[2]
                K += 0.125 * grad @ grad.T
                M += 0.125 * np.outer(phi, phi)
    return K, M


def trilinear_values(xi: np.ndarray) -> np.ndarray:
    """Values of the 8 trilinear basis functions at local points xi[..., 3]."""
    out = np.empty(xi.shape[:-1] + (8,))
    for l in range(8):
        a, b, c = l & 1, (l >> 1) & 1, (l >> 2) & 1
        fx = xi[..., 0] if a else 1.0 - xi[..., 0]
        fy = xi[..., 1] if b else 1.0 - xi[..., 1]
        fz = xi[..., 2] if c else 1.0 - xi[..., 2]
        out[..., l] = fx * fy * fz
    return out


def grid_node_xyz(n_cells: int) -> np.ndarray:
    """Coordinates of the (N+1)^3 grid nodes, index i + n j + n^2 k (x fastest)."""
    n = n_cells + 1
    h = 1.0 / n_cells
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.stack([i.ravel() * h, j.ravel() * h, k.ravel() * h], axis=1)


def boundary_mask(n_cells: int) -> np.ndarray:
    n = n_cells + 1
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    b = (i == 0) | (i == n - 1) | (j == 0) | (j == n - 1) | (k == 0) | (k == n - 1)
    return b.ravel()


def cell_node_ids(n_cells: int) -> np.ndarray:
    """[N^3, 8] global node ids of every cell, local order l = a + 2b + 4c."""
    n = n_cells + 1
    ck, cj, ci = np.meshgrid(np.arange(n_cells), np.arange(n_cells), np.arange(n_cells), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    ids = np.empty((ci.size, 8), dtype=np.int64)
    for l in range(8):
        a, b, c = l & 1, (l >> 1) & 1, (l >> 2) & 1
        ids[:, l] = (ci + a) + n * (cj + b) + n * n * (ck + c)
    return ids


# --------------------------------------------------------------------------
# 1D graph mesh
# --------------------------------------------------------------------------

def graph_mesh(vertex_xyz, seg, elems_per_segment):
    """P1 mesh of the vessel tree.

    Returns node positions [N1D, 3], elements [S*E, 2] (local 1D indices, from
    the parent end towards the child end) and the segment of each element.
    """
    V = vertex_xyz.shape[0]
    S = seg.shape[0]
    E = elems_per_segment
    n1d = V + S * (E - 1)
    pos = np.zeros((n1d, 3))
    pos[:V] = vertex_xyz
    elems = np.zeros((S * E, 2), dtype=np.int64)
    eseg = np.zeros(S * E, dtype=np.int64)
    for s in range(S):
        p, q = int(seg[s, 0]), int(seg[s, 1])
        P, Q = vertex_xyz[p], vertex_xyz[q]
        chain = [p] + [V + s * (E - 1) + t for t in range(E - 1)] + [q]
        for t in range(1, E):
            pos[V + s * (E - 1) + t - 1] = P + (t / E) * (Q - P)
        for e in range(E):
            elems[s * E + e] = (chain[e], chain[e + 1])
            eseg[s * E + e] = s
    return pos, elems, eseg


def wall_frame(tau: np.ndarray):
    """Orthonormal (n1, n2) normal to the unit tangent tau.

    n1 = normalise(tau x e_a) with a = argmin_k |tau_k| (first on ties),
    n2 = tau x n1.
    """
    a = int(np.argmin(np.abs(tau)))
    e = np.zeros(3)
    e[a] = 1.0
    n1 = np.cross(tau, e)
    n1 /= np.linalg.norm(n1)
    n2 = np.cross(tau, n1)
    return n1, n2


# --------------------------------------------------------------------------
# Assembled system
# --------------------------------------------------------------------------

@dataclass
class System:
    n_cells: int
    n3d: int
    n1d: int
    A: sp.csr_matrix          # full block matrix after Dirichlet elimination (if Dirichlet)
    F: np.ndarray             # right-hand side [0; f_1]
    boundary: np.ndarray      # bool [n3d]
    dist: Optional[np.ndarray]  # distance field d_h at the 3D nodes (None if not tabulated)
    alpha: float              # RMS of diag(A00) over free 3D nodes
    Pi: sp.csr_matrix         # averaging operator, [n_gauss, n3d] (before BCs)
    Phi: sp.csr_matrix        # 1D evaluation at Gauss points, [n_gauss, n1d]
    W: np.ndarray             # c * quadrature weight per Gauss point
    K11: sp.csr_matrix        # 1D stiffness block (before coupling)
    gauss_xyz: np.ndarray     # Gauss point positions on the centre line
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.n3d + self.n1d

    def blocks(self):
        A, m = self.A, self.n3d
        return A[:m, :m].tocsr(), A[:m, m:].tocsr(), A[m:, :m].tocsr(), A[m:, m:].tocsr()


def averaging_operator(n_cells, gauss_xyz, gauss_tau, gauss_radius, n_circle):
    """Pi[q, j] = (1/n_circle) sum_k phi_j(x_{q,k}) (cross-section average, T_Lambda).

    The circle points x_{q,k} = lambda_q + R (cos th_k n1 + sin th_k n2),
    th_k = 2 pi k / n_circle.  Every point contributes to all 8 nodes of the
    cell containing it, also where a basis value is zero (structural entry).
    Cell index per axis: min(floor(x / h), N - 1); local coordinate x/h - i.
    """
    N = n_cells
    n = N + 1
    h = 1.0 / N
    nq = gauss_xyz.shape[0]
    th = 2.0 * math.pi * np.arange(n_circle) / n_circle
    rows, cols, vals = [], [], []
    for q in range(nq):
        n1, n2 = wall_frame(gauss_tau[q])
        pts = (gauss_xyz[q][None, :]
               + gauss_radius[q] * (np.cos(th)[:, None] * n1[None, :] + np.sin(th)[:, None] * n2[None, :]))
        cell = np.clip(np.floor(pts / h).astype(np.int64), 0, N - 1)
        xi = pts / h - cell
        phi = trilinear_values(xi)  # [n_circle, 8]
        for l in range(8):
            a, b, c = l & 1, (l >> 1) & 1, (l >> 2) & 1
            node = (cell[:, 0] + a) + n * (cell[:, 1] + b) + n * n * (cell[:, 2] + c)
            rows.append(np.full(n_circle, q))
            cols.append(node)
            vals.append(phi[:, l] / n_circle)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    Pi = sp.coo_matrix((vals, (rows, cols)), shape=(nq, n ** 3)).tocsr()
    Pi.sum_duplicates()
    Pi.sort_indices()
    return Pi


def distance_field(n_cells, vertex_xyz, seg) -> np.ndarray:
    """d(x) = min over segments of |x - proj_[P,Q](x)| at every grid node (Section 2.1)."""
    X = grid_node_xyz(n_cells)
    d = np.full(X.shape[0], np.inf)
    for s in range(seg.shape[0]):
        P = vertex_xyz[seg[s, 0]]
        Q = vertex_xyz[seg[s, 1]]
        D = Q - P
        t = np.clip(((X - P) @ D) / (D @ D), 0.0, 1.0)
        dist = np.linalg.norm(X - (P + t[:, None] * D), axis=1)
        d = np.minimum(d, dist)
    return d


def assemble(inst, with_distance: bool = True) -> System:
    """Assemble A = K + M and F for one instance (eq. "mainsys").

    with_distance=False leaves System.dist as None: the distance field is only
    an input of the network and costs O(nodes x segments) to tabulate.

    K00: trilinear stiffness k_Omega (grad u, grad v) plus sigma_Omega mass.
    K11: k_Lambda pi R^2 (u', v') on the P1 graph mesh.
    M  : sum over Gauss points q of W_q (Pi_q u0 - Phi_q u1)(Pi_q v0 - Phi_q v1),
         W_q = 2 pi R beta * (l/2), i.e. M00 = Pi^T W Pi, M01 = -Pi^T W Phi,
         M10 = M01^T, M11 = Phi^T W Phi.
    F  : [0; int_Lambda f_Lambda phi_a ds].
    The sparsity pattern is structural: all node pairs of each trilinear cell,
    all pairs among the 3D nodes of the located cells and the two 1D nodes of
    each Gauss point, and the 1D element pairs; Dirichlet rows and columns are
    removed and a unit diagonal put back.
    """
    N = inst.n_cells
    n = N + 1
    h = 1.0 / N
    n3d = n ** 3
    E = inst.elems_per_segment
    V = inst.vertex_xyz.shape[0]
    S = inst.seg.shape[0]

    Kref, Mref = q1_reference_matrices()
    Ke = inst.k_omega * h * Kref + inst.sigma_omega * h ** 3 * Mref
    ids = cell_node_ids(N)
    r3 = np.repeat(ids, 8, axis=1).ravel()
    c3 = np.tile(ids, (1, 8)).ravel()
    v3 = np.tile(Ke.ravel(), ids.shape[0])

    pos1d, elems, eseg = graph_mesh(inst.vertex_xyz, inst.seg, E)
    n1d = pos1d.shape[0]

    # 1D stiffness and load
    Pa, Pb = pos1d[elems[:, 0]], pos1d[elems[:, 1]]
    ell = np.linalg.norm(Pb - Pa, axis=1)
    R = inst.radius[eseg]
    beta = inst.beta[eseg]
    kk = inst.k_lambda * math.pi * R ** 2 / ell
    loc = np.array([[1.0, -1.0], [-1.0, 1.0]])
    r11 = np.stack([elems[:, 0], elems[:, 0], elems[:, 1], elems[:, 1]], axis=1).ravel()
    c11 = np.stack([elems[:, 0], elems[:, 1], elems[:, 0], elems[:, 1]], axis=1).ravel()
    v11 = (kk[:, None] * loc.ravel()[None, :]).ravel()
    K11 = sp.coo_matrix((v11, (r11, c11)), shape=(n1d, n1d)).tocsr()
    F1 = np.zeros(n1d)
    np.add.at(F1, elems[:, 0], inst.f_lambda * ell / 2)
    np.add.at(F1, elems[:, 1], inst.f_lambda * ell / 2)

    # Gauss points on the centre line
    tq = np.array(GAUSS2)
    ne = elems.shape[0]
    gauss_xyz = (Pa[:, None, :] + tq[None, :, None] * (Pb - Pa)[:, None, :]).reshape(-1, 3)
    tau = (Pb - Pa) / ell[:, None]
    gauss_tau = np.repeat(tau, 2, axis=0)
    gauss_R = np.repeat(R, 2)
    W = np.repeat(2.0 * math.pi * R * beta * ell / 2.0, 2)
    phi1 = np.stack([1.0 - tq, tq], axis=1)  # [2, 2]
    Phi_rows = np.repeat(np.arange(2 * ne), 2)
    Phi_cols = np.stack([np.repeat(elems[:, 0], 2), np.repeat(elems[:, 1], 2)], axis=1).ravel()
    Phi_vals = np.tile(phi1, (ne, 1)).ravel()
    Phi = sp.coo_matrix((Phi_vals, (Phi_rows, Phi_cols)), shape=(2 * ne, n1d)).tocsr()

    Pi = averaging_operator(N, gauss_xyz, gauss_tau, gauss_R, inst.n_circle)

    # Coupling triplets, one Gauss point at a time
    rc, cc, vc = [], [], []
    for q in range(2 * ne):
        J = Pi.indices[Pi.indptr[q]:Pi.indptr[q + 1]].astype(np.int64)
        p = Pi.data[Pi.indptr[q]:Pi.indptr[q + 1]]
        T = n3d + Phi.indices[Phi.indptr[q]:Phi.indptr[q + 1]].astype(np.int64)
        f = Phi.data[Phi.indptr[q]:Phi.indptr[q + 1]]
        nodes = np.concatenate([J, T])
        coef = np.concatenate([p, -f])  # (Pi v0 - Phi v1)
        rc.append(np.repeat(nodes, nodes.size))
        cc.append(np.tile(nodes, nodes.size))
        vc.append(W[q] * np.outer(coef, coef).ravel())
    rows = np.concatenate([r3, n3d + r11] + rc)
    cols = np.concatenate([c3, n3d + c11] + cc)
    vals = np.concatenate([v3, v11] + vc)

    # symmetric Dirichlet elimination on the 3D boundary; with the natural
    # (Neumann) condition every 3D node stays free and nothing is removed
    if getattr(inst, "boundary", "dirichlet") == "neumann":
        bnd = np.zeros(n3d, dtype=bool)
    else:
        bnd = boundary_mask(N)
        isb = np.zeros(n3d + n1d, dtype=bool)
        isb[:n3d] = bnd
        keep = ~(isb[rows] | isb[cols])
        bidx = np.nonzero(bnd)[0]
        rows = np.concatenate([rows[keep], bidx])
        cols = np.concatenate([cols[keep], bidx])
        vals = np.concatenate([vals[keep], np.ones(bidx.size)])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n3d + n1d, n3d + n1d)).tocsr()
    A.sum_duplicates()
    A.sort_indices()

    F = np.zeros(n3d + n1d)
    F[n3d:] = F1

    dist = distance_field(N, inst.vertex_xyz, inst.seg) if with_distance else None
    dg = A.diagonal()[:n3d][~bnd]
    alpha = float(np.sqrt(np.mean(dg ** 2)))
    out = System(n_cells=N, n3d=n3d, n1d=n1d, A=A, F=F, boundary=bnd, dist=dist, alpha=alpha,
                 Pi=Pi, Phi=Phi, W=W, K11=K11, gauss_xyz=gauss_xyz,
                 extra={"pos1d": pos1d, "elems": elems, "eseg": eseg, "gauss_tau": gauss_tau,
                        "gauss_R": gauss_R})
    if getattr(inst, "problem", "coupled") == "block3d":
        return block3d_system(out)
    return out


def block3d_rhs(system):
    """Right-hand side of the 3D block problem (eq. "decoupled_3d_problem" with
    z = F, eq. "setB"): b = -A01 x with A11 x = f_1, i.e. the 3D forcing that the
    1D solution exerts through the coupling (A01 = 2 pi eps M01, A11 = K11 +
    2 pi eps M11)."""
    A00, A01, A10, A11 = system.blocks()
    x1 = spla.spsolve(A11.tocsc(), system.F[system.n3d:])
    return -(A01 @ x1)


def block3d_system(system):
    """The 3D block C = K00 + 2 pi eps M00 alone (eq. "matrixC"), written in
    the coupled layout as [C 0; 0 I] [u0; u1] = [b; 0] with b from
    `block3d_rhs`: the 1D unknowns are decoupled identities whose part of every
    Krylov vector stays zero, so any solver of the coupled layout solves
    C u0 = b.  The coupling operators Pi, Phi, W describe the tree as before."""
    m = system.n3d
    A00 = system.blocks()[0]
    b = block3d_rhs(system)
    A = sp.bmat([[A00, None], [None, sp.identity(system.n1d, format="csr")]], format="csr")
    A.sort_indices()
    F = np.concatenate([b, np.zeros(system.n1d)])
    extra = dict(system.extra)
    extra["coupled_A"] = system.A
    extra["coupled_F"] = system.F
    return System(n_cells=system.n_cells, n3d=m, n1d=system.n1d, A=A, F=F, boundary=system.boundary,
                  dist=system.dist, alpha=system.alpha, Pi=system.Pi, Phi=system.Phi, W=system.W,
                  K11=system.K11, gauss_xyz=system.gauss_xyz, extra=extra)
