"""Pins of the oracle assembly (Section 2.1, eq. "mainsys") against closed forms,
invariants, dense factorisations, brute force and a manufactured solution."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import fem


def small_instance(n_cells=8, seed=7, n_segments=4, E=3, radius=0.02, beta=1.0, **kw):
    return synth.make_instance(seed, n_cells, n_segments=n_segments, elems_per_segment=E,
                               radius=radius, beta=beta, **kw)


# ---------------------------------------------------------------- trilinear element

def test_q1_element_closed_form():
    """Trilinear stiffness on the unit cube: diagonal 1/3; pairs differing in one
    coordinate 0; in two or three coordinates -1/12 (tensor products of the 1D
    matrices [[1,-1],[-1,1]] and [[1/3,1/6],[1/6,1/3]])."""
    K, M = fem.q1_reference_matrices()
    for a in range(8):
        for b in range(8):
            ndiff = bin(a ^ b).count("1")
            expect = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[ndiff]
            assert K[a, b] == pytest.approx(expect, abs=1e-15)
            assert M[a, b] == pytest.approx((1 / 3) ** (3 - ndiff) * (1 / 6) ** ndiff, abs=1e-15)


def test_assembled_stencil_values():
    """Interior 3D rows far from the vessel: k h {8/3 centre, 0 faces, -1/6 edges, -1/12 corners}."""
    inst = small_instance(n_cells=12, n_segments=1, k_omega=2.0)
    s = fem.assemble(inst)
    n, h = 13, 1 / 12
    A = s.A
    Pi_nodes = set(s.Pi.indices.tolist())
    checked = 0
    for k in range(2, n - 2):
        for j in range(2, n - 2):
            for i in range(2, n - 2):
                r = i + n * j + n * n * k
                if any((i + a) + n * (j + b) + n * n * (k + c) in Pi_nodes
                       for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)):
                    continue
                cols = A.indices[A.indptr[r]:A.indptr[r + 1]]
                vals = A.data[A.indptr[r]:A.indptr[r + 1]]
                assert len(cols) == 27
                for c, v in zip(cols, vals):
                    ci, cj, ck = c % n, (c // n) % n, c // (n * n)
                    nd = int(ci != i) + int(cj != j) + int(ck != k)
                    expect = 2.0 * h * {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[nd]
                    assert v == pytest.approx(expect, abs=1e-15)
                checked += 1
    assert checked > 10


def test_stiffness_kernel_and_mass():
    """Before boundary conditions the stiffness annihilates constants and the
    mass integrates 1 to the cell volume: checked on rows with no boundary column."""
    inst = small_instance(n_cells=6, beta=0.0, sigma_omega=0.0)
    s = fem.assemble(inst)
    A00 = s.blocks()[0]
    # rows whose 27-point neighbourhood holds no boundary node (index 2..n-3 on every axis)
    X = np.rint(fem.grid_node_xyz(6) * 6).astype(int)
    rows = np.all((X >= 2) & (X <= 4), axis=1)
    assert rows.sum() > 0
    assert np.max(np.abs(A00 @ np.ones(s.n3d))[rows]) < 1e-15
    inst2 = small_instance(n_cells=6, beta=0.0, k_omega=0.0, sigma_omega=1.0)
    s2 = fem.assemble(inst2)
    m = s2.blocks()[0] @ np.ones(s2.n3d)
    assert np.allclose(m[rows], (1 / 6) ** 3, rtol=1e-13)


def test_symmetry_and_spd():
    """A = A^T; A, A00 and A11 are SPD (dense Cholesky) on the 16^3 single-instance case."""
    s = fem.assemble(synth.workload_single_fp64()[0])
    A = s.A
    assert abs(A - A.T).max() < 1e-15
    A00, A01, A10, A11 = s.blocks()
    sla.cholesky(A11.toarray())
    Ad = A.toarray()
    sla.cholesky(Ad)
    sla.cholesky(A00.toarray())


# ---------------------------------------------------------------- 1D blocks

def test_1d_blocks_closed_form():
    """K11 = k pi R^2 / l [[1,-1],[-1,1]], M11 = c l/6 [[2,1],[1,2]] per element,
    sum F1 = total length (f = 1), K11 1 = 0."""
    inst = small_instance(n_cells=8, n_segments=5, E=4, radius=0.015, beta=1.7, k_lambda=3.0)
    s = fem.assemble(inst)
    pos, elems = s.extra["pos1d"], s.extra["elems"]
    ell = np.linalg.norm(pos[elems[:, 1]] - pos[elems[:, 0]], axis=1)
    K = np.zeros((s.n1d, s.n1d))
    Mm = np.zeros((s.n1d, s.n1d))
    c = 2 * math.pi * 0.015 * 1.7
    for (a, b), l in zip(elems, ell):
        K[np.ix_([a, b], [a, b])] += 3.0 * math.pi * 0.015 ** 2 / l * np.array([[1, -1], [-1, 1]])
        Mm[np.ix_([a, b], [a, b])] += c * l / 6 * np.array([[2, 1], [1, 2]])
    assert np.allclose(s.K11.toarray(), K, rtol=1e-13, atol=1e-18)
    A11 = s.blocks()[3].toarray()
    assert np.allclose(A11, K + Mm, rtol=1e-12, atol=1e-17)
    assert np.max(np.abs(s.K11 @ np.ones(s.n1d))) < 1e-15
    seglen = np.linalg.norm(inst.vertex_xyz[inst.seg[:, 1]] - inst.vertex_xyz[inst.seg[:, 0]], axis=1)
    assert s.F[s.n3d:].sum() == pytest.approx(seglen.sum(), rel=1e-13)


def test_graph_numbering():
    """Vertices first, then V + s(E-1) + t from the parent end; V = S + 1 and the
    element graph is a tree (edges = nodes - 1, connected)."""
    inst = small_instance(n_segments=6, E=3)
    pos, elems, eseg = fem.graph_mesh(inst.vertex_xyz, inst.seg, 3)
    V, S, E = inst.n_vertices, inst.n_segments, 3
    assert V == S + 1
    assert pos.shape[0] == V + S * (E - 1)
    assert elems.shape[0] == pos.shape[0] - 1
    for s in range(S):
        chain = [inst.seg[s, 0]] + [V + s * (E - 1) + t for t in range(E - 1)] + [inst.seg[s, 1]]
        assert [tuple(e) for e in elems[s * E:(s + 1) * E]] == list(zip(chain[:-1], chain[1:]))
        P, Q = inst.vertex_xyz[inst.seg[s, 0]], inst.vertex_xyz[inst.seg[s, 1]]
        for t in range(1, E):
            assert np.allclose(pos[V + s * (E - 1) + t - 1], P + t / E * (Q - P))
    G = sp.coo_matrix((np.ones(len(elems)), (elems[:, 0], elems[:, 1])), shape=(len(pos),) * 2)
    ncomp, _ = sp.csgraph.connected_components(G, directed=False)
    assert ncomp == 1
    assert np.all((inst.vertex_xyz >= 0.2) & (inst.vertex_xyz <= 0.8))


# ---------------------------------------------------------------- averaging operator

def test_wall_frame_orthonormal():
    rng = np.random.default_rng(3)
    for _ in range(50):
        t = rng.normal(size=3)
        t /= np.linalg.norm(t)
        n1, n2 = fem.wall_frame(t)
        F = np.stack([t, n1, n2])
        assert np.allclose(F @ F.T, np.eye(3), atol=1e-14)
    n1, n2 = fem.wall_frame(np.array([0.0, 0.0, 1.0]))   # tie rule: first minimal axis
    assert np.allclose(n1, np.cross([0, 0, 1.0], [1.0, 0, 0]))


def test_averaging_reproduces_polynomials():
    """Pi 1 = 1; for an affine f the circle average equals f at the centre; for
    the trilinear f = x y z it equals the closed form
    E[(a0+a.u)(b0+b.u)(c0+c.u)] = a0 b0 c0 + (a0 b.c + b0 a.c + c0 a.b)/2
    over u = (cos th, sin th) (equispaced rules with >= 4 points integrate
    trigonometric degree 3 exactly, and the Q1 interpolant of x y z is exact)."""
    inst = small_instance(n_cells=8, n_segments=6, E=3, radius=0.03)
    s = fem.assemble(inst)
    X = fem.grid_node_xyz(8)
    one = s.Pi @ np.ones(s.n3d)
    assert np.allclose(one, 1.0, atol=1e-14)
    g = s.gauss_xyz
    lin = 0.3 + 1.2 * X[:, 0] - 0.7 * X[:, 1] + 2.1 * X[:, 2]
    assert np.allclose(s.Pi @ lin, 0.3 + 1.2 * g[:, 0] - 0.7 * g[:, 1] + 2.1 * g[:, 2], atol=1e-13)
    tri = X[:, 0] * X[:, 1] * X[:, 2]
    got = s.Pi @ tri
    R = s.extra["gauss_R"]
    for q in range(g.shape[0]):
        n1, n2 = fem.wall_frame(s.extra["gauss_tau"][q])
        a0, b0, c0 = g[q]
        a = R[q] * np.array([n1[0], n2[0]])
        b = R[q] * np.array([n1[1], n2[1]])
        c = R[q] * np.array([n1[2], n2[2]])
        expect = a0 * b0 * c0 + 0.5 * (a0 * (b @ c) + b0 * (a @ c) + c0 * (a @ b))
        assert got[q] == pytest.approx(expect, abs=1e-14)


def test_coupling_annihilates_constants():
    """M [1; 1] = 0 since T 1 = 1 and the P1 basis sums to one: with k = sigma = 0
    the assembled matrix is M (plus boundary identity rows)."""
    inst = small_instance(n_cells=8, n_segments=5, E=4, radius=0.02, beta=1.3, k_omega=0.0,
                          k_lambda=0.0)
    s = fem.assemble(inst)
    y = s.A @ np.ones(s.n)
    rows = np.ones(s.n, dtype=bool)
    rows[:s.n3d] = ~s.boundary
    assert np.max(np.abs(y[rows])) < 1e-15
    w = np.linalg.eigvalsh(s.A.toarray()[np.ix_(rows, rows)])
    assert w.min() > -1e-15            # M is positive semi-definite


def test_sparsity_structure():
    """Boundary rows hold only the unit diagonal; columns sorted and unique;
    every 1D node row holds its graph neighbours."""
    s = fem.assemble(small_instance(n_cells=8))
    A = s.A
    for r in np.nonzero(s.boundary)[0]:
        assert list(A.indices[A.indptr[r]:A.indptr[r + 1]]) == [r]
        assert A.data[A.indptr[r]] == 1.0
    for r in range(A.shape[0]):
        c = A.indices[A.indptr[r]:A.indptr[r + 1]]
        assert np.all(np.diff(c) > 0)
    for a, b in s.extra["elems"]:
        row = A.indices[A.indptr[s.n3d + a]:A.indptr[s.n3d + a + 1]]
        assert s.n3d + b in row


def test_distance_field_brute_force():
    inst = small_instance(n_cells=4, n_segments=3)
    d = fem.distance_field(4, inst.vertex_xyz, inst.seg)
    X = fem.grid_node_xyz(4)
    for idx in range(X.shape[0]):
        best = 1e9
        for s in range(inst.n_segments):
            P = inst.vertex_xyz[inst.seg[s, 0]]
            Q = inst.vertex_xyz[inst.seg[s, 1]]
            # brute force: dense sampling of the segment plus its end points
            ts = np.linspace(0, 1, 20001)
            pts = P[None, :] + ts[:, None] * (Q - P)[None, :]
            best = min(best, float(np.min(np.linalg.norm(pts - X[idx], axis=1))))
        assert d[idx] == pytest.approx(best, abs=2e-5)
    # single segment closed form: distance to the x axis-parallel segment
    v = np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]])
    d1 = fem.distance_field(4, v, np.array([[0, 1]]))
    for idx in range(X.shape[0]):
        x, y, z = X[idx]
        dx = max(0.25 - x, 0.0, x - 0.75)
        assert d1[idx] == pytest.approx(math.sqrt(dx ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2), abs=1e-15)


def test_direct_solve_matches_dense_lu():
    s = fem.assemble(synth.workload_single_fp64()[0])
    from oracle import krylov
    x = krylov.direct_solve(s)
    xd = sla.lu_solve(sla.lu_factor(s.A.toarray()), s.F)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12


# ---------------------------------------------------------------- manufactured solution

def _gauss3():
    p = np.array([0.5 - 0.5 * math.sqrt(3 / 5), 0.5, 0.5 + 0.5 * math.sqrt(3 / 5)])
    w = np.array([5 / 18, 8 / 18, 5 / 18])
    return p, w


def _manufactured_errors(N):
    """Galerkin solution of the coupled problem with exact solution
    u_O = sin(pi x) sin(pi y) sin(pi z), u_L = T u_O + g, g = 0.5 + x y.
    Loads (consistent with the weak form of Section 2.1):
      F0 = int 3 pi^2 u_O phi - sum_q W_q g(s_q) Pi_q,
      F1 = K11 I(u_L) + sum_q W_q g(s_q) Phi_q
    (a_Lambda(u, phi_a) depends only on the nodal values of u for P1 tests).
    Returns the H1-seminorm and L2 errors of the 3D part."""
    inst = synth.make_instance(11, N, n_segments=6, elems_per_segment=6, radius=0.01, beta=1.0)
    s = fem.assemble(inst)
    n = N + 1
    h = 1.0 / N
    uex = lambda P: np.sin(np.pi * P[..., 0]) * np.sin(np.pi * P[..., 1]) * np.sin(np.pi * P[..., 2])
    g = lambda P: 0.5 + P[..., 0] * P[..., 1]
    # exact circle average of u_O at the 1D nodes (a 64-point rule is exact to rounding for R << 1)
    pos = s.extra["pos1d"]
    elems = s.extra["elems"]
    eseg = s.extra["eseg"]
    tang = np.zeros_like(pos)
    for (a, b), sg in zip(elems, eseg):
        t = pos[b] - pos[a]
        tang[a] = t / np.linalg.norm(t)
        tang[b] = t / np.linalg.norm(t)
    th = 2 * np.pi * np.arange(64) / 64
    Tu = np.zeros(pos.shape[0])
    for i in range(pos.shape[0]):
        n1, n2 = fem.wall_frame(tang[i])
        pts = pos[i] + 0.01 * (np.cos(th)[:, None] * n1 + np.sin(th)[:, None] * n2)
        Tu[i] = uex(pts).mean()
    uL = Tu + g(pos)
    gq = g(s.gauss_xyz)
    # 3D load by 3x3x3 Gauss per cell
    p, w = _gauss3()
    ids = fem.cell_node_ids(N)
    cz, cy, cx = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    org = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1) * h
    F0 = np.zeros(s.n3d)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                xi = np.array([p[a], p[b], p[c]])
                phi = fem.trilinear_values(xi[None, :])[0]
                P = org + h * xi
                val = 3 * np.pi ** 2 * uex(P) * w[a] * w[b] * w[c] * h ** 3
                for l in range(8):
                    np.add.at(F0, ids[:, l], val * phi[l])
    F0 -= s.Pi.T @ (s.W * gq)
    F1 = s.K11 @ uL + s.Phi.T @ (s.W * gq)
    F = np.concatenate([F0, F1])
    F[:s.n3d][s.boundary] = 0.0
    u = spla.spsolve(s.A.tocsc(), F)
    uh = u[:s.n3d]
    # H1 seminorm and L2 errors by 3x3x3 Gauss
    eh1 = 0.0
    el2 = 0.0
    corners = [(l & 1, (l >> 1) & 1, (l >> 2) & 1) for l in range(8)]
    U = uh[ids]
    for a in range(3):
        for b in range(3):
            for c in range(3):
                xi = np.array([p[a], p[b], p[c]])
                wt = w[a] * w[b] * w[c] * h ** 3
                phi = fem.trilinear_values(xi[None, :])[0]
                grad = np.zeros((8, 3))
                for l, cc in enumerate(corners):
                    f = [xi[d] if cc[d] else 1 - xi[d] for d in range(3)]
                    df = [1.0 if cc[d] else -1.0 for d in range(3)]
                    grad[l] = [df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]]
                P = org + h * xi
                gx = np.pi * np.cos(np.pi * P[:, 0]) * np.sin(np.pi * P[:, 1]) * np.sin(np.pi * P[:, 2])
                gy = np.pi * np.sin(np.pi * P[:, 0]) * np.cos(np.pi * P[:, 1]) * np.sin(np.pi * P[:, 2])
                gz = np.pi * np.sin(np.pi * P[:, 0]) * np.sin(np.pi * P[:, 1]) * np.cos(np.pi * P[:, 2])
                gh = U @ grad / h
                eh1 += wt * np.sum((gx - gh[:, 0]) ** 2 + (gy - gh[:, 1]) ** 2 + (gz - gh[:, 2]) ** 2)
                el2 += wt * np.sum((uex(P) - U @ phi) ** 2)
    e1d = np.max(np.abs(u[s.n3d:] - uL))
    return math.sqrt(eh1), math.sqrt(el2), e1d


def test_manufactured_solution_convergence():
    """H1-seminorm error of the 3D part falls like O(h) (slope >= 0.9), L2 like O(h^2)."""
    errs = [_manufactured_errors(N) for N in (8, 16, 32)]
    h1 = [e[0] for e in errs]
    l2 = [e[1] for e in errs]
    s1 = [math.log2(h1[i] / h1[i + 1]) for i in range(2)]
    s2 = [math.log2(l2[i] / l2[i + 1]) for i in range(2)]
    assert min(s1) >= 0.9, (h1, s1)
    assert min(s2) >= 1.7, (l2, s2)
    assert errs[-1][2] < 0.05


# ---------------------------------------------------------------- network normalisation alpha (Section 5.1)

@pytest.mark.parametrize("k_omega,sigma", [(1.0, 0.0), (2.5, 0.0), (1.0, 30.0)])
def test_alpha_closed_form_without_coupling(k_omega, sigma):
    """alpha = RMS of diag(A00) over the free 3D nodes.  With beta = 0 the
    coupling vanishes and every free node has the trilinear diagonal
    k h 8/3 + sigma (2h/3)^3 (stiffness 8 x h/3 per cell around the node; the
    mass diagonal is the cube of the 1D value 2h/3), so alpha equals it."""
    N = 8
    h = 1.0 / N
    s = fem.assemble(small_instance(n_cells=N, beta=0.0, k_omega=k_omega, sigma_omega=sigma))
    expect = k_omega * h * 8.0 / 3.0 + sigma * (2.0 * h / 3.0) ** 3
    assert s.alpha == pytest.approx(expect, rel=1e-14)


def _brute_coupling_diagonal(inst):
    """Diagonal of the coupling block M00 = Pi^T W Pi by direct loops: for each
    P1 element, its two Gauss points, the n_circle points of the wall circle
    (frame n1 = tau x e_a / |.|, a = argmin |tau_k|, n2 = tau x n1), the
    trilinear weights of the containing cell, then W_q (Pi_qj)^2 per node."""
    N = inst.n_cells
    n = N + 1
    h = 1.0 / N
    diag = np.zeros(n ** 3)
    E = inst.elems_per_segment
    g = 0.5 / math.sqrt(3.0)
    for s_id, (p, q) in enumerate(inst.seg):
        P, Q = inst.vertex_xyz[p], inst.vertex_xyz[q]
        R, beta = inst.radius[s_id], inst.beta[s_id]
        tau = (Q - P) / np.linalg.norm(Q - P)
        a = int(np.argmin(np.abs(tau)))
        e = np.zeros(3)
        e[a] = 1.0
        n1 = np.cross(tau, e)
        n1 /= np.linalg.norm(n1)
        n2 = np.cross(tau, n1)
        ell = np.linalg.norm(Q - P) / E
        for el in range(E):
            for tq in (0.5 - g, 0.5 + g):
                c = P + (el + tq) / E * (Q - P)
                W = 2.0 * math.pi * R * beta * ell / 2.0
                pi = {}
                for k in range(inst.n_circle):
                    th = 2.0 * math.pi * k / inst.n_circle
                    x = c + R * (math.cos(th) * n1 + math.sin(th) * n2)
                    cell = [min(int(math.floor(x[d] / h)), N - 1) for d in range(3)]
                    xi = [x[d] / h - cell[d] for d in range(3)]
                    for dz in (0, 1):
                        for dy in (0, 1):
                            for dx in (0, 1):
                                wgt = ((xi[0] if dx else 1 - xi[0]) * (xi[1] if dy else 1 - xi[1])
                                       * (xi[2] if dz else 1 - xi[2]))
                                node = (cell[0] + dx) + n * (cell[1] + dy) + n * n * (cell[2] + dz)
                                pi[node] = pi.get(node, 0.0) + wgt / inst.n_circle
                for node, v in pi.items():
                    diag[node] += W * v * v
    return diag


def test_alpha_with_coupling_brute_force():
    """alpha on an 8^3 instance with coupling: RMS over the free nodes of
    k h 8/3 + the brute-force coupling diagonal."""
    inst = small_instance(n_cells=8, n_segments=5, radius=0.03, beta=3.0)
    s = fem.assemble(inst)
    h = 1.0 / 8
    free = ~fem.boundary_mask(8)
    d = h * 8.0 / 3.0 + _brute_coupling_diagonal(inst)
    expect = math.sqrt(float(np.mean(d[free] ** 2)))
    assert s.alpha == pytest.approx(expect, rel=1e-13)
    # the coupling is large enough here to move alpha well away from 8h/3
    assert s.alpha > (1 + 1e-4) * h * 8.0 / 3.0
    # and the assembled diagonal itself agrees node by node
    assert np.allclose(s.A.diagonal()[:s.n3d][free], d[free], rtol=1e-13)


# ---------------------------------------------------------------- natural (Neumann) boundary and the 3D block (Section 5)

def _neumann(n_cells=6, **kw):
    kw.setdefault("seed", 7)
    return small_instance(n_cells=n_cells, boundary="neumann", **kw)


def test_neumann_stiffness_kernel_and_symmetry():
    """With the natural boundary every node is free; the stiffness annihilates
    constants on every row (also the boundary rows), is symmetric and
    positive semi-definite with exactly one zero eigenvalue."""
    s = fem.assemble(_neumann(beta=0.0, sigma_omega=0.0))
    assert not s.boundary.any()
    A00 = s.blocks()[0]
    assert np.max(np.abs(A00 @ np.ones(s.n3d))) < 1e-14
    assert abs(A00 - A00.T).max() < 1e-15
    ev = np.linalg.eigvalsh(A00.toarray())
    assert abs(ev[0]) < 1e-12 and ev[1] > 1e-3


def test_neumann_mass_integrates_volume_and_node_counts():
    """k = 0, sigma = 1: 1^T M 1 = 1 (the unit cube's volume) and every row sum
    is the volume of the node's support (h^3 times 1, 1/2, 1/4, 1/8 for
    interior, face, edge and corner nodes); the stiffness diagonal scales with
    the same counts: k h 8/3 x (cells around the node) / 8."""
    N = 6
    h = 1.0 / N
    s = fem.assemble(_neumann(n_cells=N, beta=0.0, k_omega=0.0, sigma_omega=1.0))
    M = s.blocks()[0]
    assert float(np.ones(s.n3d) @ (M @ np.ones(s.n3d))) == pytest.approx(1.0, rel=1e-13)
    X = np.rint(fem.grid_node_xyz(N) * N).astype(int)
    on_face = ((X == 0) | (X == N)).sum(axis=1)          # 0 interior, 1 face, 2 edge, 3 corner
    cells = 8 / 2 ** on_face
    assert np.allclose(M @ np.ones(s.n3d), cells / 8 * h ** 3, rtol=1e-13)
    K = fem.assemble(_neumann(n_cells=N, beta=0.0, k_omega=1.0, sigma_omega=0.0)).blocks()[0]
    assert np.allclose(K.diagonal(), h * 8 / 3 * cells / 8, rtol=1e-13)


def test_neumann_coupled_system_spd():
    """With sigma > 0 the Neumann 3D block, the coupled matrix and C = A00 are
    SPD (dense Cholesky), at the paper's coefficients k = sigma = 1e-3."""
    s = fem.assemble(_neumann(n_cells=6, radius=1e-3, k_omega=1e-3, sigma_omega=1e-3))
    assert abs(s.A - s.A.T).max() < 1e-18
    sla.cholesky(s.A.toarray())
    sla.cholesky(s.blocks()[0].toarray())


def _neumann_manufactured_errors(N):
    """-k Lap u + sigma u = f in the unit cube with du/dn = 0 on its faces:
    u = cos(pi x) cos(pi y) cos(pi z), f = (3 pi^2 k + sigma) u, k = sigma = 1;
    no coupling (beta = 0).  Returns the H1-seminorm and L2 errors of the
    Galerkin solution of A00 u = int f phi."""
    s = fem.assemble(_neumann(n_cells=N, seed=11, beta=0.0, k_omega=1.0, sigma_omega=1.0))
    h = 1.0 / N
    c = lambda t: np.cos(np.pi * t)
    sn = lambda t: np.sin(np.pi * t)
    uex = lambda P: c(P[..., 0]) * c(P[..., 1]) * c(P[..., 2])
    p, w = _gauss3()
    ids = fem.cell_node_ids(N)
    cz, cy, cx = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    org = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1) * h
    F0 = np.zeros(s.n3d)
    for a in range(3):
        for b in range(3):
            for cc in range(3):
                xi = np.array([p[a], p[b], p[cc]])
                phi = fem.trilinear_values(xi[None, :])[0]
                val = (3 * np.pi ** 2 + 1.0) * uex(org + h * xi) * w[a] * w[b] * w[cc] * h ** 3
                for l in range(8):
                    np.add.at(F0, ids[:, l], val * phi[l])
    U = spla.spsolve(s.blocks()[0].tocsc(), F0)[ids]
    corners = [(l & 1, (l >> 1) & 1, (l >> 2) & 1) for l in range(8)]
    eh1 = el2 = 0.0
    for a in range(3):
        for b in range(3):
            for cc in range(3):
                xi = np.array([p[a], p[b], p[cc]])
                wt = w[a] * w[b] * w[cc] * h ** 3
                phi = fem.trilinear_values(xi[None, :])[0]
                grad = np.zeros((8, 3))
                for l, co in enumerate(corners):
                    f = [xi[d] if co[d] else 1 - xi[d] for d in range(3)]
                    df = [1.0 if co[d] else -1.0 for d in range(3)]
                    grad[l] = [df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]]
                P = org + h * xi
                gx = -np.pi * sn(P[:, 0]) * c(P[:, 1]) * c(P[:, 2])
                gy = -np.pi * c(P[:, 0]) * sn(P[:, 1]) * c(P[:, 2])
                gz = -np.pi * c(P[:, 0]) * c(P[:, 1]) * sn(P[:, 2])
                gh = U @ grad / h
                eh1 += wt * np.sum((gx - gh[:, 0]) ** 2 + (gy - gh[:, 1]) ** 2 + (gz - gh[:, 2]) ** 2)
                el2 += wt * np.sum((uex(P) - U @ phi) ** 2)
    return math.sqrt(eh1), math.sqrt(el2)


def test_neumann_manufactured_solution_convergence():
    """Natural boundary: H1-seminorm error O(h) (slope >= 0.9), L2 O(h^2) (>= 1.7)."""
    errs = [_neumann_manufactured_errors(N) for N in (8, 16, 32)]
    s1 = [math.log2(errs[i][0] / errs[i + 1][0]) for i in range(2)]
    s2 = [math.log2(errs[i][1] / errs[i + 1][1]) for i in range(2)]
    assert min(s1) >= 0.9, (errs, s1)
    assert min(s2) >= 1.7, (errs, s2)


def test_block3d_rhs_is_the_back_substitution_of_twosteps():
    """b = -A01 A11^-1 f1: solving the block upper-triangular system
    [C A01; 0 A11] [u0; u1] = [0; f1] (eq. "twosteps") by a generic sparse LU
    gives u0 = C^-1 b; and the block-3D layout is [C 0; 0 I] with F = [b; 0]."""
    inst = _neumann(n_cells=8, radius=5e-3, k_omega=1e-3, sigma_omega=1e-3)
    s = fem.assemble(inst)
    A00, A01, A10, A11 = s.blocks()
    U = sp.bmat([[A00, A01], [None, A11]], format="csc")
    u = spla.spsolve(U, s.F)
    b = fem.block3d_rhs(s)
    assert np.linalg.norm(b) > 0
    u0 = spla.spsolve(A00.tocsc(), b)
    assert np.allclose(u[:s.n3d], u0, rtol=1e-10, atol=1e-12 * np.max(np.abs(u0)))
    inst.problem = "block3d"
    t = fem.assemble(inst)
    assert (abs(t.A[:t.n3d, :t.n3d] - A00)).max() == 0.0
    assert t.A[:t.n3d, t.n3d:].nnz == 0 and t.A[t.n3d:, :t.n3d].nnz == 0
    assert (abs(t.A[t.n3d:, t.n3d:] - sp.identity(t.n1d))).max() == 0.0
    assert np.array_equal(t.F[:t.n3d], b) and not np.any(t.F[t.n3d:])
    assert t.alpha == s.alpha
