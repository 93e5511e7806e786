"""Pins of the oracle FGMRES and block preconditioner (Sections 2.2 and 4)."""
import math
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import synth
from oracle import cnn, fem, krylov


def random_spd(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.normal(size=(n, n))
    return B @ B.T + n * np.eye(n)


@pytest.mark.parametrize("n", [4, 7, 20, 50])
def test_gmres_textbook_finite_termination(n):
    """P = I, m >= n: converges in at most n steps, to the dense solution."""
    A = random_spd(n, n)
    b = np.random.default_rng(1).normal(size=n)
    r = krylov.fgmres(sp.csr_matrix(A), b, restart=n, tol=1e-12, max_iters=n)
    assert r.converged and r.iters <= n
    assert np.allclose(r.x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)


def test_residual_estimate_equals_true_residual():
    """rho_j = |g_{j+1}| equals ||b - A x_j|| (x_j the j-step iterate) and is monotone."""
    A = random_spd(40, 3) + np.triu(np.random.default_rng(4).normal(size=(40, 40)), 1)  # non-symmetric
    b = np.random.default_rng(5).normal(size=40)
    full = krylov.fgmres(sp.csr_matrix(A), b, restart=25, tol=1e-30, max_iters=25)
    assert np.all(np.diff(full.history) <= 1e-15)
    for k in range(1, 25):
        part = krylov.fgmres(sp.csr_matrix(A), b, restart=k, tol=1e-30, max_iters=k)
        true = np.linalg.norm(b - A @ part.x) / np.linalg.norm(b)
        assert full.history[k - 1] == pytest.approx(true, rel=1e-9)


def test_exact_preconditioner_one_step():
    A = random_spd(30, 8)
    b = np.ones(30)
    Ainv = np.linalg.inv(A)
    r = krylov.fgmres(sp.csr_matrix(A), b, precond=lambda v: Ainv @ v, restart=10, tol=1e-12)
    assert r.iters == 1 and r.converged


def test_hessenberg_matches_arnoldi_relation():
    """Unrotated Arnoldi relation A Z_j = V_{j+1} H_j checked through a second,
    dense computation of the least-squares minimiser."""
    A = random_spd(25, 9) + 0.3 * np.random.default_rng(2).normal(size=(25, 25))
    b = np.random.default_rng(6).normal(size=25)
    D = np.diag(A).copy()
    r = krylov.fgmres(sp.csr_matrix(A), b, precond=lambda v: v / D, restart=8, tol=1e-30,
                      max_iters=8)
    # the 8-step iterate minimises ||b - A x|| over x in span(D^-1 K_8(A D^-1, b))
    Kb = [b / np.linalg.norm(b)]
    for _ in range(7):
        Kb.append(A @ (Kb[-1] / D))
        Kb[-1] /= np.linalg.norm(Kb[-1])
    Q, _ = np.linalg.qr(np.stack(Kb, axis=1))
    Zs = Q / D[:, None]
    y, *_ = np.linalg.lstsq(A @ Zs, b, rcond=None)
    assert np.allclose(r.x, Zs @ y, rtol=1e-8, atol=1e-10)


def _c1():
    return fem.assemble(synth.workload_single_fp64()[0])


def test_jacobi_gmres_c1_converges_to_direct_solution():
    s = _c1()
    r = krylov.fgmres(s.A, s.F, precond=krylov.jacobi(s.A), restart=50, tol=1e-8, max_iters=20000)
    assert r.converged and r.rel_res <= 1e-8
    xs = krylov.direct_solve(s)
    # error bounded by cond(A) * residual
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-5


def test_block_preconditioner_exact_blocks_spectrum():
    """With exact A00^-1 and A11^-1, A Q has eigenvalue 1 (multiplicity N3D) and the
    eigenvalues of S A11^-1 (S = A11 - A10 A00^-1 A01), all in (0, 1]; FGMRES then
    terminates in at most N1D + 1 steps."""
    inst = synth.make_instance(5, 8, n_segments=3, elems_per_segment=3, radius=0.02, beta=1.0)
    s = fem.assemble(inst)
    A00, A01, A10, A11 = (b.toarray() for b in s.blocks())
    Q = krylov.BlockPreconditioner(s, krylov.p3d_exact(s))
    n = s.n
    AQ = np.stack([s.A @ Q(e) for e in np.eye(n)], axis=1)
    ev = np.sort(np.linalg.eigvals(AQ).real)
    S = A11 - A10 @ np.linalg.solve(A00, A01)
    evS = np.sort(np.linalg.eigvals(S @ np.linalg.inv(A11)).real)
    assert evS.min() > 0 and evS.max() <= 1 + 1e-12
    expect = np.sort(np.concatenate([np.ones(s.n3d), evS]))
    assert np.allclose(ev, expect, atol=1e-9)
    r = krylov.fgmres(s.A, s.F, precond=Q, restart=s.n1d + 5, tol=1e-10, max_iters=s.n1d + 5)
    assert r.converged and r.iters <= s.n1d + 1


def test_fgmres_invariant_to_rescaled_preconditioner():
    """FGMRES iterates depend on span(Z) only: multiplying each z_j of a nonlinear
    (random-network) block preconditioner by a different positive factor leaves
    the residual history and the solution unchanged."""
    inst = synth.make_instance(3, 8, n_segments=4, elems_per_segment=3, radius=0.02, beta=1.0)
    s = fem.assemble(inst)
    theta = cnn.init_params(1)
    net = lambda X: cnn.forward(theta, X)[0]
    p1 = krylov.p3d_neural(s, net)
    Q1 = krylov.BlockPreconditioner(s, p1)
    scales = iter([7.3, 0.25, 3.0] * 20)
    Q2 = lambda v: next(scales) * Q1(v)
    r1 = krylov.fgmres(s.A, s.F, precond=Q1, restart=10, tol=1e-8, max_iters=30)
    r2 = krylov.fgmres(s.A, s.F, precond=Q2, restart=10, tol=1e-8, max_iters=30)
    assert r1.iters == r2.iters
    assert np.allclose(r1.history, r2.history, rtol=1e-7)
    assert np.allclose(r1.x, r2.x, rtol=1e-7, atol=1e-12)


def test_tree_solve_block_is_exact():
    s = _c1()
    A00, A01, A10, A11 = s.blocks()
    Q = krylov.BlockPreconditioner(s, krylov.p3d_jacobi(s))
    v1 = np.random.default_rng(0).normal(size=s.n1d)
    z = Q.solve_1d(v1)
    zd = np.linalg.solve(A11.toarray(), v1)
    assert np.linalg.norm(z - zd) / np.linalg.norm(zd) < 1e-13


def _smoothing_case():
    inst = synth.make_instance(5, 8, n_segments=3, elems_per_segment=3, radius=0.02, beta=1.0)
    s = fem.assemble(inst)
    A00 = s.blocks()[0].toarray()
    b = np.random.default_rng(11).normal(size=s.n3d)
    return s, A00, b


def test_smoothed_exact_inner_solve_stays_exact():
    """With P3D = A00^-1 the pre-smoothing error is removed exactly by the
    correction and post-smoothing leaves the exact solution in place."""
    s, A00, b = _smoothing_case()
    for omega, sweeps in [(0.8, 1), (0.6, 2), (1.0, 3)]:
        z = krylov.p3d_smoothed(s, krylov.p3d_exact(s), omega, sweeps)(b)
        zx = np.linalg.solve(A00, b)
        assert np.linalg.norm(z - zx) / np.linalg.norm(zx) < 1e-12


def test_smoothed_error_propagation():
    """For a linear inner preconditioner B the smoothed preconditioner P has
    error propagation I - P A00 = S^k (I - B A00) S^k with the relaxation
    matrix S = I - omega D^-1 A00 (k sweeps on each side); with B = 0 that is
    2 k plain relaxation steps from zero."""
    s, A00, b = _smoothing_case()
    n = A00.shape[0]
    I = np.eye(n)
    Dinv = np.diag(1.0 / np.diag(A00))
    Bj = Dinv.copy()
    for omega, k in [(0.8, 1), (0.6, 2)]:
        S = I - omega * Dinv @ A00
        Sk = np.linalg.matrix_power(S, k)
        for B, p3 in [(Bj, krylov.p3d_jacobi(s)), (np.zeros((n, n)), lambda r: np.zeros_like(r))]:
            E = Sk @ (I - B @ A00) @ Sk
            expect = (I - E) @ np.linalg.solve(A00, b)
            z = krylov.p3d_smoothed(s, p3, omega, k)(b)
            assert np.linalg.norm(z - expect) / np.linalg.norm(expect) < 1e-10


def test_smoothing_lowers_neural_iterations():
    """Jacobi smoothing around the trained network lowers the FGMRES step count
    on a 16^3 instance (the effect Section 5 reports)."""
    from paper_2505_08491_amd import weights as W
    import os
    if not os.path.exists(W.default_path() + ".bin"):
        pytest.skip("trained weights not present")
    theta = W.load(W.default_path())[0].astype(np.float64)
    inst = synth.make_instance(21, 16, n_segments=12, elems_per_segment=4, radius=0.008, beta=1.0)
    s = fem.assemble(inst)
    net = lambda X: cnn.forward(theta, X)[0]
    plain = krylov.BlockPreconditioner(s, krylov.p3d_neural(s, net))
    smooth = krylov.BlockPreconditioner(s, krylov.p3d_smoothed(s, krylov.p3d_neural(s, net), 0.8, 1))
    r0 = krylov.fgmres(s.A, s.F, precond=plain, restart=30, tol=1e-8, max_iters=300)
    r1 = krylov.fgmres(s.A, s.F, precond=smooth, restart=30, tol=1e-8, max_iters=300)
    assert r0.converged and r1.converged
    assert r1.iters < r0.iters


def test_inner_fgmres_with_exact_preconditioner_is_exact():
    """P-FGMRES with P = A00^-1 solves A00 z = b in its first step."""
    s, A00, b = _smoothing_case()
    z = krylov.p3d_inner_fgmres(s, krylov.p3d_exact(s), 3)(b)
    zx = np.linalg.solve(A00, b)
    assert np.linalg.norm(z - zx) / np.linalg.norm(zx) < 1e-11


def test_inner_fgmres_minimises_residual_over_its_directions():
    """After k steps from zero, z minimises ||b - A00 z|| over span{P(v_1) .. P(v_k)}
    (the directions the preconditioner returned), checked by a dense
    least-squares solve; with a nonlinear (random-network) P."""
    s, A00, b = _smoothing_case()
    theta = cnn.init_params(2)
    base = krylov.p3d_neural(s, lambda X: cnn.forward(theta, X)[0])
    Z = []

    def rec(v):
        z = base(v)
        Z.append(z)
        return z
    for k in (1, 3):
        Z.clear()
        z = krylov.p3d_inner_fgmres(s, rec, k)(b)
        Zm = np.stack(Z, axis=1)
        c, *_ = np.linalg.lstsq(A00 @ Zm, b, rcond=None)
        zs = Zm @ c
        assert len(Z) == k
        assert np.linalg.norm(z - zs) / np.linalg.norm(zs) < 1e-9
        assert np.linalg.norm(b - A00 @ z) <= np.linalg.norm(b) * (1 + 1e-12)


def test_distance_input_is_the_unit_norm_distance_field():
    s = _c1()
    d = krylov.distance_input(s)
    assert abs(np.linalg.norm(d) - 1.0) < 1e-12
    k = np.argmax(s.dist)
    assert np.allclose(d * (s.dist[k] / d[k]), s.dist, rtol=1e-12, atol=0)


def test_neural_3d_solve_scaling_and_dirichlet_rule():
    """P3D(b) = ||b|| alpha^-1 U([b/||b||, d/||d||]) with Dirichlet rows z = b
    (Section 4.1: the network sees unit-norm inputs; Section 5.1: alpha).  With
    stub networks that return one input channel, the result is fixed by hand:
    U = channel 0 gives z = b / alpha on the free rows; U = channel 1 gives
    ||b|| / alpha * d / ||d||; every Dirichlet row returns b whatever U is."""
    s = _c1()
    n = s.n_cells + 1
    bnd = s.boundary
    rng = np.random.default_rng(21)
    b = rng.normal(size=s.n3d)
    dg = s.A.diagonal()[:s.n3d][~bnd]
    alpha = math.sqrt(float(np.sum(dg * dg)) / dg.size)
    z = krylov.p3d_neural(s, lambda X: X[..., 0])(b)
    assert np.allclose(z[~bnd], b[~bnd] / alpha, rtol=1e-13, atol=0)
    assert np.array_equal(z[bnd], b[bnd])
    z = krylov.p3d_neural(s, lambda X: X[..., 1])(b)
    d = np.asarray(s.dist, dtype=np.float64)
    expect = np.linalg.norm(b) / alpha * d / np.linalg.norm(d)
    assert np.allclose(z[~bnd], expect[~bnd], rtol=1e-13, atol=0)
    assert np.array_equal(z[bnd], b[bnd])
    # the input tensor is laid out [z][y][x][channel] on the n^3 grid
    seen = {}

    def spy(X):
        seen["X"] = X.copy()
        return np.zeros(X.shape[:3])
    z = krylov.p3d_neural(s, spy)(b)
    assert seen["X"].shape == (n, n, n, 2)
    assert np.allclose(seen["X"][..., 0].ravel(), b / np.linalg.norm(b), rtol=1e-15, atol=0)
    assert np.all(z[~bnd] == 0.0)
    # zero input maps to zero without calling the network
    assert not np.any(krylov.p3d_neural(s, lambda X: 1 / 0)(np.zeros(s.n3d)))


def test_neural_3d_solve_positively_homogeneous():
    """For the real (nonlinear) network P3D(c b) = c P3D(b) for c > 0: the
    input is normalised and the output rescaled by ||b||."""
    s = _c1()
    theta = cnn.init_params(4)
    p = krylov.p3d_neural(s, lambda X: cnn.forward(theta, X)[0])
    b = np.random.default_rng(22).normal(size=s.n3d)
    z1 = p(b)
    for c in (1e-6, 0.37, 250.0):
        assert np.allclose(p(c * b), c * z1, rtol=1e-12, atol=0)
    # not odd: the network is not linear, so P(-b) differs from -P(b)
    assert np.linalg.norm(p(-b) + z1) > 1e-3 * np.linalg.norm(z1)


@pytest.mark.parametrize("k_omega,sigma", [(1.0, 0.0), (1.7, 25.0)])
def test_stiffness_eigenvalues_match_dense(k_omega, sigma):
    """The sine-mode eigenvalues of the free-node 3D block (no coupling)
    against a dense symmetric eigensolver on a 6^3 grid."""
    inst = synth.make_instance(3, 6, n_segments=2, elems_per_segment=2, radius=0.02, beta=0.0,
                               k_omega=k_omega, sigma_omega=sigma)
    s = fem.assemble(inst)
    A00 = s.blocks()[0].toarray()
    free = ~s.boundary
    ev = np.sort(np.linalg.eigvalsh(A00[np.ix_(free, free)]))
    lam = np.sort(krylov.stiffness_eigenvalues(6, k_omega, sigma).ravel())
    assert np.allclose(lam, ev, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("N,k_omega,sigma", [(8, 1.0, 0.0), (12, 2.0, 7.0)])
def test_stiffness_inverse_solves_uncoupled_block(N, k_omega, sigma):
    """With beta = 0 the 3D block is the stiffness-plus-mass matrix alone and
    the sine-transform solve is its exact inverse: A00 z = b to rounding, equal
    to a sparse LU solve, and the identity on the Dirichlet rows."""
    inst = synth.make_instance(5, N, n_segments=3, elems_per_segment=3, radius=0.02, beta=0.0,
                               k_omega=k_omega, sigma_omega=sigma)
    s = fem.assemble(inst)
    A00 = s.blocks()[0].tocsc()
    b = np.random.default_rng(N).normal(size=s.n3d)
    z = krylov.p3d_stiffness_inverse(s, k_omega, sigma)(b)
    assert np.linalg.norm(A00 @ z - b) <= 1e-12 * np.linalg.norm(b)
    zd = spla_solve(A00, b)
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)
    assert np.array_equal(z[s.boundary], b[s.boundary])


def spla_solve(A, b):
    import scipy.sparse.linalg as spla
    return spla.spsolve(A, b)


def test_reference_solution_equals_direct_solve():
    """The reference solution (FGMRES with the stiffness-inverse block
    preconditioner, tol 1e-13) equals the sparse LU solution of the coupled
    system within 1e-11 on a 12^3 instance with strong coupling, in few steps."""
    inst = synth.make_instance(8, 12, n_segments=9, elems_per_segment=3, radius=0.02, beta=2.0)
    s = fem.assemble(inst)
    r = krylov.reference_solution(s, tol=1e-13)
    xd = krylov.direct_solve(s)
    assert r.converged and r.iters <= 40
    assert np.linalg.norm(r.x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_reference_pool_reports_errors():
    """The per-instance error helper on two worker processes: the direct
    solution has error ~1e-12 and residual ~1e-13; a perturbed one reports the
    perturbation it carries, in both norms."""
    from oracle import reference
    insts = [synth.make_instance(30 + i, 8, n_segments=3 + i, elems_per_segment=3, radius=0.02, beta=1.0)
             for i in range(2)]
    xd = [krylov.direct_solve(fem.assemble(i)) for i in insts]
    bad = [x.copy() for x in xd]
    for x in bad:
        x[3] += 1e-3 * np.max(np.abs(x))
    res = reference.errors_vs_oracle(insts, [[x, y] for x, y in zip(xd, bad)], workers=2)
    for r, x in zip(res, xd):
        assert r["ref_converged"] and r["ref_rel_res"] <= 1e-12
        good, off = r["cands"]
        assert good["rel_res"] <= 1e-12 and good["err"] <= 1e-10 and good["err_max"] <= 1e-10
        assert off["err_max"] == pytest.approx(1e-3, rel=1e-6)
        assert off["err"] == pytest.approx(1e-3 * np.max(np.abs(x)) / np.linalg.norm(x), rel=1e-6)


def test_block3d_layout_runs_fgmres_on_c_alone():
    """FGMRES on the block-3D layout [C 0; 0 I] [u0; u1] = [b; 0] with the block
    preconditioner (exact solve of the identity block, no extension term)
    takes the same steps as FGMRES on C u0 = b with the 3D preconditioner
    alone (Section 5 setup: FGMRES(20) to 1e-6): same step count, same
    history, same u0, and u1 stays zero."""
    inst = synth.make_instance(5, 8, n_segments=5, elems_per_segment=3, radius=1e-3, beta=1.0, k_omega=1e-3,
                               sigma_omega=1e-3, boundary="neumann", problem="block3d")
    t = fem.assemble(inst)
    C = t.A[:t.n3d, :t.n3d].tocsr()
    b = t.F[:t.n3d]
    p3d = krylov.p3d_jacobi(t)
    ref = krylov.fgmres(C, b, precond=p3d, restart=20, tol=1e-6, max_iters=1000)
    got = krylov.fgmres(t.A, t.F, precond=krylov.BlockPreconditioner(t, p3d), restart=20, tol=1e-6,
                        max_iters=1000)
    assert ref.converged and got.converged and got.iters == ref.iters
    assert np.allclose(got.history, ref.history, rtol=1e-9, atol=0)
    assert np.allclose(got.x[:t.n3d], ref.x, rtol=1e-9, atol=1e-12 * np.max(np.abs(ref.x)))
    assert not np.any(got.x[t.n3d:])
