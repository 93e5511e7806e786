"""Restarted (flexible) GMRES and the preconditioners of the method (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* FGMRES(m) with right preconditioning (Section 4: the flexible variant of
  Saad 1993, chosen because the neural preconditioner is nonlinear), written
  in its textbook form: Arnoldi by modified Gram-Schmidt, Givens rotations
  for the least-squares problem, restart every m steps, stop on the relative
  residual ||r|| / ||r_0|| with x_0 = 0 (Section 5.1 and Section 6 stopping
  rule).  GMRES with a fixed linear right preconditioner is the same loop.
* The block preconditioner Q of Section 2.2 (eq. "right-prec" and
  "twosteps"): an exact 1D solve with the lower diagonal block, then the 3D
  correction b0 - A01 z1 handed to a 3D solver P3D (eq. "decoupled_3d_problem").
* P3D choices: Jacobi (diag(A00)^-1), exact (A00^-1, pins only) and the
  neural operator (module `cnn`), optionally wrapped in damped-Jacobi pre-
  and post-smoothing (Section 5, "Effect of pre- and post-smoothing") or
  used as the preconditioner of a few inner FGMRES steps on A00 (Section 6).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    converged: bool
    rel_res: float                                       # true ||b - A x|| / ||b||
    history: list = field(default_factory=list)          # rho_j / ||b|| per Arnoldi step
    cycle_true: list = field(default_factory=list)       # true rel-res at each cycle start/end
    H: list = field(default_factory=list)                # Hessenberg columns per cycle (for pins)
    g: list = field(default_factory=list)                # rotated rhs per cycle
    V: list = field(default_factory=list)                # Arnoldi basis v_1..v_{j+1} per cycle (for pins)


def fgmres(A, b, precond=None, restart=30, tol=1e-8, max_iters=1000, x0=None,
           breakdown=1e-14, keep_arnoldi=False) -> GmresResult:
    """Right-preconditioned restarted FGMRES(m).

    A        : sparse matrix or callable v -> A v (float64)
    precond  : callable v -> z (may be nonlinear); None = identity
    Cycle: r = b - A x; if ||r|| <= tol ||b|| stop; v1 = r/||r||; g = ||r|| e1;
    for j = 1..m: z_j = P(v_j); w = A z_j; MGS against v_1..v_j; h_{j+1,j} = ||w||;
    apply the previous rotations to column j, form rotation j from
    (h_jj, h_{j+1,j}); rotate g; rho = |g_{j+1}|; stop the cycle on
    rho <= tol ||b||, on happy breakdown (h_{j+1,j} <= breakdown * ||A z_j||),
    or at j = m.  Then solve the triangular system R y = g and set
    x += Z y.  Iterations count Arnoldi steps (= preconditioner applications).
    """
    mv = A if callable(A) else (lambda v: A @ v)
    P = precond if precond is not None else (lambda v: v.copy())
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return GmresResult(x=np.zeros(n), iters=0, converged=True, rel_res=0.0)
    res = GmresResult(x=x, iters=0, converged=False, rel_res=np.inf)
    while True:
        r = b - mv(x)
        beta = float(np.linalg.norm(r))
        res.cycle_true.append(beta / bnorm)
        if beta <= tol * bnorm:
            res.converged = True
            break
        if res.iters >= max_iters:
            break
        m = restart
        Vb = np.zeros((m + 1, n))
        Zb = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        Vb[0] = r / beta
        jend = 0
        for j in range(m):
            Zb[j] = P(Vb[j])
            w = mv(Zb[j])
            wnorm0 = float(np.linalg.norm(w))
            for i in range(j + 1):          # modified Gram-Schmidt
                H[i, j] = float(np.dot(w, Vb[i]))
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):              # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = math.hypot(a, bb)
            cs[j], sn[j] = (1.0, 0.0) if den == 0.0 else (a / den, bb / den)
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            rho = abs(g[j + 1])
            res.iters += 1
            jend = j + 1
            res.history.append(rho / bnorm)
            hbreak = bb <= breakdown * wnorm0
            if rho <= tol * bnorm or hbreak or res.iters >= max_iters:
                break
            Vb[j + 1] = w / bb
        y = np.zeros(jend)
        for i in range(jend - 1, -1, -1):   # back substitution R y = g
            y[i] = (g[i] - H[i, i + 1:jend] @ y[i + 1:jend]) / H[i, i]
        x = x + Zb[:jend].T @ y
        if keep_arnoldi:
            res.H.append(H[:jend + 1, :jend].copy())
            res.g.append(g[:jend + 1].copy())
            res.V.append(Vb[:jend + 1].copy())
    res.x = x
    res.rel_res = float(np.linalg.norm(b - mv(x)) / bnorm)
    return res


def jacobi(A):
    """z = D^-1 v with D = diag(A)."""
    dinv = 1.0 / A.diagonal()
    return lambda v: dinv * v


class BlockPreconditioner:
    """Right block preconditioner of Section 2.2 (eq. "twosteps").

    Given v = [v0; v1]:  z1 = A11^-1 v1 (exact 1D solve);
                         b0 = v0 - A01 z1;
                         z0 = P3D(b0).
    A11 = K11 + 2 pi eps M11 and A01 = 2 pi eps M01 are the blocks of the
    assembled matrix.  The 1D solve is exact (the paper reports no difference
    between ILU and a direct solver there, Section 6).
    """

    def __init__(self, system, p3d):
        self.sys = system
        A00, A01, A10, A11 = system.blocks()
        self.A00, self.A01, self.A11 = A00, A01, A11
        self.lu11 = spla.splu(A11.tocsc())
        self.p3d = p3d
        self.m = system.n3d

    def solve_1d(self, v1):
        return self.lu11.solve(v1)

    def extension(self, v0, z1):
        return v0 - self.A01 @ z1

    def __call__(self, v):
        v0, v1 = v[:self.m], v[self.m:]
        z1 = self.solve_1d(v1)
        b0 = self.extension(v0, z1)
        z0 = self.p3d(b0)
        return np.concatenate([z0, z1])


def p3d_jacobi(system):
    """The method without the network: diag(A00)^-1 on the 3D block."""
    d = system.A.diagonal()[:system.n3d]
    return lambda b: b / d


def p3d_exact(system):
    A00 = system.blocks()[0]
    lu = spla.splu(A00.tocsc())
    return lambda b: lu.solve(b)


def distance_input(system):
    """The network's parameter channel: the distance field of the tree (Section
    2.1) scaled to unit Euclidean norm over the grid, the scale of the unit
    residual channel it is stacked with (the paper does not fix its scale)."""
    d = np.asarray(system.dist, dtype=np.float64)
    nd = float(np.linalg.norm(d))
    return d / nd if nd > 0.0 else d


def p3d_neural(system, net_apply):
    """P3D(b) = ||b|| alpha^-1 U([b / ||b||, d / ||d||]) with Dirichlet rows z = b.

    `net_apply(x2)` evaluates the U-net on a [n, n, n, 2] input and returns
    [n, n, n] (module `cnn`).  alpha is the RMS of diag(A00) over the free
    nodes (training normalisation of Section 5.1).  A zero b maps to zero.
    """
    n = system.n_cells + 1
    bnd = system.boundary
    d = distance_input(system).reshape(n, n, n)
    alpha = system.alpha

    def apply(b):
        s = float(np.linalg.norm(b))
        if s == 0.0:
            return np.zeros_like(b)
        X = np.stack([(b / s).reshape(n, n, n), d], axis=-1)
        U = net_apply(X).reshape(-1)
        z = (s / alpha) * U
        z[bnd] = b[bnd]
        return z
    return apply


def jacobi_sweeps(A, b, z, omega, sweeps):
    """`sweeps` damped Jacobi steps z <- z + omega D^-1 (b - A z), D = diag(A)
    (the relaxation S_J of Section 5, "Effect of pre- and post-smoothing")."""
    dinv = 1.0 / A.diagonal()
    for _ in range(sweeps):
        z = z + omega * dinv * (b - A @ z)
    return z


def p3d_smoothed(system, p3d, omega, sweeps):
    """P3D wrapped in Jacobi pre- and post-smoothing on A00 (Section 5,
    "Effect of pre- and post-smoothing"): `sweeps` relaxation steps on
    A00 z = b from z = 0, the correction z += P3D(b - A00 z) on the remaining
    residual, then `sweeps` relaxation steps from the corrected z.  The paper
    names the smoother S_J(A, r, x0, maxit) without its damping or step count;
    omega and sweeps are parameters here."""
    A00 = system.blocks()[0].tocsr()

    def apply(b):
        z = jacobi_sweeps(A00, b, np.zeros_like(b), omega, sweeps)
        z = z + p3d(b - A00 @ z)
        return jacobi_sweeps(A00, b, z, omega, sweeps)
    return apply


def p3d_inner_fgmres(system, p3d, steps):
    """The 3D solve of Section 6: `steps` FGMRES steps on A00 z = b from z = 0,
    right-preconditioned by P3D (the paper's P-FGMRES with the network as P).
    A zero b maps to zero."""
    A00 = system.blocks()[0].tocsr()

    def apply(b):
        if not np.any(b):
            return np.zeros_like(b)
        return fgmres(A00, b, precond=p3d, restart=steps, tol=0.0, max_iters=steps).x
    return apply


def stiffness_eigenvalues(n_cells, k_omega, sigma_omega):
    """Eigenvalues of the 3D stiffness-plus-mass block on the free nodes of the
    Dirichlet problem (the A00 block of eq. "mainsys" without the coupling
    term), as an [N-1, N-1, N-1] array over sine modes (a, b, c).

    On the uniform grid the trilinear element matrices are tensor products of
    the 1D P1 stiffness (1/h) [[1, -1], [-1, 1]] and mass (h/6) [[2, 1], [1, 2]],
    so the assembled block is k (K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1)
    + sigma M1 x M1 x M1 with the tridiagonal Toeplitz matrices
    K1 = (1/h) tridiag(-1, 2, -1) and M1 = (h/6) tridiag(1, 4, 1) on the N - 1
    interior nodes of each axis.  Both are diagonalised by the sine vectors
    sin(pi j m / N), with eigenvalues (1/h)(2 - 2 cos(pi m / N)) and
    (h/6)(4 + 2 cos(pi m / N)), m = 1 .. N - 1."""
    N = n_cells
    h = 1.0 / N
    c = np.cos(np.pi * np.arange(1, N) / N)
    K1 = (2.0 - 2.0 * c) / h
    M1 = (4.0 + 2.0 * c) * h / 6.0
    Ka, Kb, Kc = K1[:, None, None], K1[None, :, None], K1[None, None, :]
    Ma, Mb, Mc = M1[:, None, None], M1[None, :, None], M1[None, None, :]
    return k_omega * (Ka * Mb * Mc + Ma * Kb * Mc + Ma * Mb * Kc) + sigma_omega * Ma * Mb * Mc


def p3d_stiffness_inverse(system, k_omega=1.0, sigma_omega=0.0):
    """Exact inverse of the 3D block without its coupling term: Dirichlet rows
    return b, the free nodes solve the stiffness-plus-mass system by the
    orthonormal 3D sine transform (type I), which is its own inverse.  A test
    tool: as the 3D solve of the block preconditioner it makes the oracle's
    FGMRES reach the solution of the coupled system in a few dozen steps at
    any resolution (the coupling is a perturbation supported on the vessels)."""
    from scipy import fft
    N = system.n_cells
    n = N + 1
    lam = stiffness_eigenvalues(N, k_omega, sigma_omega)

    def apply(b):
        z = np.array(b, dtype=np.float64)
        g = z.reshape(n, n, n)
        inner = g[1:-1, 1:-1, 1:-1]
        g[1:-1, 1:-1, 1:-1] = fft.dstn(fft.dstn(inner, type=1, norm="ortho") / lam, type=1, norm="ortho")
        return z
    return apply


def reference_solution(system, tol=1e-12, restart=50, max_iters=3000, k_omega=1.0, sigma_omega=0.0):
    """x* = A^-1 F to true relative residual `tol`, for error checks at sizes
    where a sparse LU is too slow: the oracle's FGMRES with the block
    preconditioner of Section 2.2 whose 3D solve is `p3d_stiffness_inverse`.
    The preconditioner only sets the step count; the result is pinned by its
    FP64 true residual on the oracle's A.  Returns the GmresResult."""
    Q = BlockPreconditioner(system, p3d_stiffness_inverse(system, k_omega, sigma_omega))
    return fgmres(system.A, system.F, precond=Q, restart=restart, tol=tol, max_iters=max_iters)


def direct_solve(system):
    """x = A^-1 F by sparse LU (the plain definition of the solver's result)."""
    return spla.spsolve(system.A.tocsc(), system.F)
