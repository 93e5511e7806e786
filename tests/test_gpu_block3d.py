"""GPU parity of the paper's 3D-block workload (Section 5 setup): natural
(Neumann) boundary on the unit cube, k_Omega = sigma_Omega = 1e-3, vessel
radius eps = 1e-3, the 3D block C = K00 + 2 pi eps M00 solved alone with
b = -A01 A11^-1 f1 (eq. "matrixC", eq. "setB") by FGMRES(20) to relative
residual 1e-6, on 21^3 and 41^3 grids; every result against the FP64 oracle
(its own assembly, preconditioners and FGMRES), in the 2-norm and the max-norm.
"""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import cnn as ocnn
from oracle import fem, krylov

pytestmark = pytest.mark.gpu

STATE = -6


def _P():
    import paper_2505_08491_amd as P
    return P


@pytest.fixture(scope="module")
def ctx():
    c = _P().Context(0)
    yield c
    c.close()


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _theta(seed, bias=0.05):
    th = ocnn.init_params(seed)
    rng = np.random.default_rng(seed)
    off = 0
    for a, b in ocnn.layer_sizes():
        th[off + a:off + a + b] = rng.uniform(-bias, bias, b)
        off += a + b
    return th.astype(np.float32).astype(np.float64)


def _check(got, ref, tol, what):
    e2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    em = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert e2 <= tol and em <= tol, (what, e2, em)
    return e2, em


def _block3d_weights(n_cells):
    from paper_2505_08491_amd import weights as W
    path = os.path.join(os.path.dirname(W.default_path()), f"unet{n_cells}_block3d")
    if not os.path.exists(path + ".bin"):
        pytest.skip("weights for the 3D-block workload not present")
    return W.load(path)[0]


@pytest.mark.parametrize("n_cells", [20, 40])
@pytest.mark.parametrize("vec,tol", [("f64", 1e-13), ("f32", 2e-6)])
@pytest.mark.parametrize("problem", ["coupled", "block3d"])
def test_spmv_neumann_matches_oracle(ctx, n_cells, vec, tol, problem):
    """y = A x with the natural boundary (boundary rows and the boundary
    columns next to them carried by the coupling-row part), for the coupled
    Neumann system and the block-3D layout, against the oracle's A."""
    insts = synth.workload_block3d(n_cells, 2)
    for i in insts:
        i.problem = problem
    S = _P().System(ctx, insts, vec_dtype=vec)
    x = synth.fast_normal(3 + n_cells, S.ntot)
    td = torch.float64 if vec == "f64" else torch.float32
    xin = x if vec == "f64" else x.astype(np.float32).astype(np.float64)
    y = S.spmv(dev(x, td)).cpu().double().numpy()
    for k, inst in enumerate(insts):
        s = fem.assemble(inst)
        o0, o1 = S.offsets[k], S.offsets[k + 1]
        _check(y[o0:o1], s.A @ xin[o0:o1], tol, (problem, k))
        # the exported operator is the oracle's (pattern bit-exact)
        rp, col, val = S.export_csr(k)
        assert np.array_equal(rp, s.A.indptr) and np.array_equal(col, s.A.indices)
    S.free()


@pytest.mark.parametrize("vec,cnn_dtype,tol,n_cells", [("f64", "f32", 2e-5, 20), ("f32", "f32", 2e-5, 20),
                                                       ("f32", "bf16", 5e-2, 20), ("f32", "f32", 2e-5, 40),
                                                       ("f32", "bf16", 5e-2, 40)])
def test_neural_precond_block3d_matches_oracle(ctx, vec, cnn_dtype, tol, n_cells):
    """Q(v) on the block-3D layout: the identity 1D block, no extension term,
    and the network's 3D solve P(b) = ||b|| alpha^-1 U([b/||b||, d/||d||]) on
    every node (no Dirichlet rows), against the oracle's block preconditioner."""
    insts = synth.workload_block3d(n_cells, 2)
    S = _P().System(ctx, insts, vec_dtype=vec)
    th = _theta(31)
    S.set_preconditioner("neural", weights=th.astype(np.float32), cnn_dtype=cnn_dtype)
    net = lambda X: ocnn.forward(th, X)[0]
    v = synth.fast_normal(8, S.ntot)
    td = torch.float64 if vec == "f64" else torch.float32
    z = S.precond_apply(dev(v, td)).cpu().double().numpy()
    for k, inst in enumerate(insts):
        s = fem.assemble(inst)
        o0, o1 = S.offsets[k], S.offsets[k + 1]
        vk = v[o0:o1] if vec == "f64" else v[o0:o1].astype(np.float32).astype(np.float64)
        ref = krylov.BlockPreconditioner(s, krylov.p3d_neural(s, net))(vk)
        e2 = np.linalg.norm(z[o0:o1] - ref) / np.linalg.norm(ref)
        assert e2 <= tol, (k, e2)
        # the boundary nodes carry the network's values too
        bmask = fem.boundary_mask(n_cells)
        zb, rb = z[o0:o0 + s.n3d][bmask], ref[:s.n3d][bmask]
        assert np.linalg.norm(zb - rb) <= 2 * tol * np.linalg.norm(rb), k
    S.free()


def test_fgmres_block3d_fp64_matches_oracle(ctx):
    """FGMRES(20) to 1e-6 on C u0 = b with the diagonal of C as the 3D
    preconditioner, FP64 vectors: the same step count as the oracle's FGMRES
    on C alone, the same solution, the true residual on the oracle's C."""
    insts = synth.workload_block3d(20, 3)
    S = _P().System(ctx, insts, vec_dtype="f64")
    S.set_preconditioner("block_jacobi")
    x, st = S.solve(S.rhs(), restart=20, max_iters=1000, tol=1e-6)
    for k, inst in enumerate(insts):
        s = fem.assemble(inst)
        C = s.A[:s.n3d, :s.n3d].tocsr()
        b = s.F[:s.n3d]
        ref = krylov.fgmres(C, b, precond=krylov.p3d_jacobi(s), restart=20, tol=1e-6, max_iters=1000)
        o0 = S.offsets[k]
        u0 = x[o0:o0 + s.n3d]
        assert st[k]["converged"] and st[k]["iters"] == ref.iters, (k, st[k], ref.iters)
        assert np.linalg.norm(b - C @ u0) <= 1e-6 * np.linalg.norm(b)
        _check(u0, ref.x, 1e-8, k)
        assert not np.any(x[o0 + s.n3d:S.offsets[k + 1]])   # the 1D part stays zero
    S.free()


@pytest.mark.parametrize("n_cells,cnt", [(20, 8), (40, 4)])
def test_neural_fgmres_block3d_gain(ctx, n_cells, cnt):
    """The network trained on the GPU for this workload at the grid it is
    used on (21^3 or 41^3 nodes, Neumann, k = sigma = 1e-3; the paper's
    U3hf(21^3) and U3hf(41^3) rows): FGMRES(20) reaches 1e-6 on every
    instance (true residual recomputed on the oracle's C) with fewer than half
    the steps of FGMRES without a preconditioner."""
    w = _block3d_weights(n_cells)
    P = _P()
    res = {}
    if True:
        insts = synth.workload_block3d(n_cells, cnt)
        S = P.System(ctx, insts, vec_dtype="f32")
        b = S.rhs()
        iters = {}
        for name in ("neural", "none"):
            if name == "neural":
                S.set_preconditioner("neural", weights=w, cnn_dtype="bf16")
            else:
                S.set_preconditioner("none")
            x, st = S.solve(b, restart=20, max_iters=1000, tol=1e-6)
            iters[name] = [q["iters"] for q in st]
            if name == "neural":
                assert all(q["converged"] for q in st), st
                for k, inst in enumerate(insts):
                    s = fem.assemble(inst, with_distance=False)
                    C = s.A[:s.n3d, :s.n3d].tocsr()
                    bb = s.F[:s.n3d]
                    o0 = S.offsets[k]
                    u0 = x[o0:o0 + s.n3d]
                    assert np.linalg.norm(bb - C @ u0) <= 1.01e-6 * np.linalg.norm(bb), k
        res[n_cells] = {k: float(np.mean(v)) for k, v in iters.items()}
        print(f"{n_cells + 1}^3 FGMRES(20) mean steps to 1e-6:", res[n_cells], flush=True)
        assert res[n_cells]["neural"] < 0.5 * res[n_cells]["none"], res
        S.free()


def test_neumann_rejects_dirichlet_only_variants(ctx):
    """Smoothing and inner FGMRES steps are built for the Dirichlet condition:
    refused on a Neumann system; mixing boundary conditions in one system is refused."""
    P = _P()
    insts = synth.workload_block3d(20, 2)
    S = P.System(ctx, insts, vec_dtype="f32")
    S.set_preconditioner("neural", weights=_theta(2).astype(np.float32), cnn_dtype="bf16")
    with pytest.raises(P.MdnpError) as e:
        S.set_smoothing(1, 0.8)
    assert e.value.status == STATE
    with pytest.raises(P.MdnpError) as e:
        S.set_inner_steps(3)
    assert e.value.status == STATE
    S.free()
    mixed = [synth.workload_block3d(20, 1)[0], synth.make_instance(5, 20, n_segments=4, elems_per_segment=4)]
    with pytest.raises(P.MdnpError):
        P.System(ctx, mixed, vec_dtype="f32")


def test_loss_grad_neumann_matches_oracle(ctx):
    """Training objective on the block-3D workload: no entry is masked (every
    node is free), loss and gradient against the oracle's formula with C."""
    insts = synth.workload_block3d(20, 2)
    S = _P().System(ctx, insts, vec_dtype="f32")
    sy = [fem.assemble(i, with_distance=False) for i in insts]
    slots = np.array([1, 0, 1], dtype=np.int32)
    n3d = S.n3d
    rng = np.random.default_rng(4)
    r = np.stack([synth.fast_normal(40 + k, n3d) for k in range(len(slots))])
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    u = rng.normal(size=(len(slots), n3d))
    loss, du = S.loss_grad(dev(slots, torch.int32), dev(r, torch.float32), dev(u, torch.float32))
    loss, du = loss.cpu().numpy(), du.cpu().double().numpy()
    for k, i in enumerate(slots):
        s = sy[i]
        C = s.A[:s.n3d, :s.n3d].tocsr()
        uk = u[k].astype(np.float32).astype(np.float64)
        e = r[k].astype(np.float32) - (C @ uk) / s.alpha
        assert loss[k] == pytest.approx(float(e @ e), rel=1e-5)
        g = -2 * (C @ e) / s.alpha
        _check(du[k], g, 1e-5, k)
