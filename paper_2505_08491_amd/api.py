"""Python binding of the C ABI (argument marshalling only).

Every step of the solve runs in the HIP library; torch tensors are used only
as device buffers and streams.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import DTYPE, PREC, STATUS_NAMES, InstanceDesc, InstStats, SolveOpts, lib

N_WEIGHTS = 353713


class MdnpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    return C.c_void_p(stream.cuda_stream)


def _desc(inst, keep: list) -> InstanceDesc:
    """Build the C descriptor of one instance (any object with the fields of
    `synth.Instance`); arrays are kept alive in `keep`."""
    v = np.ascontiguousarray(inst.vertex_xyz, dtype=np.float64)
    s = np.ascontiguousarray(inst.seg, dtype=np.int32)
    r = np.ascontiguousarray(inst.radius, dtype=np.float64)
    b = np.ascontiguousarray(inst.beta, dtype=np.float64)
    keep += [v, s, r, b]
    d = InstanceDesc()
    d.n_cells = int(inst.n_cells)
    d.k_omega = float(inst.k_omega)
    d.sigma_omega = float(inst.sigma_omega)
    d.n_vertices = int(v.shape[0])
    d.vertex_xyz = v.ctypes.data_as(C.POINTER(C.c_double))
    d.n_segments = int(s.shape[0])
    d.seg_vertices = s.ctypes.data_as(C.POINTER(C.c_int32))
    d.seg_radius = r.ctypes.data_as(C.POINTER(C.c_double))
    d.seg_beta = b.ctypes.data_as(C.POINTER(C.c_double))
    d.elems_per_segment = int(inst.elems_per_segment)
    d.k_lambda = float(inst.k_lambda)
    d.f_lambda = float(inst.f_lambda)
    d.n_circle = int(inst.n_circle)
    d.boundary = {"dirichlet": 0, "neumann": 1}[getattr(inst, "boundary", "dirichlet")]
    d.problem = {"coupled": 0, "block3d": 1}[getattr(inst, "problem", "coupled")]
    return d


# ---------------------------------------------------------------- host-only assembly

@dataclass
class HostSystem:
    n3d: int
    n1d: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    F: np.ndarray
    dist: np.ndarray
    alpha: float
    n_levels: int
    _handle: C.c_void_p = None

    def tree_solve(self, v1: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(v1, dtype=np.float64)
        z = np.empty_like(v)
        st = lib.mdnp_host_tree_solve(self._handle, v.ctypes.data, z.ctypes.data)
        if st != 0:
            raise MdnpError(st, "host tree solve failed")
        return z

    def coupling(self):
        """The factored coupling M = B^T W B + R of this assembly as SciPy CSR
        matrices (B: one row per Gauss point, columns over all n3d + n1d
        unknowns), the weights W and, per Gauss point, where its 1D entries
        start in B's entry arrays."""
        import scipy.sparse as sp
        nq, nb, nr = C.c_int32(), C.c_int64(), C.c_int64()
        lib.mdnp_host_coupling_sizes(self._handle, C.byref(nq), C.byref(nb), C.byref(nr))
        n = self.n3d + self.n1d
        bp = np.empty(nq.value + 1, np.int32)
        bs = np.empty(nq.value, np.int32)
        bc = np.empty(nb.value, np.int32)
        bv = np.empty(nb.value, np.float64)
        w = np.empty(nq.value, np.float64)
        rp = np.empty(n + 1, np.int32)
        rc = np.empty(nr.value, np.int32)
        rv = np.empty(nr.value, np.float64)
        st = lib.mdnp_host_coupling(self._handle, bp.ctypes.data, bs.ctypes.data, bc.ctypes.data, bv.ctypes.data,
                                    w.ctypes.data, rp.ctypes.data, rc.ctypes.data, rv.ctypes.data)
        if st != 0:
            raise MdnpError(st, "host coupling export failed")
        B = sp.csr_matrix((bv, bc, bp), shape=(nq.value, n))
        R = sp.csr_matrix((rv, rc, rp), shape=(n, n))
        return B, w, R, bs

    def __del__(self):
        if self._handle is not None and lib is not None:
            lib.mdnp_host_free(self._handle)
            self._handle = None


def host_assemble(inst) -> HostSystem:
    """Assemble one instance on the host (no GPU touched)."""
    keep: list = []
    d = _desc(inst, keep)
    h = C.c_void_p()
    err = C.create_string_buffer(512)
    st = lib.mdnp_host_assemble(C.byref(d), C.byref(h), err, 512)
    if st != 0:
        raise MdnpError(st, err.value.decode())
    n3d, n1d, nlev = C.c_int32(), C.c_int32(), C.c_int32()
    nnz = C.c_int64()
    lib.mdnp_host_sizes(h, C.byref(n3d), C.byref(n1d), C.byref(nnz), C.byref(nlev))
    n = n3d.value + n1d.value
    rp = np.empty(n + 1, np.int32)
    col = np.empty(nnz.value, np.int32)
    val = np.empty(nnz.value, np.float64)
    F = np.empty(n, np.float64)
    dist = np.empty(n3d.value, np.float32)
    alpha = C.c_double()
    lib.mdnp_host_export(h, rp.ctypes.data, col.ctypes.data, val.ctypes.data, F.ctypes.data, dist.ctypes.data,
                         C.byref(alpha))
    return HostSystem(n3d.value, n1d.value, rp, col, val, F, dist, alpha.value, nlev.value, h)


# ---------------------------------------------------------------- device API

class Context:
    """A library context on one GPU (HIP device index).

    The library works on its own (non-default, default-priority) torch stream;
    every device call is ordered after the caller's current stream and the
    caller's stream waits for it afterwards, so torch tensors can be passed
    freely.
    """

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        h = C.c_void_p()
        self._check(lib.mdnp_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream)), None)
        self.h = h

    def run(self, fn, *args):
        """Call a library entry point on the context stream, in order with torch."""
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        st = fn(*args)
        cur.wait_stream(self.stream)
        self._check(st)

    def _check(self, st, h="self"):
        if st != 0:
            handle = self.h if h == "self" else h
            msg = lib.mdnp_last_error(handle).decode() if handle is not None else ""
            raise MdnpError(st, msg)

    def close(self):
        if getattr(self, "h", None) is not None:
            lib.mdnp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # stand-alone network calls ------------------------------------------------
    def cnn_forward(self, w: torch.Tensor, x: torch.Tensor, n: int, dtype: str = "f32",
                    saved: torch.Tensor | None = None) -> torch.Tensor:
        batch = x.shape[0]
        y = torch.empty(batch, n ** 3, device=x.device, dtype=torch.float32)
        self.run(lib.mdnp_cnn_forward, self.h, _ptr(w), _ptr(x), _ptr(y), _ptr(saved), batch, n, DTYPE[dtype],
                 _stream(self.stream))
        return y

    def saved_bytes(self, batch: int, n: int, dtype: str = "f32") -> int:
        return int(lib.mdnp_cnn_saved_bytes(batch, n, DTYPE[dtype]))

    def cnn_backward(self, w, saved, dy, batch, n, dtype="f32", want_dx=False):
        dw = torch.empty(N_WEIGHTS, device=dy.device, dtype=torch.float32)
        dx = torch.empty(batch, n ** 3, 2, device=dy.device, dtype=torch.float32) if want_dx else None
        self.run(lib.mdnp_cnn_backward, self.h, _ptr(w), _ptr(saved), _ptr(dy), _ptr(dx), _ptr(dw), batch, n,
                 DTYPE[dtype], _stream(self.stream))
        return dw, dx

    def adam_step(self, w, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
        self.run(lib.mdnp_adam_step, self.h, _ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), lr, b1, b2, eps,
                 step, _stream(self.stream))


class System:
    """A batch of instances uploaded to the GPU (Section 2.1 assembly on the host)."""

    def __init__(self, ctx: Context, instances, vec_dtype: str = "f32"):
        self.ctx = ctx
        keep: list = []
        arr = (InstanceDesc * len(instances))(*[_desc(i, keep) for i in instances])
        h = C.c_void_p()
        ctx._check(lib.mdnp_upload(ctx.h, arr, len(instances), DTYPE[vec_dtype], C.byref(h)))
        self.h = h
        self.n_inst = len(instances)
        self.vec_dtype = vec_dtype
        self.torch_dtype = torch.float64 if vec_dtype == "f64" else torch.float32
        self.n_cells = instances[0].n_cells
        self.n = self.n_cells + 1
        self.sizes = [self._sizes(i) for i in range(self.n_inst)]
        self.n3d = self.sizes[0][0]
        self.offsets = [s[3] for s in self.sizes] + [self.sizes[-1][3] + self.sizes[-1][0] + self.sizes[-1][1]]
        self.ntot = self.offsets[-1]

    def _sizes(self, i):
        a, b, c, d = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        self.ctx._check(lib.mdnp_sys_sizes(self.h, i, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return a.value, b.value, c.value, d.value

    def split_sizes(self, i):
        """(entries, non-empty rows) of the coupling part M of A = S + M."""
        a, b = C.c_int64(), C.c_int64()
        self.ctx._check(lib.mdnp_sys_split_sizes(self.h, i, C.byref(a), C.byref(b)))
        return a.value, b.value

    def coupling_sizes(self, i):
        """(Gauss points, entries of W B, entries of B^T | R) of the factored
        coupling M = B^T W B + R that the stencil-sweep path applies."""
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self.ctx._check(lib.mdnp_sys_coupling_sizes(self.h, i, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def free(self):
        if getattr(self, "h", None) is not None and self.ctx.h is not None:
            lib.mdnp_sys_free(self.ctx.h, self.h)
            self.h = None

    def export_csr(self, i):
        n3d, n1d, nnz, _ = self.sizes[i]
        rp = np.empty(n3d + n1d + 1, np.int32)
        col = np.empty(nnz, np.int32)
        val = np.empty(nnz, np.float64)
        self.ctx._check(lib.mdnp_export_csr(self.h, i, rp.ctypes.data, col.ctypes.data, val.ctypes.data))
        return rp, col, val

    def export_rhs(self, i):
        n3d, n1d, _, _ = self.sizes[i]
        F = np.empty(n3d + n1d)
        d = np.empty(n3d)
        a = C.c_double()
        self.ctx._check(lib.mdnp_export_rhs(self.h, i, F.ctypes.data, d.ctypes.data, C.byref(a)))
        return F, d, a.value

    def rhs(self) -> np.ndarray:
        return np.concatenate([self.export_rhs(i)[0] for i in range(self.n_inst)])

    def set_preconditioner(self, kind: str, weights=None, alpha: float = 0.0, cnn_dtype: str = "f32"):
        w = None
        n = 0
        if weights is not None:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
            n = w.size
        self.ctx._check(lib.mdnp_set_preconditioner(self.ctx.h, self.h, PREC[kind],
                                                    w.ctypes.data if w is not None else None, n, alpha,
                                                    DTYPE[cnn_dtype]))

    def set_fp8_scales(self, scales):
        """Activation scales of the cnn_dtype "fp8a" network (X, L0a, L0b, L1a,
        L1b, L2a, L2b, U1, D1, U0, D0; powers of two)."""
        a = np.ascontiguousarray(np.asarray(scales, dtype=np.float32))
        self.ctx._check(lib.mdnp_set_fp8_scales(self.ctx.h, self.h, a.ctypes.data, a.size))

    def fp8_scales(self):
        out = (C.c_float * 11)()
        self.ctx._check(lib.mdnp_get_fp8_scales(self.ctx.h, self.h, out, 11))
        return list(out)

    def fp8_calibrate(self, v: torch.Tensor):
        """Set the "fp8a" activation scales from the FP32 network on the
        preconditioner input of v (a device vector of the system's type)."""
        self.ctx.run(lib.mdnp_fp8_calibrate, self.ctx.h, self.h, _ptr(v), _stream(self.ctx.stream))
        return self.fp8_scales()

    def autotune(self):
        """Time and fix the launch shapes: the z split / M blocks of each BF16
        layer ([0..10], by layer), the SpMV stencil sweep's z split ([11]) and
        the output rows of L1b, D1, L0b, D0 ([12..15]), the workgroups of
        U1, U0 ([16], [17]) and the x blocks per workgroup of L0a, L0b, L1b,
        D1, D0 ([18..22])."""
        out = (C.c_int32 * 23)()
        self.ctx._check(lib.mdnp_autotune(self.ctx.h, self.h, out))
        return list(out)

    def set_tuning(self, chosen):
        """Set the launch shapes in the layout `autotune` returns."""
        arr = (C.c_int32 * 23)(*[int(v) for v in chosen])
        self.ctx._check(lib.mdnp_set_tuning(self.ctx.h, self.h, arr))

    def layer_times(self, reps: int = 5):
        """Average milliseconds of each stage of the in-solver network
        application (L0a, L0b, L1a, L1b, L2a, L2b, U1, D1, U0, D0 + head),
        HIP events on the library stream."""
        out = (C.c_float * 10)()
        self.ctx._check(lib.mdnp_cnn_layer_times(self.ctx.h, self.h, int(reps), out))
        return list(out)

    def set_inner_steps(self, steps: int):
        """Inner FGMRES(steps) 3D solve with the network as preconditioner (0: off)."""
        self.ctx._check(lib.mdnp_set_inner_steps(self.ctx.h, self.h, int(steps)))

    def set_smoothing(self, sweeps: int, omega: float = 0.8):
        """Jacobi pre/post-smoothing of the neural 3D solve (0 sweeps: off)."""
        self.ctx._check(lib.mdnp_set_smoothing(self.ctx.h, self.h, int(sweeps), float(omega)))

    @staticmethod
    def opts(restart=30, max_iters=1000, fallback_restart=50, fallback_max_iters=0, tol=1e-8, history=True,
             use_graph=False) -> SolveOpts:
        o = SolveOpts()
        o.restart, o.max_iters, o.fallback_restart, o.fallback_max_iters = restart, max_iters, fallback_restart, \
            fallback_max_iters
        o.tol, o.record_history, o.use_graph = tol, int(history), int(use_graph)
        return o

    def solve(self, b: np.ndarray, x0: np.ndarray | None = None, **kw):
        """Host solve: returns (x, stats list)."""
        o = self.opts(**kw)
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
        stats = (InstStats * self.n_inst)()
        self.ctx._check(lib.mdnp_solve(self.ctx.h, self.h, b.ctypes.data, x.ctypes.data, C.byref(o), stats))
        return x, [self._stat(s) for s in stats]

    def solve_device(self, d_b: torch.Tensor, d_x: torch.Tensor, **kw):
        o = self.opts(**kw)
        stats = (InstStats * self.n_inst)()
        self.ctx.run(lib.mdnp_solve_device, self.ctx.h, self.h, _ptr(d_b), _ptr(d_x), C.byref(o), stats,
                     _stream(self.ctx.stream))
        return [self._stat(s) for s in stats]

    @staticmethod
    def _stat(s):
        return {"iters": s.iters, "fallback_iters": s.fallback_iters, "converged": bool(s.converged),
                "used_fallback": bool(s.used_fallback), "final_rel_res": s.final_rel_res}

    def history(self, i):
        n = C.c_int32()
        self.ctx._check(lib.mdnp_history(self.h, i, None, 0, C.byref(n)))
        out = np.empty(n.value)
        self.ctx._check(lib.mdnp_history(self.h, i, out.ctypes.data, n.value, C.byref(n)))
        return out

    def export_basis(self, k: int) -> torch.Tensor:
        out = torch.empty(self.ntot, device="cuda", dtype=self.torch_dtype)
        self.ctx.run(lib.mdnp_export_basis, self.ctx.h, self.h, k, _ptr(out), _stream(self.ctx.stream))
        return out

    # path steps on device tensors ----------------------------------------------
    def spmv(self, x: torch.Tensor, block: int = 0) -> torch.Tensor:
        y = torch.empty_like(x)
        dt = "f64" if x.dtype == torch.float64 else "f32"
        self.ctx.run(lib.mdnp_spmv, self.ctx.h, self.h, block, _ptr(x), _ptr(y), DTYPE[dt], _stream(self.ctx.stream))
        return y

    def spmv_repeat(self, x: torch.Tensor, y: torch.Tensor, reps: int):
        """y = A x launched `reps` times back to back (kernel timing)."""
        dt = "f64" if x.dtype == torch.float64 else "f32"
        self.ctx.run(lib.mdnp_spmv_repeat, self.ctx.h, self.h, _ptr(x), _ptr(y), DTYPE[dt], int(reps),
                     _stream(self.ctx.stream))

    def tree_solve(self, v: torch.Tensor, z: torch.Tensor | None = None) -> torch.Tensor:
        z = torch.zeros_like(v) if z is None else z
        self.ctx.run(lib.mdnp_tree_solve, self.ctx.h, self.h, _ptr(v), _ptr(z), _stream(self.ctx.stream))
        return z

    def precond_apply(self, v: torch.Tensor) -> torch.Tensor:
        z = torch.zeros_like(v)
        self.ctx.run(lib.mdnp_precond_apply, self.ctx.h, self.h, _ptr(v), _ptr(z), _stream(self.ctx.stream))
        return z

    def loss_grad(self, inst: torch.Tensor, r: torch.Tensor, u: torch.Tensor):
        du = torch.empty_like(u)
        loss = torch.empty(inst.numel(), device=u.device, dtype=torch.float64)
        self.ctx.run(lib.mdnp_loss_grad, self.ctx.h, self.h, _ptr(inst), inst.numel(), _ptr(r), _ptr(u), _ptr(du),
                     _ptr(loss), _stream(self.ctx.stream))
        return loss, du

    def loss_grad_noalloc(self, inst: torch.Tensor, r: torch.Tensor, u: torch.Tensor, du: torch.Tensor,
                          loss: torch.Tensor):
        """`loss_grad` into caller-owned du and loss, with the library's fixed
        workspace (no device allocation in the library)."""
        self.ctx.run(lib.mdnp_loss_grad_noalloc, self.ctx.h, self.h, _ptr(inst), inst.numel(), _ptr(r), _ptr(u),
                     _ptr(du), _ptr(loss), _stream(self.ctx.stream))

    def pack_input(self, inst: torch.Tensor, r: torch.Tensor) -> torch.Tensor:
        x = torch.empty(inst.numel(), self.n3d, 2, device=r.device, dtype=torch.float32)
        self.ctx.run(lib.mdnp_pack_input, self.ctx.h, self.h, _ptr(inst), inst.numel(), _ptr(r), _ptr(x),
                     _stream(self.ctx.stream))
        return x

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
