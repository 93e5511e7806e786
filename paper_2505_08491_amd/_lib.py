"""ctypes loader of `libmdnp.so` and the C structures of `include/mdnp.h`.

The library must be built (``python -m paper_2505_08491_amd.build``); there is
no fallback: importing this module without the library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  -- loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdnp.so")

MDNP_OK, MDNP_E_ARG, MDNP_E_HIP, MDNP_E_OOM, MDNP_E_GEOM, MDNP_E_NONFINITE, MDNP_E_STATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "MDNP_OK", -1: "MDNP_E_ARG", -2: "MDNP_E_HIP", -3: "MDNP_E_OOM", -4: "MDNP_E_GEOM",
                -5: "MDNP_E_NONFINITE", -6: "MDNP_E_STATE"}
PREC = {"none": 0, "jacobi": 1, "neural": 2, "block_jacobi": 3}
DTYPE = {"f64": 0, "f32": 1, "bf16": 2, "fp8": 3, "fp8a": 4}


class InstanceDesc(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("k_omega", C.c_double), ("sigma_omega", C.c_double),
                ("n_vertices", C.c_int32), ("vertex_xyz", C.POINTER(C.c_double)),
                ("n_segments", C.c_int32), ("seg_vertices", C.POINTER(C.c_int32)),
                ("seg_radius", C.POINTER(C.c_double)), ("seg_beta", C.POINTER(C.c_double)),
                ("elems_per_segment", C.c_int32), ("k_lambda", C.c_double), ("f_lambda", C.c_double),
                ("n_circle", C.c_int32), ("boundary", C.c_int32), ("problem", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iters", C.c_int32), ("fallback_restart", C.c_int32),
                ("fallback_max_iters", C.c_int32), ("tol", C.c_double), ("record_history", C.c_int32),
                ("use_graph", C.c_int32)]


class InstStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("fallback_iters", C.c_int32), ("converged", C.c_int32),
                ("used_fallback", C.c_int32), ("final_rel_res", C.c_double)]


# exported symbols and their signatures (name, restype, argtypes)
VP = C.c_void_p
P = C.POINTER
SIGNATURES = [
    ("mdnp_create", C.c_int, [P(VP), C.c_int, VP]),
    ("mdnp_destroy", C.c_int, [VP]),
    ("mdnp_last_error", C.c_char_p, [VP]),
    ("mdnp_upload", C.c_int, [VP, P(InstanceDesc), C.c_int32, C.c_int, P(VP)]),
    ("mdnp_sys_free", C.c_int, [VP, VP]),
    ("mdnp_sys_sizes", C.c_int, [VP, C.c_int32, P(C.c_int32), P(C.c_int32), P(C.c_int64), P(C.c_int64)]),
    ("mdnp_sys_split_sizes", C.c_int, [VP, C.c_int32, P(C.c_int64), P(C.c_int64)]),
    ("mdnp_sys_coupling_sizes", C.c_int, [VP, C.c_int32, P(C.c_int64), P(C.c_int64), P(C.c_int64)]),
    ("mdnp_export_csr", C.c_int, [VP, C.c_int32, VP, VP, VP]),
    ("mdnp_export_rhs", C.c_int, [VP, C.c_int32, VP, VP, P(C.c_double)]),
    ("mdnp_set_preconditioner", C.c_int, [VP, VP, C.c_int, VP, C.c_int64, C.c_double, C.c_int]),
    ("mdnp_set_smoothing", C.c_int, [VP, VP, C.c_int32, C.c_double]),
    ("mdnp_set_inner_steps", C.c_int, [VP, VP, C.c_int32]),
    ("mdnp_autotune", C.c_int, [VP, VP, P(C.c_int32)]),
    ("mdnp_set_tuning", C.c_int, [VP, VP, P(C.c_int32)]),
    ("mdnp_cnn_layer_times", C.c_int, [VP, VP, C.c_int32, P(C.c_float)]),
    ("mdnp_solve", C.c_int, [VP, VP, VP, VP, P(SolveOpts), P(InstStats)]),
    ("mdnp_solve_device", C.c_int, [VP, VP, VP, VP, P(SolveOpts), P(InstStats), VP]),
    ("mdnp_history", C.c_int, [VP, C.c_int32, VP, C.c_int32, P(C.c_int32)]),
    ("mdnp_export_basis", C.c_int, [VP, VP, C.c_int32, VP, VP]),
    ("mdnp_spmv", C.c_int, [VP, VP, C.c_int32, VP, VP, C.c_int, VP]),
    ("mdnp_spmv_repeat", C.c_int, [VP, VP, VP, VP, C.c_int, C.c_int32, VP]),
    ("mdnp_tree_solve", C.c_int, [VP, VP, VP, VP, VP]),
    ("mdnp_precond_apply", C.c_int, [VP, VP, VP, VP, VP]),
    ("mdnp_set_fp8_scales", C.c_int, [VP, VP, VP, C.c_int32]),
    ("mdnp_get_fp8_scales", C.c_int, [VP, VP, VP, C.c_int32]),
    ("mdnp_fp8_calibrate", C.c_int, [VP, VP, VP, VP]),
    ("mdnp_cnn_forward", C.c_int, [VP, VP, VP, VP, VP, C.c_int32, C.c_int32, C.c_int, VP]),
    ("mdnp_cnn_saved_bytes", C.c_int64, [C.c_int32, C.c_int32, C.c_int]),
    ("mdnp_cnn_backward", C.c_int, [VP, VP, VP, VP, VP, VP, C.c_int32, C.c_int32, C.c_int, VP]),
    ("mdnp_loss_grad", C.c_int, [VP, VP, VP, C.c_int32, VP, VP, VP, VP, VP]),
    ("mdnp_loss_grad_noalloc", C.c_int, [VP, VP, VP, C.c_int32, VP, VP, VP, VP, VP]),
    ("mdnp_pack_input", C.c_int, [VP, VP, VP, C.c_int32, VP, VP, VP]),
    ("mdnp_adam_step", C.c_int, [VP, VP, VP, VP, VP, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                                 C.c_int32, VP]),
    ("mdnp_host_assemble", C.c_int, [P(InstanceDesc), P(VP), C.c_char_p, C.c_int32]),
    ("mdnp_host_sizes", C.c_int, [VP, P(C.c_int32), P(C.c_int32), P(C.c_int64), P(C.c_int32)]),
    ("mdnp_host_export", C.c_int, [VP, VP, VP, VP, VP, VP, P(C.c_double)]),
    ("mdnp_host_coupling_sizes", C.c_int, [VP, P(C.c_int32), P(C.c_int64), P(C.c_int64)]),
    ("mdnp_host_coupling", C.c_int, [VP, VP, VP, VP, VP, VP, VP, VP, VP]),
    ("mdnp_host_tree_solve", C.c_int, [VP, VP, VP]),
    ("mdnp_host_free", None, [VP]),
]


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_08491_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()
