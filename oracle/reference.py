"""Reference solutions x* = A^-1 F and the error of given solutions against
them, one instance per CPU process (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For each instance a worker assembles the oracle's own system (Section 2.1,
eq. "mainsys"), computes x* to FP64 true relative residual `tol` with
`krylov.reference_solution` and, for every candidate solution x given with the
instance, reports
  rel_res  ||F - A x|| / ||F|| on the oracle's A,
  err      ||x - x*|| / ||x*||,
  err_max  max |x - x*| / max |x*|.
Workers are processes started with "spawn", one BLAS thread each, so the
caller may already hold a GPU context.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


def _worker(args):
    inst, cands, tol = args
    from oracle import fem, krylov
    s = fem.assemble(inst, with_distance=False)
    ref = krylov.reference_solution(s, tol=tol, k_omega=inst.k_omega, sigma_omega=inst.sigma_omega)
    xs = ref.x
    F = s.F
    out = {"ref_iters": ref.iters, "ref_rel_res": ref.rel_res, "ref_converged": bool(ref.converged), "n": s.n,
           "cands": []}
    for x in cands:
        x = np.asarray(x, dtype=np.float64)
        out["cands"].append({"rel_res": float(np.linalg.norm(F - s.A @ x) / np.linalg.norm(F)),
                             "err": float(np.linalg.norm(x - xs) / np.linalg.norm(xs)),
                             "err_max": float(np.max(np.abs(x - xs)) / np.max(np.abs(xs)))})
    return out


def pool_size(count: int, cap: int = 16) -> int:
    """Workers for `count` instances: at most `cap` and the host's CPU count."""
    return max(1, min(cap, count, os.cpu_count() or 1))


def errors_vs_oracle(instances, candidates, tol=1e-12, workers=None):
    """candidates[i] is a list of FP64 solution vectors of instance i (may be
    empty); returns one dict per instance (see the module docstring)."""
    jobs = [(inst, list(c), tol) for inst, c in zip(instances, candidates)]
    workers = pool_size(len(jobs)) if workers is None else workers
    if workers == 1:
        return [_worker(j) for j in jobs]
    names = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    keep = {k: os.environ.get(k) for k in names}
    for k in names:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            return pool.map(_worker, jobs, chunksize=1)
    finally:
        for k, v in keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
