"""Benchmark: batched solves/s to true relative residual 1e-8 at 64^3 cells,
neural-preconditioned FGMRES(30) vs Jacobi-preconditioned GMRES(50), on one GPU.

One step = one batched solve of all instances of the workload (16 seeded random
trees of 512 segments x 16 P1 elements, R = 0.002, 64^3 trilinear cells, 16 x
282,818 unknowns), with b and x0 resident in HBM: every row of the hot path
(true residual, 1D tree solve, extension, U-net, unscaling, SpMV, modified
Gram-Schmidt, Givens, cycle end) runs inside it.

Prints one JSON line (see the keys below).  `--gpus N` with N > 1 is refused:
the instances would shard over GPUs with no per-iteration communication, but
this build measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BF16_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-cells", type=int, default=64)
    ap.add_argument("--count", type=int, default=None, help="instances (default 16 at 64^3, 2 at 128^3, 256 batched)")
    ap.add_argument("--workload", default="transfer", choices=["transfer", "batched32"],
                    help="transfer: 512-segment trees at --n-cells (the metric at 64^3); batched32: 256 instances "
                         "at 32^3 with trees of 8-128 segments, R ~ U[0.003, 0.01]")
    ap.add_argument("--weights", default=None)
    ap.add_argument("--cnn-dtype", default="bf16", choices=["bf16", "f32"])
    ap.add_argument("--jacobi-steps", type=int, default=1)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-jacobi", action="store_true")
    ap.add_argument("--smooth-sweeps", type=int, default=1,
                    help="Jacobi pre/post-smoothing steps of the extra smoothed solve (0: skip it)")
    ap.add_argument("--smooth-omega", type=float, default=0.8)
    ap.add_argument("--no-distance-run", type=int, default=1,
                    help="also time the network trained without the distance input (0: skip)")
    ap.add_argument("--inner-steps", type=int, default=3,
                    help="inner FGMRES steps of the extra inner-solve run (0: skip it)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="time and fix the launch shapes (SpMV sweep, BF16 sweep layers) before the timed solves (0: defaults)")
    ap.add_argument("--precision-runs", default="fp8,fp8a,f32",
                    help="network dtypes also timed on the same workload (comma list of f32/bf16/fp8; empty: none)")
    ap.add_argument("--block3d", type=int, default=1,
                    help="also run the paper's 3D-block workload (Neumann, k = sigma = eps = 1e-3, FGMRES(20) to "
                         "1e-6 at 21^3 / 41^3 / 81^3 nodes; 0: skip)")
    ap.add_argument("--cpu-neural-iters", type=int, default=3)
    ap.add_argument("--cpu-jacobi-iters", type=int, default=50)
    return ap.parse_args()


def spmv_bytes(S, vec_bytes=4):
    """Algorithmic bytes of one batched y = A x with A = S + M and M applied in
    its factored form B^T W B + R: x read once and y written once; the stencil
    S has a handful of constants per instance and no stored entries; the
    entries of W B (one row per Gauss point, with a row pointer each) and of
    the row-wise B^T | R (with a row index and a row pointer per listed row)
    streamed once each, values and column indices.  The intermediate t = W B x
    (one value per Gauss point) is not counted."""
    nb = ns = nq = rows = 0
    for i in range(S.n_inst):
        q, b, e = S.coupling_sizes(i)
        nq += q
        nb += b
        ns += e
        rows += S.split_sizes(i)[1]
    return 2 * S.ntot * vec_bytes + (nb + ns) * (vec_bytes + 4) + nq * 4 + rows * 8


def unet_flops(n):
    """Algorithmic FLOPs of one U-net forward at grid side n (n = 2^k + 1):
    2 * taps * Cin * Cout per output voxel; a strided convolution counts its
    27 taps (zero padding included), the transposed convolution the taps that
    reach each output parity (1, 2 or 4 or 8), the head 1 tap."""
    from paper_2505_08491_amd.weights import LAYERS
    sizes = [n, (n + 1) // 2, (n + 3) // 4]
    lvl = {"L0a": 0, "L0b": 0, "L1a": 1, "L1b": 1, "L2a": 2, "L2b": 2, "U1": 1, "D1": 1, "U0": 0, "D0": 0, "H": 0}
    tot = 0
    for name, kind, ci, co, _ in LAYERS:
        m = sizes[lvl[name]]
        if kind == "t2":
            ne = (m + 1) // 2
            taps = (ne + 2 * (m - ne)) ** 3      # output sides: even index 1 tap, odd 2 taps
            tot += 2 * taps * ci * co
        else:
            tot += 2 * (1 if kind == "pt" else 27) * ci * co * m ** 3
    return tot


STAGES = ("L0a", "L0b", "L1a", "L1b", "L2a", "L2b", "U1", "D1", "U0", "D0+H")


def stage_costs(n):
    """Per instance, for each stage of the in-solver network at grid side n:
    algorithmic FLOPs (as in `unet_flops`; D0 carries the 1x1 head) and
    compulsory HBM bytes (each input read once and each output written once:
    BF16 activations, FP32 Krylov vector and distance field in L0a, FP32 z0
    out of D0 + H)."""
    n1, n2 = (n + 1) // 2, (n + 3) // 4
    c0, c1, c2 = n ** 3, n1 ** 3, n2 ** 3
    ne = (n1 + 1) // 2
    t2_1 = (ne + 2 * (n1 - ne)) ** 3          # U1 output taps (64 -> 32 at n1)
    ne0 = (n + 1) // 2
    t2_0 = (ne0 + 2 * (n - ne0)) ** 3         # U0 output taps (32 -> 16 at n)
    fl = [2 * 27 * 2 * 16 * c0, 2 * 27 * 16 * 16 * c0, 2 * 27 * 16 * 32 * c1, 2 * 27 * 32 * 32 * c1,
          2 * 27 * 32 * 64 * c2, 2 * 27 * 64 * 64 * c2, 2 * t2_1 * 64 * 32, 2 * 27 * 64 * 32 * c1,
          2 * t2_0 * 32 * 16, 2 * 27 * 32 * 16 * c0 + 2 * 16 * c0]
    by = [8 * c0 + 32 * c0, 64 * c0, 32 * c0 + 64 * c1, 128 * c1, 64 * c1 + 128 * c2, 256 * c2, 128 * c2 + 64 * c1,
          192 * c1, 64 * c1 + 32 * c0, 64 * c0 + 4 * c0]
    return fl, by


def spmv_traffic(target):
    """HBM bytes per batched SpMV launch at the stencil sweep's z-split target
    `target` (0: the default 2048) from the committed rocprofv3 PMC summary
    (FETCH_SIZE + WRITE_SIZE scaled by a copy kernel), or None when the kernel
    source changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "spmv_64x16_traffic.txt")
    src = os.path.join(ROOT, "paper_2505_08491_amd", "csrc", "krylov.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^krylov.hip sha256: ([0-9a-f]+)$", text, re.M)
    if not m or m.group(1) != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    m = re.search(r"^traffic bytes per launch \[%d\]: (\d+)$" % (target or 2048), text, re.M)
    return float(m.group(1)) if m else None


def stage_traffic(stage):
    """HBM bytes per launch of one network stage at 64^3 x 16 from the
    committed rocprofv3 PMC summary, or None when the convolution sources
    changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "unet_64x16_traffic.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    for name in ("conv_mfma.hip", "conv.hip"):
        src = os.path.join(ROOT, "paper_2505_08491_amd", "csrc", name)
        m = re.search(r"^%s sha256: ([0-9a-f]+)$" % re.escape(name), text, re.M)
        if not m or m.group(1) != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
    m = re.search(r"^traffic bytes per launch \[%s\]: (\d+)$" % re.escape(stage), text, re.M)
    return float(m.group(1)) if m else None


def host_cpu():
    """Cores this process may run on and the CPU model name of the host."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        nproc = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    return nproc, model


def time_kernel(ctx, fn, reps):
    """Average duration (ms) of `fn` launches measured with HIP events on the
    library's stream."""
    import torch
    fn()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(ctx.stream):
        start.record(ctx.stream)
        for _ in range(reps):
            fn()
        end.record(ctx.stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


# the paper's mean FGMRES(20) iterations to 1e-6 on its own 3D-block test sets
# (k = sigma = 1e-3; 100 unseen graphs each; Section 5, iteration/time table),
# quoted as context: other graphs, other elements, other hardware
PAPER_BLOCK3D = {"none": {"21^3": 147.72, "41^3": 431.91, "81^3": ">1000"},
                 "U3hf(21^3)": {"21^3": 17.38, "41^3": 37.24, "81^3": 100.73}}


def block3d_runs(ctx, count=16):
    """The 3D-block problem of Section 5 at 21^3, 41^3 and 81^3 nodes: C u0 = b
    by FGMRES(20) to relative residual 1e-6 (cap 1000) for `count` seeded
    graphs per size, with no preconditioner, with diag(C)^-1 and with the
    networks trained on the GPU at 21^3 and at 41^3 (BF16); mean steps and
    solves/s."""
    import numpy as np
    import torch

    import synth
    import paper_2505_08491_amd as P
    from paper_2505_08491_amd import weights as W
    nets = {}
    for nc in (20, 40):
        wpath = os.path.join(os.path.dirname(W.default_path()), f"unet{nc}_block3d")
        if os.path.exists(wpath + ".bin"):
            nets[f"neural_trained_{nc + 1}^3"] = W.load(wpath)[0]
    out = {"tol": 1e-6, "restart": 20, "cap": 1000, "graphs_per_size": count,
           "weights": {k: f"paper_2505_08491_amd/weights/unet{int(k.split('_')[-1][:-2]) - 1}_block3d"
                       for k in nets}, "paper_context": PAPER_BLOCK3D}
    for n_cells in (20, 40, 80):
        S = P.System(ctx, synth.workload_block3d(n_cells, count), vec_dtype="f32")
        b = torch.from_numpy(S.rhs()).cuda()
        row = {}
        for name in ["none", "block_jacobi"] + list(nets):
            if name in nets:
                S.set_preconditioner("neural", weights=nets[name], cnn_dtype="bf16")
            else:
                S.set_preconditioner(name)
            x = torch.zeros_like(b)
            S.solve_device(b, x, restart=20, max_iters=1000, tol=1e-6, use_graph=True)   # warm-up
            torch.cuda.synchronize()
            x.zero_()
            t = time.perf_counter()
            st = S.solve_device(b, x, restart=20, max_iters=1000, tol=1e-6, use_graph=True)
            torch.cuda.synchronize()
            T = time.perf_counter() - t
            row[name] = {"iters_mean": float(np.mean([q["iters"] for q in st])),
                         "converged": int(sum(q["converged"] for q in st)), "ms_per_batch": T * 1e3,
                         "solves_per_s": S.n_inst / T}
        out[f"{n_cells + 1}^3"] = row
        S.free()
    return out


def cpu_baseline(inst, gpu_neural_iters, gpu_jacobi_iters, weights, n_neural, n_jacobi, x_gpu=None):
    """The FP64 oracle on the host cores: a bounded sample of the same solve
    (n_neural FGMRES iterations with the FP64 network and n_jacobi
    Jacobi-GMRES iterations on instance 0), scaled to solves/s with the
    per-solve iteration counts the GPU needed.  With x_gpu (the GPU's
    solution of instance 0) it also states that solution's error against the
    oracle: the oracle's reference solution x* to FP64 true relative residual
    1e-12, ||x - x*|| / ||x*||, max |x - x*| / max |x*| and the true relative
    residual of x on the oracle's own A."""
    import numpy as np
    from oracle import cnn as ocnn
    from oracle import fem, krylov
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    nproc, model = host_cpu()
    t0 = time.time()
    s = fem.assemble(inst)
    t_asm = time.time() - t0
    err = None
    if x_gpu is not None:
        t0 = time.time()
        ref = krylov.reference_solution(s, tol=1e-12, k_omega=inst.k_omega, sigma_omega=inst.sigma_omega)
        xs = ref.x
        err = {"instance": 0, "oracle_ref_rel_res": float(ref.rel_res),
               "err": float(np.linalg.norm(x_gpu - xs) / np.linalg.norm(xs)),
               "err_max": float(np.max(np.abs(x_gpu - xs)) / np.max(np.abs(xs))),
               "true_rel_res_on_oracle_A": float(np.linalg.norm(s.F - s.A @ x_gpu) / np.linalg.norm(s.F)),
               "s": time.time() - t0}
    th = weights.astype(np.float64)
    net = lambda X: ocnn.forward(th, X)[0]
    Q = krylov.BlockPreconditioner(s, krylov.p3d_neural(s, net))
    t0 = time.time()
    krylov.fgmres(s.A, s.F, precond=Q, restart=30, tol=1e-30, max_iters=n_neural)
    t_neu = (time.time() - t0) / n_neural
    t0 = time.time()
    krylov.fgmres(s.A, s.F, precond=krylov.jacobi(s.A), restart=50, tol=1e-30, max_iters=n_jacobi)
    t_jac = (time.time() - t0) / n_jacobi
    return {"value": 1.0 / (t_neu * gpu_neural_iters), "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "host_nproc": int(nproc), "host_cpu_model": model, "error_vs_oracle": err,
            "sample": (f"instance 0 of the workload: {n_neural} neural FGMRES(30) iterations (FP64 network, "
                       f"{t_neu:.2f} s/iter) and {n_jacobi} Jacobi-GMRES(50) iterations ({t_jac * 1e3:.1f} ms/iter), "
                       f"scaled by the GPU's mean iterations per solve ({gpu_neural_iters:.1f} neural, "
                       f"{gpu_jacobi_iters:.1f} Jacobi); host assembly {t_asm:.1f} s excluded"),
            "jacobi_value": 1.0 / (t_jac * gpu_jacobi_iters) if gpu_jacobi_iters else None}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported: instances shard over GPUs without "
              f"per-iteration communication, so the whole-job rate would be the per-GPU rate times the GPU count.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2505_08491_amd as P
    from paper_2505_08491_amd import weights as W

    if a.workload == "batched32":
        a.n_cells = 32
        a.count = a.count or 256
        insts = synth.workload_batched_32(a.count)
        wl_desc = (f"{a.count} seeded random trees (8-128 segments x 8 P1 elements, R ~ U[0.003, 0.01]) at "
                   f"32^3 trilinear cells")
    else:
        a.count = a.count or (16 if a.n_cells == 64 else 2)
        insts = synth.workload_transfer(a.n_cells, a.count)
        wl_desc = f"{a.count} seeded random trees (512 segments x 16 P1 elements, R=0.002) at {a.n_cells}^3 trilinear cells"
    wpath = a.weights or W.default_path()
    trained = os.path.exists(wpath + ".bin")
    w = W.load(wpath)[0] if trained else W.init(0)
    ctx = P.Context(0)
    t0 = time.time()
    S = P.System(ctx, insts, vec_dtype="f32")
    t_upload = time.time() - t0
    b = torch.from_numpy(S.rhs()).cuda()
    x = torch.zeros_like(b)
    neural_opts = dict(restart=30, max_iters=3000, fallback_restart=50, fallback_max_iters=20000, tol=1e-8,
                       use_graph=True)
    jac_opts = dict(restart=50, max_iters=40000, tol=1e-8, use_graph=True)

    def run(opts, steps, warmup):
        for _ in range(warmup):
            x.zero_()
            S.solve_device(b, x, **opts)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = None
        for _ in range(steps):
            x.zero_()
            st = S.solve_device(b, x, **opts)
        torch.cuda.synchronize()
        return (time.perf_counter() - t), st

    def true_rel():
        r = b - S.spmv(x.clone())
        out = []
        for i in range(S.n_inst):
            o0, o1 = S.offsets[i], S.offsets[i + 1]
            out.append(float(r[o0:o1].norm() / b[o0:o1].norm()))
        return out

    S.set_preconditioner("neural", weights=w, cnn_dtype=a.cnn_dtype)
    tuned, t_tune = None, 0.0
    if a.autotune:
        t0 = time.time()
        tuned = S.autotune()
        t_tune = time.time() - t0
    T, st = run(neural_opts, a.steps, a.warmup)
    rel_n = true_rel()
    x0_neural = x[S.offsets[0]:S.offsets[1]].cpu().numpy()   # instance 0, for the error against the oracle
    neural_iters = [s["iters"] + s["fallback_iters"] for s in st]
    conv_all = all(s["converged"] for s in st)
    n_fb = sum(s["used_fallback"] for s in st)

    # the network stage by stage as the solver applies it (HIP events between
    # the stages on the library stream, launch shapes as tuned)
    n = a.n_cells + 1
    stage_ms = S.layer_times(reps=10)
    fl, by = stage_costs(n)
    stages = []
    for k, name in enumerate(STAGES):
        f, b_ = fl[k] * S.n_inst, by[k] * S.n_inst
        floor = max(b_ / (HBM_PEAK_GBPS * 1e9), f / (BF16_PEAK_TFLOPS * 1e12)) * 1e3
        stages.append({"stage": name, "ms": stage_ms[k], "gflop": f / 1e9, "algorithmic_mb": b_ / 1e6,
                       "tflops": f / (stage_ms[k] * 1e-3) / 1e12,
                       "frac_bf16_peak": f / (stage_ms[k] * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                       "floor_ms": floor, "frac_of_floor": floor / stage_ms[k],
                       "bound": "hbm" if b_ / (HBM_PEAK_GBPS * 1e9) > f / (BF16_PEAK_TFLOPS * 1e12) else "mfma"})
    dom = max(range(len(STAGES)), key=lambda k: stage_ms[k])

    # the batched FP32 SpMV (HBM-bound): every timed launch starts after a
    # 1 GiB read, which evicts the 256 MB last-level cache (MALL) without
    # leaving dirty lines to write back, so operator and vectors come from
    # HBM; events on the library stream around each launch
    xs = torch.randn(S.ntot, device="cuda")
    ys = torch.empty_like(xs)
    flush = torch.ones(1 << 28, device="cuda")
    fsum = torch.empty(20, device="cuda")
    e0 = [torch.cuda.Event(enable_timing=True) for _ in range(20)]
    e1 = [torch.cuda.Event(enable_timing=True) for _ in range(20)]
    S.spmv_repeat(xs, ys, 1)
    with torch.cuda.stream(ctx.stream):
        for k in range(20):
            torch.sum(flush, dim=0, out=fsum[k])
            e0[k].record(ctx.stream)
            S.spmv_repeat(xs, ys, 1)
            e1[k].record(ctx.stream)
    e1[-1].synchronize()
    ms_spmv = sum(e0[k].elapsed_time(e1[k]) for k in range(20)) / 20
    gbps = spmv_bytes(S) / (ms_spmv * 1e-3) / 1e9
    # the same launches back to back (operator partly resident in the MALL)
    reps = 50
    ms_spmv_warm = time_kernel(ctx, lambda: S.spmv_repeat(xs, ys, reps), 3) / reps
    # practical copy bandwidth (1 GiB device-to-device) on the same stream
    cbuf = torch.empty(2, 1 << 28, device="cuda")
    with torch.cuda.stream(ctx.stream):
        ms_copy = time_kernel(ctx, lambda: cbuf[1].copy_(cbuf[0]), 10)
    copy_gbps = 2 * cbuf[0].numel() * 4 / (ms_copy * 1e-3) / 1e9
    del cbuf, flush, fsum
    # preconditioner application (1D solve + extension + U-net + unscale) on the batch
    ms_prec = time_kernel(ctx, lambda: S.precond_apply(xs), 5)
    cnn_flop = unet_flops(n) * S.n_inst
    # the network alone (stored activations, BF16 MFMA) on the same batch
    wd = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    xin = torch.randn(S.n_inst, n ** 3, 2, device="cuda")
    ms_cnn = time_kernel(ctx, lambda: ctx.cnn_forward(wd, xin, n, a.cnn_dtype), 5)
    del xin

    # the same solve with Jacobi pre/post-smoothing of the network's 3D solve
    smoothed = None
    if a.smooth_sweeps > 0:
        S.set_preconditioner("neural", weights=w, cnn_dtype=a.cnn_dtype)
        S.set_smoothing(a.smooth_sweeps, a.smooth_omega)
        Ts, sts = run(neural_opts, a.steps, 1)
        rel_s = true_rel()
        ms_prec_s = time_kernel(ctx, lambda: S.precond_apply(xs), 5)
        S.set_smoothing(0)
        smoothed = {"sweeps": a.smooth_sweeps, "omega": a.smooth_omega,
                    "solves_per_s": S.n_inst * a.steps / Ts, "ms_per_solve": Ts / a.steps * 1e3,
                    "iters_mean": float(np.mean([q["iters"] + q["fallback_iters"] for q in sts])),
                    "converged_all": all(q["converged"] for q in sts),
                    "used_fallback": int(sum(q["used_fallback"] for q in sts)), "max_true_rel_res": max(rel_s),
                    "ms_per_apply": ms_prec_s}

    # the 3D block solved by inner FGMRES steps with the network as preconditioner
    inner = None
    if a.inner_steps > 0:
        S.set_preconditioner("neural", weights=w, cnn_dtype=a.cnn_dtype)
        S.set_inner_steps(a.inner_steps)
        Ti, sti = run(neural_opts, a.steps, 1)
        rel_i = true_rel()
        ms_prec_i = time_kernel(ctx, lambda: S.precond_apply(xs), 5)
        S.set_inner_steps(0)
        inner = {"steps": a.inner_steps, "solves_per_s": S.n_inst * a.steps / Ti, "ms_per_solve": Ti / a.steps * 1e3,
                 "iters_mean": float(np.mean([q["iters"] + q["fallback_iters"] for q in sti])),
                 "converged_all": all(q["converged"] for q in sti),
                 "used_fallback": int(sum(q["used_fallback"] for q in sti)), "max_true_rel_res": max(rel_i),
                 "ms_per_apply": ms_prec_i}

    # the network trained with its distance-channel weights held at zero (ablation)
    nodist = None
    npath = os.path.join(os.path.dirname(W.default_path()), "unet32_nodist")
    if a.no_distance_run and os.path.exists(npath + ".bin"):
        wnd = W.load(npath)[0]
        S.set_preconditioner("neural", weights=wnd, cnn_dtype=a.cnn_dtype)
        Tn, stn = run(neural_opts, a.steps, 1)
        rel_nd = true_rel()
        nodist = {"weights": os.path.relpath(npath, ROOT), "solves_per_s": S.n_inst * a.steps / Tn,
                  "ms_per_solve": Tn / a.steps * 1e3,
                  "iters_mean": float(np.mean([q["iters"] + q["fallback_iters"] for q in stn])),
                  "converged_all": all(q["converged"] for q in stn),
                  "used_fallback": int(sum(q["used_fallback"] for q in stn)), "max_true_rel_res": max(rel_nd)}

    # the same network in other arithmetic: FP32 (FP32 matrix cores), E4M3
    # weights with per-channel power-of-two scales on the BF16 kernels (fp8),
    # and E4M3 weights and activations on the FP8 matrix cores (fp8a, its
    # activation scales calibrated on the right-hand side)
    precision = {}
    for dt in [d for d in a.precision_runs.split(",") if d and d != a.cnn_dtype]:
        S.set_preconditioner("neural", weights=w, cnn_dtype=dt)
        fp8_scales = S.fp8_calibrate(b.to(torch.float32)) if dt == "fp8a" else None
        Tp, stp = run(neural_opts, 1, 1)
        rel_p = true_rel()
        precision[dt] = {"solves_per_s": S.n_inst / Tp, "ms_per_solve": Tp * 1e3,
                         "iters_mean": float(np.mean([q["iters"] + q["fallback_iters"] for q in stp])),
                         "converged_all": all(q["converged"] for q in stp),
                         "used_fallback": int(sum(q["used_fallback"] for q in stp)), "max_true_rel_res": max(rel_p),
                         "ms_per_apply": time_kernel(ctx, lambda: S.precond_apply(xs), 3)}
        if fp8_scales:
            precision[dt]["activation_scales"] = fp8_scales

    block3d = block3d_runs(ctx) if a.block3d else None

    jac = None
    if not a.skip_jacobi:
        S.set_preconditioner("jacobi")
        Tj, stj = run(jac_opts, a.jacobi_steps, 0)
        rel_j = true_rel()
        jac = {"solves_per_s": S.n_inst * a.jacobi_steps / Tj, "ms_per_solve": Tj / a.jacobi_steps * 1e3,
               "iters_mean": float(np.mean([s["iters"] for s in stj])),
               "converged": all(s["converged"] for s in stj), "max_true_rel_res": max(rel_j)}

    value = S.n_inst * a.steps / T
    out = {
        "metric": "solves/s to rel-res 1e-8 at 64^3: neural FGMRES vs Jacobi GMRES; HBM GB/s",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": T / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16/f32/f64", "data": "synthetic",
        "config": {"workload": f"{wl_desc}, FP32 vectors and SpMV, FP64 MGS/Givens/x/true residual, "
                               f"{a.cnn_dtype} U-net with FP32 accumulation", "instances": a.count,
                   "n_cells": a.n_cells,
                   "restart": 30, "tol": 1e-8, "cnn_dtype": a.cnn_dtype,
                   "weights": os.path.relpath(wpath, ROOT) if trained else "untrained (Kaiming init)"},
        "neural": {"iters_mean": float(np.mean(neural_iters)), "iters_max": int(max(neural_iters)),
                   "converged_all": conv_all, "used_fallback": int(n_fb), "max_true_rel_res": max(rel_n)},
        "neural_smoothed": smoothed,
        "neural_inner_fgmres": inner,
        "neural_no_distance": nodist,
        "neural_precision": precision or None,
        "paper_block3d": block3d,
        "jacobi": jac,
        "roofline": {"bound": stages[dom]["bound"],
                     "kernel": f"network stage {STAGES[dom]} (BF16 MFMA convolution launch, in-solver shape)",
                     "achieved": stages[dom]["tflops"], "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": stages[dom]["frac_bf16_peak"],
                     "traffic": (stage_traffic(STAGES[dom])
                                 if (a.workload, a.n_cells, a.count, a.cnn_dtype) == ("transfer", 64, 16, "bf16")
                                 else None),
                     "algorithmic_flops": fl[dom] * S.n_inst, "algorithmic_bytes": by[dom] * S.n_inst,
                     "ms_per_launch": stage_ms[dom]},
        "unet_stages": stages,
        "spmv": {"bound": "hbm", "kernel": "k_cgather + k_stencil_sweep + k_cscatter (batched y = (S + B^T W B + R) x, FP32)",
                 "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                 "timing": "each launch after a 1 GiB read that evicts the last-level cache",
                 "traffic": (spmv_traffic(tuned[11] if tuned else 0)
                             if (a.workload, a.n_cells, a.count) == ("transfer", 64, 16) else None),
                 "algorithmic_bytes": spmv_bytes(S), "ms_per_launch": ms_spmv,
                 "ms_per_launch_back_to_back": ms_spmv_warm, "copy_gbps": copy_gbps},
        "unet": {"bound": "mfma", "dtype": a.cnn_dtype, "gflop_per_forward": cnn_flop / 1e9,
                 "ms_in_solver": sum(stage_ms), "frac_in_solver": cnn_flop / (sum(stage_ms) * 1e-3) / 1e12 /
                 BF16_PEAK_TFLOPS,
                 "ms_per_forward": ms_cnn, "achieved": cnn_flop / (ms_cnn * 1e-3) / 1e12,
                 "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": cnn_flop / (ms_cnn * 1e-3) / 1e12 / BF16_PEAK_TFLOPS},
        "preconditioner": {"ms_per_apply": ms_prec, "cnn_tflops": cnn_flop / (ms_prec * 1e-3) / 1e12},
        "upload_s": t_upload,
        "autotune": {"conv_sweep_blocks": tuned[:11], "spmv_sweep_target": tuned[11],
                     "conv_rows_l1b_d1_l0b_d0": tuned[12:16],
                     "tconv_workgroups_u1_u0": tuned[16:18],
                     "conv_xblocks_l0a_l0b_l1b_d1_d0": tuned[18:23], "s": t_tune} if tuned else None,
    }
    if not a.skip_cpu:
        out["cpu_baseline"] = cpu_baseline(insts[0], float(np.mean(neural_iters)),
                                           jac["iters_mean"] if jac else 0.0, w, a.cpu_neural_iters,
                                           a.cpu_jacobi_iters, x_gpu=x0_neural)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
