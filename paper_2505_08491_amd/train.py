"""On-device training of the U-net preconditioner (Section 5.1 objective).

Minimises the empirical risk  mean_k || r_k - alpha^-1 C_k U([r_k, d_k]) ||^2
over unit-norm samples r_k of seeded random training graphs, with every step
of the computation in the library's kernels: input packing, the forward pass
(BF16 or FP32 activations, FP32 accumulation), the loss and its gradient with
the FP32 SpMV of C = A00, the backward (adjoint) pass and Adam on FP32 master
weights.

Training set (Section 4.1): per graph the normalised right-hand side of the
decoupled 3D problem b = -A01 A11^-1 f1, solver-generated Arnoldi vectors
v5..v8 of a Jacobi-GMRES cycle on the coupled system (3D parts), and fresh
random unit vectors r = v / ||v||, v ~ N(0, I) (the high-frequency
augmentation), all vanishing on the Dirichlet boundary.

With --workload block3d the network is trained for the 3D-block problem of
Section 5 (natural boundary, k = sigma = 1e-3, eps = 1e-3, C = A00 alone): the
Arnoldi vectors are those of an unpreconditioned GMRES cycle on C u0 = b, an
orthonormal basis of the Krylov space K_8(C, b) of Section 5.1, and no entry
is fixed on the boundary.

    python -m paper_2505_08491_amd.train --steps 2000 --batch 32 --graphs 128
    python -m paper_2505_08491_amd.train --workload block3d --n-cells 20 --out weights/unet20_block3d
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import weights as W
from .api import Context, System
from .autograd import residual_loss, unet

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def boundary_mask(n: int, device) -> torch.Tensor:
    idx = torch.arange(n, device=device)
    e = (idx == 0) | (idx == n - 1)
    return (e[None, None, :] | e[None, :, None] | e[:, None, None]).reshape(-1)


def build_bank(ctx: Context, S: System, krylov_ids=(5, 6, 7, 8), block3d=False) -> torch.Tensor:
    """[G][1 + len(krylov_ids)][n3d] unit vectors: b/||b|| and Arnoldi vectors."""
    G, n3d, dev = S.n_inst, S.n3d, "cuda"
    F = torch.from_numpy(S.rhs()).to(dev, torch.float32)
    bank = torch.zeros(G, 1 + len(krylov_ids), n3d, device=dev)
    if block3d:                              # F = [b; 0] already
        for i in range(G):
            o0 = S.offsets[i]
            b = F[o0:o0 + n3d]
            bank[i, 0] = b / b.norm()
    else:
        v = torch.zeros_like(F)
        for i in range(G):                   # v = [0; f1]
            o0, o1 = S.offsets[i], S.offsets[i + 1]
            v[o0 + n3d:o1] = F[o0 + n3d:o1]
        z = S.tree_solve(v)                  # [0; A11^-1 f1]
        y = S.spmv(z)                        # [A01 A11^-1 f1; ...]
        for i in range(G):
            o0 = S.offsets[i]
            b = -y[o0:o0 + n3d]
            bank[i, 0] = b / b.norm()
    # one GMRES cycle (Jacobi-preconditioned on the coupled system, plain on
    # C for the 3D block); its Arnoldi vectors are the samples
    S.set_preconditioner("none" if block3d else "jacobi")
    m = max(krylov_ids)
    S.solve(S.rhs(), restart=m, max_iters=m, tol=1e-30)
    for c, k in enumerate(krylov_ids):
        vk = S.export_basis(k)
        for i in range(G):
            o0 = S.offsets[i]
            q = vk[o0:o0 + n3d].float()
            bank[i, 1 + c] = q / q.norm()
    return bank


def dist_weight_mask() -> np.ndarray:
    """Indices of the first layer's weights on the distance channel (input
    channel 1 of L0a, laid out [16][27][2] at the start of the flat vector)."""
    return np.arange(16 * 27) * 2 + 1


def train(steps=2000, batch=32, graphs=128, n_cells=32, lr=1e-3, lr_min=1e-5, dtype="bf16", seed=0,
          p_random=0.5, p_rhs=0.25, out=None, log_every=50, val_graphs=16, resume=None, no_dist=False,
          workload="coupled"):
    """no_dist: the first layer's distance-channel weights are held at zero, so
    the network never sees the distance field (parameterisation ablation).
    workload: "coupled" (Dirichlet, k = 1, the coupled system's 3D block) or
    "block3d" (the 3D-block problem of Section 5, natural boundary)."""
    torch.manual_seed(seed)
    ctx = Context(0)
    t0 = time.time()
    import synth
    block3d = workload == "block3d"
    if block3d:
        pool = synth.workload_training_block3d(graphs, n_cells=n_cells)
        val = synth.workload_training_block3d(val_graphs, n_cells=n_cells, base=40_000)
    else:
        pool = synth.workload_training(graphs, n_cells=n_cells)
        val = synth.workload_training(val_graphs, n_cells=n_cells, base=20_000)
    S = System(ctx, pool, vec_dtype="f32")
    bank = build_bank(ctx, S, block3d=block3d)
    SV = System(ctx, val, vec_dtype="f32")
    vbank = build_bank(ctx, SV, block3d=block3d)
    n = n_cells + 1
    n3d = S.n3d
    bnd = boundary_mask(n, "cuda") if not block3d else torch.zeros(n3d, dtype=torch.bool, device="cuda")
    print(f"setup {time.time() - t0:.1f}s: {graphs} graphs at {n_cells}^3, bank {tuple(bank.shape)}", flush=True)

    w = torch.from_numpy(W.init(seed)).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    step0 = 0
    if resume:
        w0, meta = W.load(resume)
        w = torch.from_numpy(w0).cuda()
        if meta.get("adam_file"):
            ad = np.fromfile(os.path.join(os.path.dirname(resume), meta["adam_file"]), dtype="<f4")
            m = torch.from_numpy(ad[:W.N_PARAMS].copy()).cuda()
            v = torch.from_numpy(ad[W.N_PARAMS:].copy()).cuda()
        step0 = int(meta.get("step", 0))
    dmask = torch.from_numpy(dist_weight_mask()).cuda() if no_dist else None
    if dmask is not None:
        w[dmask] = 0.0
    w.requires_grad_(True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed + 1)
    history = []
    tstart = time.time()

    def sample(B, bk, G):
        inst = torch.randint(0, G, (B,), device="cuda", generator=gen, dtype=torch.int64)
        u = torch.rand(B, device="cuda", generator=gen)
        kind = torch.where(u < p_random, 0, torch.where(u < p_random + p_rhs, 1, 2))
        kk = torch.randint(1, bk.shape[1], (B,), device="cuda", generator=gen)
        col = torch.where(kind == 1, torch.zeros_like(kk), kk)
        r = bk[inst, col]
        rnd = torch.randn(B, n3d, device="cuda", generator=gen)
        rnd[:, bnd] = 0
        rnd = rnd / rnd.norm(dim=1, keepdim=True)
        r = torch.where((kind == 0)[:, None], rnd, r).contiguous()
        return inst.to(torch.int32).contiguous(), r

    def evaluate(wt):
        inst, r = sample(batch, vbank, SV.n_inst)
        X = SV.pack_input(inst, r)
        with torch.no_grad():
            y = ctx.cnn_forward(wt.detach(), X, n, dtype)
            loss, _ = SV.loss_grad(inst, r, y)
        return float(loss.mean())

    for step in range(step0 + 1, steps + 1):
        inst, r = sample(batch, bank, S.n_inst)
        X = S.pack_input(inst, r)
        # forward, loss and adjoint through the library's kernels, chained by autograd
        loss = residual_loss(unet(w, X, ctx, n, dtype), r, inst, S)
        w.grad = None
        loss.sum().backward()
        frac = (step - 1) / max(1, steps - 1)
        lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * frac))
        ctx.adam_step(w.data, w.grad, m, v, lr_t, step)
        if dmask is not None:
            w.data[dmask] = 0.0
        if step % log_every == 0 or step == step0 + 1 or step == steps:
            lv = float(loss.detach().mean())
            vl = evaluate(w)
            el = time.time() - tstart
            history.append({"step": step, "loss": lv, "val_loss": vl, "lr": lr_t, "time_s": el})
            print(f"step {step:5d} loss {lv:.4e} val {vl:.4e} lr {lr_t:.2e} {el:.1f}s", flush=True)
            if not math.isfinite(lv):
                raise RuntimeError("training diverged")
    torch.cuda.synchronize()
    elapsed = time.time() - tstart
    wn = w.detach().cpu().numpy()
    meta = {"step": steps, "batch": batch, "graphs": graphs, "n_cells": n_cells, "lr": lr, "lr_min": lr_min,
            "schedule": "cosine", "dtype": dtype, "seed": seed, "p_random": p_random, "p_rhs": p_rhs,
            "no_dist": bool(no_dist), "workload": workload, "train_seconds": elapsed, "history": history}
    if out:
        os.makedirs(os.path.dirname(out), exist_ok=True)
        W.save(out, wn, meta, adam=(m.cpu().numpy(), v.cpu().numpy()))
        print("saved", out, flush=True)
    S.free()
    SV.free()
    return wn, meta


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--graphs", type=int, default=128)
    ap.add_argument("--n-cells", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--dtype", default="bf16", choices=["bf16", "f32"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--log-every", type=int, default=50)
    ap.add_argument("--p-random", type=float, default=0.5, help="share of random unit samples")
    ap.add_argument("--p-rhs", type=float, default=0.25, help="share of b/||b|| samples (the rest: Arnoldi vectors)")
    ap.add_argument("--no-dist", action="store_true", help="keep the distance-channel weights at zero")
    ap.add_argument("--workload", default="coupled", choices=["coupled", "block3d"],
                    help="coupled: the coupled system (Dirichlet, k = 1); block3d: the 3D block of Section 5 "
                         "(natural boundary, k = sigma = eps = 1e-3)")
    a = ap.parse_args(argv)
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    train(steps=a.steps, batch=a.batch, graphs=a.graphs, n_cells=a.n_cells, lr=a.lr, dtype=a.dtype, seed=a.seed,
          p_random=a.p_random, p_rhs=a.p_rhs, out=a.out, log_every=a.log_every, resume=a.resume,
          no_dist=a.no_dist, workload=a.workload)


if __name__ == "__main__":
    main()
