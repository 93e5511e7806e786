"""Training-set augmentation and parameterisation ablation (Section 5.1,
tables on the effect of the training data and of the distance input).

Trains the U-net at 32^3 with the library's own kernels on different sample
mixes and evaluates each network as the 3D preconditioner of FGMRES(30) on
the coupled system:

    none     b/||b|| only (the B set, no augmentation)
    krylov   B set + Arnoldi vectors v5..v8 of a Jacobi-GMRES cycle
    hf       B set + random unit vectors (high-frequency augmentation)
    all      B set + Arnoldi vectors + random vectors (the shipped network)
    all-nod  as `all` with the distance-channel weights held at zero

Evaluation: mean FGMRES steps to rel-res 1e-8 on 64 instances at 32^3 and on
the 16-instance 64^3 workload (plain and with one Jacobi smoothing step on each
side), next to block-Jacobi (the method without the network).

    python -m paper_2505_08491_amd.ablation --out paper_2505_08491_amd/weights/ablation.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import train as T
from . import weights as W
from .api import Context, System

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

VARIANTS = {
    "none": dict(p_random=0.0, p_rhs=1.0),
    "krylov": dict(p_random=0.0, p_rhs=0.5),
    "hf": dict(p_random=0.5, p_rhs=0.5),
    "all": dict(p_random=0.5, p_rhs=0.25),
    "all-nod": dict(p_random=0.5, p_rhs=0.25, no_dist=True),
}


def mean_iters(ctx, S, prec, w=None, smooth=0):
    if prec == "neural":
        S.set_preconditioner("neural", weights=w, cnn_dtype="bf16")
        S.set_smoothing(smooth, 0.8)
    else:
        S.set_preconditioner(prec)
    b = torch.from_numpy(S.rhs()).cuda()
    x = torch.zeros_like(b)
    st = S.solve_device(b, x, restart=30, max_iters=3000, fallback_restart=50, fallback_max_iters=20000, tol=1e-8,
                        use_graph=True)
    if prec == "neural":
        S.set_smoothing(0)
    it = [q["iters"] + q["fallback_iters"] for q in st]
    return {"iters_mean": float(np.mean(it)), "iters_max": int(max(it)),
            "converged": int(sum(q["converged"] for q in st)), "fallback": int(sum(q["used_fallback"] for q in st))}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--variants", default=",".join(VARIANTS))
    ap.add_argument("--reuse-shipped", action="store_true", help="take the shipped weights for `all`")
    ap.add_argument("--reuse-nodist", action="store_true",
                    help="take the shipped no-distance weights for `all-nod` (their distance weights are zero, "
                         "so the distance scaling does not change them)")
    ap.add_argument("--save-dir", default=None, help="save every trained network as <dir>/unet32_<variant>")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import synth
    nets = {}
    meta = {}
    for name in a.variants.split(","):
        nodist_path = os.path.join(os.path.dirname(W.default_path()), "unet32_nodist")
        if name == "all" and a.reuse_shipped and os.path.exists(W.default_path() + ".bin"):
            nets[name], m = W.load(W.default_path())
        elif name == "all-nod" and a.reuse_nodist and os.path.exists(nodist_path + ".bin"):
            nets[name], m = W.load(nodist_path)
        else:
            print(f"training {name}", flush=True)
            out = os.path.join(a.save_dir, "unet32_" + name) if a.save_dir else None
            nets[name], m = T.train(steps=a.steps, out=out, **VARIANTS[name])
        meta[name] = {k: m.get(k) for k in ("p_random", "p_rhs", "no_dist", "train_seconds")}
        meta[name]["final_val_loss"] = m["history"][-1]["val_loss"] if m.get("history") else None
    ctx = Context(0)
    res = {"variants": meta, "eval": {}}
    for wl, insts in (("32^3 x 64", synth.workload_batched_32(64)), ("64^3 x 16", synth.workload_transfer(64, 16))):
        t0 = time.time()
        S = System(ctx, insts, vec_dtype="f32")
        row = {"block-jacobi": mean_iters(ctx, S, "block_jacobi")}
        for name, w in nets.items():
            row[name] = mean_iters(ctx, S, "neural", w)
            if wl.startswith("64"):
                row[name + " +smooth"] = mean_iters(ctx, S, "neural", w, smooth=1)
        S.free()
        res["eval"][wl] = row
        print(wl, f"{time.time() - t0:.1f}s", json.dumps(row), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
        print("saved", a.out, flush=True)
    return res


if __name__ == "__main__":
    main()
