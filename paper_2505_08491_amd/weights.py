"""U-net parameter layout, initialisation and checkpoint files.

Layout (Section 4.2 network with three levels of 16/32/64 channels): layers
L0a L0b L1a L1b L2a L2b U1 D1 U0 D0 H, each stored as [Cout][kz][ky][kx][Cin]
followed by its bias; 353,713 FP32 values in total.

A checkpoint is a raw little-endian FP32 file `<name>.bin` plus `<name>.json`
with the architecture, the storage format ("storage"), the training
configuration (its "dtype" is the arithmetic of the training forward pass)
and the Adam state file.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

# (name, kind, cin, cout, relu); kinds: s1 conv stride 1, s2 conv stride 2,
# t2 transposed conv stride 2, pt 1x1 conv
LAYERS = [("L0a", "s1", 2, 16, True), ("L0b", "s1", 16, 16, True), ("L1a", "s2", 16, 32, True),
          ("L1b", "s1", 32, 32, True), ("L2a", "s2", 32, 64, True), ("L2b", "s1", 64, 64, True),
          ("U1", "t2", 64, 32, False), ("D1", "s1", 64, 32, True), ("U0", "t2", 32, 16, False),
          ("D0", "s1", 32, 16, True), ("H", "pt", 16, 1, False)]

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def layer_sizes():
    return [((1 if k == "pt" else 27) * ci * co, co) for _, k, ci, co, _ in LAYERS]


N_PARAMS = sum(a + b for a, b in layer_sizes())


def init(seed: int) -> np.ndarray:
    """Kaiming-uniform weights (fan-in; gain sqrt(2) before a ReLU, 1 otherwise), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for (name, kind, ci, co, relu), (nw, nb) in zip(LAYERS, layer_sizes()):
        fan_in = nw // co
        bound = math.sqrt((6.0 if relu else 3.0) / fan_in)
        out.append(rng.uniform(-bound, bound, nw))
        out.append(np.zeros(nb))
    return np.concatenate(out).astype(np.float32)


def save(path_stem: str, w: np.ndarray, meta: dict, adam: tuple | None = None) -> None:
    w = np.ascontiguousarray(w, dtype="<f4")
    assert w.size == N_PARAMS
    w.tofile(path_stem + ".bin")
    meta = dict(meta, n_params=N_PARAMS, layers=[list(l) for l in LAYERS], storage="float32-le")
    if adam is not None:
        np.concatenate([np.asarray(adam[0], "<f4"), np.asarray(adam[1], "<f4")]).tofile(path_stem + ".adam.bin")
        meta["adam_file"] = os.path.basename(path_stem) + ".adam.bin"
    with open(path_stem + ".json", "w") as f:
        json.dump(meta, f, indent=1)


def load(path_stem: str):
    """(weights float32 [N_PARAMS], metadata dict)."""
    w = np.fromfile(path_stem + ".bin", dtype="<f4")
    if w.size != N_PARAMS:
        raise ValueError(f"{path_stem}.bin holds {w.size} values, expected {N_PARAMS}")
    meta = {}
    if os.path.exists(path_stem + ".json"):
        with open(path_stem + ".json") as f:
            meta = json.load(f)
    return w, meta


def default_path() -> str:
    return os.path.join(WEIGHTS_DIR, "unet32")
