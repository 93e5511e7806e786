"""The U-net preconditioner in FP64: forward, adjoint (backward), loss, Adam (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Architecture (Section 4.2, recursion U_j = Psi_j([U_{j-1} o Phi_j | Phi_j]))
with three levels of 16 / 32 / 64 channels, 3x3x3 kernels, ReLU, stride-2
convolutions going down and stride-2 transposed convolutions going up, skip
connections by channel stacking:

  L0a conv s1 2->16 ReLU      L0b conv s1 16->16 ReLU  (skip0)
  L1a conv s2 16->32 ReLU     L1b conv s1 32->32 ReLU  (skip1)
  L2a conv s2 32->64 ReLU     L2b conv s1 64->64 ReLU
  U1  tconv s2 64->32         D1  conv s1 [U1|skip1] 64->32 ReLU
  U0  tconv s2 32->16         D0  conv s1 [U0|skip0] 32->16 ReLU
  H   conv 1x1 16->1

Tensors are [n, n, n, C] (z, y, x, channel); a batch adds a leading axis.
Convolution is the cross-correlation y[p] = b + sum_t sum_c w[o, t, c]
x[s p + t - 1, c] with zero padding (the paper writes the flipped form
x(p - q); with learned weights the two are the same family).  The transposed
convolution is its adjoint: y[o] = b + sum over (i, t) with o = 2 i + t - 1.
Weights are stored per layer as [Cout][kz][ky][kx][Cin] followed by the bias.
"""
from __future__ import annotations

import math

import numpy as np

# (name, kind, cin, cout, relu)
LAYERS = [
    ("L0a", "conv1", 2, 16, True),
    ("L0b", "conv1", 16, 16, True),
    ("L1a", "conv2", 16, 32, True),
    ("L1b", "conv1", 32, 32, True),
    ("L2a", "conv2", 32, 64, True),
    ("L2b", "conv1", 64, 64, True),
    ("U1", "tconv", 64, 32, False),
    ("D1", "conv1", 64, 32, True),
    ("U0", "tconv", 32, 16, False),
    ("D0", "conv1", 32, 16, True),
    ("H", "point", 16, 1, False),
]


def layer_sizes():
    out = []
    for name, kind, cin, cout, _ in LAYERS:
        taps = 1 if kind == "point" else 27
        out.append((taps * cin * cout, cout))
    return out


def n_params():
    return sum(a + b for a, b in layer_sizes())


def unflatten(theta):
    """Flat parameter vector -> list of (w [Cout, taps, Cin], b [Cout])."""
    params = []
    off = 0
    for (name, kind, cin, cout, _), (nw, nb) in zip(LAYERS, layer_sizes()):
        taps = 1 if kind == "point" else 27
        w = np.asarray(theta[off:off + nw], dtype=np.float64).reshape(cout, taps, cin)
        off += nw
        b = np.asarray(theta[off:off + nb], dtype=np.float64)
        off += nb
        params.append((w, b))
    return params


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def taps3():
    return [(tz, ty, tx) for tz in range(3) for ty in range(3) for tx in range(3)]


# --------------------------------------------------------------------------
# single layers (one sample, [n, n, n, C])
# --------------------------------------------------------------------------

def conv3d(x, w, b, stride):
    """y[p, o] = b[o] + sum_t sum_c w[o, t, c] x[stride p + t - 1, c], zero padded."""
    n = x.shape[0]
    no = (n - 1) // stride + 1
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((no, no, no, w.shape[0]))
    for t, (tz, ty, tx) in enumerate(taps3()):
        span = stride * (no - 1) + 1
        xs = xp[tz:tz + span:stride, ty:ty + span:stride, tx:tx + span:stride, :]
        y += xs @ w[:, t, :].T
    return y + b


def tconv3d(x, w, b):
    """y[o, co] = b[co] + sum over (i, t) with o = 2 i + t - 1 of w[co, t, c] x[i, c]; size 2n - 1."""
    n = x.shape[0]
    no = 2 * n - 1
    yp = np.zeros((no + 2, no + 2, no + 2, w.shape[0]))   # index o + 1
    for t, (tz, ty, tx) in enumerate(taps3()):
        contrib = x @ w[:, t, :].T
        yp[tz:tz + 2 * n - 1:2, ty:ty + 2 * n - 1:2, tx:tx + 2 * n - 1:2, :] += contrib
    return yp[1:no + 1, 1:no + 1, 1:no + 1, :] + b


def point(x, w, b):
    return x @ w[:, 0, :].T + b


def conv3d_backward(x, w, dy, stride):
    """Adjoint of conv3d: (dx, dw, db) for the upstream gradient dy."""
    n = x.shape[0]
    no = dy.shape[0]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    span = stride * (no - 1) + 1
    for t, (tz, ty, tx) in enumerate(taps3()):
        sl = (slice(tz, tz + span, stride), slice(ty, ty + span, stride), slice(tx, tx + span, stride))
        dxp[sl] += dy @ w[:, t, :]
        dw[:, t, :] = np.einsum("zyxo,zyxc->oc", dy, xp[sl])
    db = dy.sum(axis=(0, 1, 2))
    return dxp[1:n + 1, 1:n + 1, 1:n + 1, :], dw, db


def tconv3d_backward(x, w, dy):
    """Adjoint of tconv3d: (dx, dw, db)."""
    n = x.shape[0]
    no = dy.shape[0]
    dyp = np.pad(dy, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (tz, ty, tx) in enumerate(taps3()):
        sl = (slice(tz, tz + 2 * n - 1, 2), slice(ty, ty + 2 * n - 1, 2), slice(tx, tx + 2 * n - 1, 2))
        dx += dyp[sl] @ w[:, t, :]
        dw[:, t, :] = np.einsum("zyxo,zyxc->oc", dyp[sl], x)
    db = dy.sum(axis=(0, 1, 2))
    return dx, dw, db


def point_backward(x, w, dy):
    dx = dy @ w[:, 0, :]
    dw = np.einsum("zyxo,zyxc->oc", dy, x)[:, None, :]
    return dx, dw, dy.sum(axis=(0, 1, 2))


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------

def _apply(kind, x, w, b):
    if kind == "conv1":
        return conv3d(x, w, b, 1)
    if kind == "conv2":
        return conv3d(x, w, b, 2)
    if kind == "tconv":
        return tconv3d(x, w, b)
    return point(x, w, b)


def _backward(kind, x, w, dy):
    if kind == "conv1":
        return conv3d_backward(x, w, dy, 1)
    if kind == "conv2":
        return conv3d_backward(x, w, dy, 2)
    if kind == "tconv":
        return tconv3d_backward(x, w, dy)
    return point_backward(x, w, dy)


def check_grid(n):
    if n < 5 or (n - 1) % 4 != 0:
        raise ValueError(f"grid side n={n} must satisfy n = 1 (mod 4), n >= 5")


def round_bf16(x):
    """Round to the nearest bfloat16 value (the upper half of an IEEE binary32:
    8 exponent bits, 8 significand bits), ties to an even significand, by way
    of the nearest binary32.  Finite inputs only."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    low = bits & 0xFFFF
    keep = bits >> 16
    up = (low > 0x8000) | ((low == 0x8000) & ((keep & 1) == 1))
    out = ((keep + up.astype(np.uint64)) << 16).astype(np.uint32)
    return out.view(np.float32).astype(np.float64)


def forward(theta, X, emulate=None):
    """U(X) for one sample X [n, n, n, 2]; returns ([n, n, n], cache).

    emulate="bf16" evaluates the network as the mixed-precision kernels do, so
    that both sides take their ReLU decisions on the same values: the input
    channels and the weights of the ten 3x3x3 layers are rounded to bfloat16
    (biases and the 1x1 head stay in full precision) and every layer's output,
    after its ReLU, is rounded to bfloat16 before the next layer reads it; the
    arithmetic itself stays FP64.  The cache then holds the rounded tensors,
    and `backward` gives the adjoint of that network at those points (the
    rounding passed straight through, the weights of the adjoint unrounded).
    """
    n = X.shape[0]
    check_grid(n)
    P = unflatten(theta)
    rnd = (lambda t: t) if emulate is None else round_bf16
    if emulate not in (None, "bf16"):
        raise ValueError(emulate)
    Pf = [(w if LAYERS[i][1] == "point" else rnd(w), b) for i, (w, b) in enumerate(P)]
    X = rnd(X)
    cache = {"X": X}
    idx = {name: i for i, (name, *_r) in enumerate(LAYERS)}

    def run(name, inp):
        i = idx[name]
        _, kind, _, _, relu = LAYERS[i]
        z = _apply(kind, inp, *Pf[i])
        cache[name] = (inp, z)
        out = np.maximum(z, 0.0) if relu else z
        return out if kind == "point" else rnd(out)

    a = run("L0a", X)
    s0 = run("L0b", a)
    a = run("L1a", s0)
    s1 = run("L1b", a)
    a = run("L2a", s1)
    a = run("L2b", a)
    u1 = run("U1", a)
    d1 = run("D1", np.concatenate([u1, s1], axis=-1))
    u0 = run("U0", d1)
    d0 = run("D0", np.concatenate([u0, s0], axis=-1))
    y = run("H", d0)
    return y[..., 0], cache


def backward(theta, cache, dy):
    """Adjoint of `forward`: returns (dtheta flat, dX)."""
    P = unflatten(theta)
    idx = {name: i for i, (name, *_r) in enumerate(LAYERS)}
    grads = [None] * len(LAYERS)

    def back(name, dout):
        i = idx[name]
        _, kind, _, _, relu = LAYERS[i]
        inp, z = cache[name]
        dz = dout * (z > 0.0) if relu else dout
        dx, dw, db = _backward(kind, inp, P[i][0], dz)
        grads[i] = (dw, db)
        return dx

    d = back("H", dy[..., None])
    dcat0 = back("D0", d)
    du0, ds0 = dcat0[..., :16], dcat0[..., 16:]
    dd1 = back("U0", du0)
    dcat1 = back("D1", dd1)
    du1, ds1 = dcat1[..., :32], dcat1[..., 32:]
    da = back("U1", du1)
    da = back("L2b", da)
    ds1 = ds1 + back("L2a", da)
    da = back("L1b", ds1)
    ds0 = ds0 + back("L1a", da)
    da = back("L0b", ds0)
    dX = back("L0a", da)
    return flatten(grads), dX


def init_params(seed: int):
    """Kaiming-uniform (fan-in, gain sqrt(2)) weights for ReLU layers, gain 1
    for the linear ones, zero biases; numpy PCG64 stream seeded by `seed`."""
    from numpy.random import Generator, PCG64
    rng = Generator(PCG64(seed))
    parts = []
    for (name, kind, cin, cout, relu), (nw, nb) in zip(LAYERS, layer_sizes()):
        fan_in = nw // cout
        bound = math.sqrt(6.0 / fan_in) if relu else math.sqrt(3.0 / fan_in)
        parts.append(rng.uniform(-bound, bound, nw))
        parts.append(np.zeros(nb))
    return np.concatenate(parts)


# --------------------------------------------------------------------------
# training objective (Section 5.1 empirical risk) and Adam
# --------------------------------------------------------------------------

def sample_loss(theta, C, r, dist, alpha, boundary):
    """|| r - alpha^-1 C mask(U([r, d])) ||^2 for one unit-norm sample r.

    C = A00, the 3D block of the assembled operator; mask sets the Dirichlet
    entries of the network output to zero (those rows of C are the identity
    and r vanishes there).  Returns (loss, dtheta).
    """
    n = round(len(r) ** (1.0 / 3.0))
    X = np.stack([r.reshape(n, n, n), dist.reshape(n, n, n)], axis=-1)
    U, cache = forward(theta, X)
    u = U.reshape(-1).copy()
    u[boundary] = 0.0
    e = r - (C @ u) / alpha
    loss = float(e @ e)
    gu = -2.0 * (C.T @ e) / alpha
    gu[boundary] = 0.0
    dtheta, _ = backward(theta, cache, gu.reshape(n, n, n))
    return loss, dtheta


def adam_step(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; step counts from 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
