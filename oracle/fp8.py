"""FP8 (E4M3) weights of the U-net preconditioner (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs its network in full precision and says nothing about 8-bit
formats; the reduced-precision variant here stores the weights of the network
of Section 4.2 in the OCP 8-bit floating-point format E4M3 (1 sign bit, 4
exponent bits with bias 7, 3 mantissa bits; exponent field 0 holds the
subnormals m/8 * 2^-6; the all-ones pattern S.1111.111 is NaN, so there is no
infinity and the largest finite magnitude is 1.75 * 2^8 = 448).

Readings (the paper fixes none of this):
  * each output channel of each layer (the taps x input channels it reads) has
    one scale, a power of two: the smallest 2^k with amax / 2^k <= 448, so that
    code * scale is exact in BF16 and the network's BF16 products are those of
    the E4M3 weights;
  * rounding is to nearest, ties to the code with even mantissa; the biases
    stay in full precision.

The value set is built from the bit fields and rounding searches it, so this
module shares nothing with a formula-based converter.
"""
from __future__ import annotations

import numpy as np

from . import cnn

E4M3_MAX = 448.0


def e4m3_table():
    """All finite E4M3 values by code 0..255 (NaN codes give nan)."""
    vals = np.empty(256, dtype=np.float64)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            vals[code] = np.nan
        elif e == 0:
            vals[code] = s * (m / 8.0) * 2.0 ** -6
        else:
            vals[code] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return vals


_TABLE = e4m3_table()
# non-negative finite values with their codes, ascending (codes 0x00 .. 0x7E)
_POS = _TABLE[:0x7F]


def round_e4m3(x):
    """Round to the nearest E4M3 value, ties to even mantissa, saturating at
    +-448 (values beyond the largest finite magnitude clamp to it)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    hi = np.searchsorted(_POS, a, side="left")          # first value >= a
    hi = np.minimum(hi, len(_POS) - 1)
    lo = np.maximum(hi - 1, 0)
    dlo = a - _POS[lo]
    dhi = _POS[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))  # even code = even mantissa bit
    q = np.where(pick_hi, _POS[hi], _POS[lo])
    return np.sign(x) * q


def channel_scale(amax):
    """Smallest power of two 2^k with amax / 2^k <= 448 (1 for amax = 0)."""
    if amax == 0.0:
        return 1.0
    k = int(np.ceil(np.log2(amax / E4M3_MAX)))
    while amax / 2.0 ** k > E4M3_MAX:   # guard against log2 rounding
        k += 1
    while k > -200 and amax / 2.0 ** (k - 1) <= E4M3_MAX:
        k -= 1
    return 2.0 ** k


def quantize_weights(theta):
    """Flat parameter vector -> the same with every layer's weights replaced by
    code * scale (per output channel), biases unchanged."""
    params = cnn.unflatten(np.asarray(theta, dtype=np.float64))
    out = []
    for w, b in params:
        wq = np.empty_like(w)
        for o in range(w.shape[0]):
            sc = channel_scale(float(np.max(np.abs(w[o]))))
            wq[o] = round_e4m3(w[o] / sc) * sc
        out.append((wq, b.copy()))
    return cnn.flatten(out)


# ---------------------------------------------------------------- E4M3 activations
#
# Further readings for the variant that also stores the network's activations
# in E4M3 (again the paper fixes none of this):
#   * every tensor a 3x3x3 layer reads is quantised: the input X and the
#     output of each of the ten 3x3x3 layers (after its ReLU), each with one
#     power-of-two scale per tensor: t -> round_e4m3(t / s) * s;
#   * the two tensors stacked into one layer input share one scale (the
#     up-sampled U1 with the skip L1b, U0 with L0b);
#   * the 1x1 head reads the quantised D0 output and stays in full precision,
#     as do the biases and the products and sums of every layer;
#   * calibration: s is the smallest power of two with 2 amax / s <= 448, amax
#     the largest magnitude of the tensor in the full-precision network on a
#     sample input (for a stacked pair: over both tensors), leaving a factor two
#     of headroom for inputs whose activations are larger than the sample's.

ACT_NAMES = ("X", "L0a", "L0b", "L1a", "L1b", "L2a", "L2b", "U1", "D1", "U0", "D0")
TIED = (("L1b", "U1"), ("L0b", "U0"))
HEADROOM = 2.0


def quantize_act(t, s):
    """t -> E4M3 code * s for a tensor with scale s."""
    return round_e4m3(np.asarray(t, dtype=np.float64) / s) * s


def forward_fp8(theta_q, X, scales, quant=quantize_act):
    """U(X) for one sample X [n, n, n, 2] with E4M3 activations: theta_q is
    already on the per-channel E4M3 grid (`quantize_weights`), `scales` holds
    one scale per name in ACT_NAMES; returns [n, n, n].  `quant(t, s)` is the
    quantiser (replaceable, so that tests can check the wiring without it)."""
    n = X.shape[0]
    cnn.check_grid(n)
    P = cnn.unflatten(np.asarray(theta_q, dtype=np.float64))
    sc = dict(zip(ACT_NAMES, scales))
    idx = {name: i for i, (name, *_r) in enumerate(cnn.LAYERS)}

    def run(name, inp):
        i = idx[name]
        _, kind, _, _, relu = cnn.LAYERS[i]
        z = cnn._apply(kind, inp, *P[i])
        out = np.maximum(z, 0.0) if relu else z
        return out if kind == "point" else quant(out, sc[name])

    a = run("L0a", quant(X, sc["X"]))
    s0 = run("L0b", a)
    a = run("L1a", s0)
    s1 = run("L1b", a)
    a = run("L2a", s1)
    a = run("L2b", a)
    u1 = run("U1", a)
    d1 = run("D1", np.concatenate([u1, s1], axis=-1))
    u0 = run("U0", d1)
    d0 = run("D0", np.concatenate([u0, s0], axis=-1))
    return run("H", d0)[..., 0]


def activation_scales(theta_q, Xs, headroom=HEADROOM):
    """Calibrated scales (one per ACT_NAMES entry) from the full-precision
    network on the sample inputs Xs (a list of [n, n, n, 2] arrays)."""
    amax = dict.fromkeys(ACT_NAMES, 0.0)
    for X in Xs:
        _, cache = cnn.forward(np.asarray(theta_q, dtype=np.float64), X)
        amax["X"] = max(amax["X"], float(np.max(np.abs(cache["X"]))))
        for name in ACT_NAMES[1:]:
            relu = next(r for (nm, _k, _ci, _co, r) in cnn.LAYERS if nm == name)
            z = cache[name][1]
            out = np.maximum(z, 0.0) if relu else z
            amax[name] = max(amax[name], float(np.max(np.abs(out))))
    for a, b in TIED:
        amax[a] = amax[b] = max(amax[a], amax[b])
    return [channel_scale(headroom * amax[name]) for name in ACT_NAMES]
