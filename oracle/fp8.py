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
