"""Pins of the E4M3 weight quantisation oracle (oracle/fp8.py): the value set
against the format's published constants, rounding against PyTorch's own
float8_e4m3fn conversion (a library routine), and the per-channel
power-of-two scales against their defining inequality."""
import numpy as np
import pytest
import torch

from oracle import cnn, fp8


def test_table_constants():
    t = fp8.e4m3_table()
    fin = t[np.isfinite(t)]
    assert len(fin) == 254                       # 256 codes minus the two NaNs
    assert np.max(fin) == 448.0 and np.min(fin) == -448.0
    pos = fin[fin > 0]
    assert np.min(pos) == 2.0 ** -9              # smallest subnormal
    assert t[0x08] == 2.0 ** -6                  # smallest normal
    assert t[0x38] == 1.0 and t[0x39] == 1.125   # exponent field 7 = bias
    assert np.all(np.diff(t[:0x7F]) > 0)         # codes 0 .. 0x7E ascend


def test_rounding_matches_torch():
    rng = np.random.default_rng(3)
    pos = fp8.e4m3_table()[:0x7F]
    mids = pos[:-1] + np.diff(pos) / 2           # every tie
    x = np.concatenate([rng.uniform(-448, 448, 50000), rng.normal(0, 0.02, 50000),
                        rng.normal(0, 1e-3, 20000), mids, -mids, pos, -pos])
    ref = torch.tensor(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(fp8.round_e4m3(x), ref)


def test_saturation_and_fixed_points():
    assert fp8.round_e4m3(1000.0) == 448.0 and fp8.round_e4m3(-1e6) == -448.0
    assert fp8.round_e4m3(464.0) == 448.0        # above the last tie: saturates, not NaN
    pos = fp8.e4m3_table()[:0x7F]
    assert np.array_equal(fp8.round_e4m3(pos), pos)


@pytest.mark.parametrize("amax", [1e-7, 3e-3, 0.37, 1.0, 447.9, 448.0, 448.1, 2e4])
def test_channel_scale(amax):
    sc = fp8.channel_scale(amax)
    k = np.log2(sc)
    assert k == np.round(k)                      # a power of two
    assert amax / sc <= 448.0 < amax / (sc / 2)  # the smallest such


def test_quantize_weights():
    theta = cnn.init_params(11)
    q = fp8.quantize_weights(theta)
    P, Q = cnn.unflatten(theta), cnn.unflatten(q)
    for (w, b), (wq, bq) in zip(P, Q):
        assert np.array_equal(b, bq)
        for o in range(w.shape[0]):
            sc = fp8.channel_scale(float(np.max(np.abs(w[o]))))
            codes = wq[o] / sc
            assert np.array_equal(fp8.round_e4m3(codes), codes)   # code * scale exactly
            big = np.abs(w[o] / sc) >= 2.0 ** -6                   # normal range: half an ulp
            assert np.all(np.abs(wq[o] - w[o])[big] <= 2.0 ** -4 * np.abs(w[o])[big])
        # exact in BF16: the BF16 network computes with the E4M3 values themselves
        bf = torch.tensor(wq.ravel()).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(bf, wq.ravel())


# ---------------------------------------------------------------- E4M3 activations

def _net9():
    th = cnn.init_params(3)
    thq = fp8.quantize_weights(th)
    X = np.random.default_rng(0).standard_normal((9, 9, 9, 2)) * 0.05
    return thq, X


def test_forward_fp8_without_rounding_is_the_network():
    """With the quantiser replaced by the identity, the E4M3-activation
    forward is exactly the full-precision network (wiring pin)."""
    thq, X = _net9()
    sc = fp8.activation_scales(thq, [X])
    y_id = fp8.forward_fp8(thq, X, sc, quant=lambda t, s: t)
    y = cnn.forward(thq, X)[0]
    assert np.array_equal(y_id, y)


def test_forward_fp8_quantises_every_read_tensor_with_its_scale():
    """The quantiser is called once per tensor a 3x3x3 layer reads, in the
    order X, L0a, ..., D0, each with its own scale."""
    thq, X = _net9()
    sc = [2.0 ** -(k + 1) for k in range(len(fp8.ACT_NAMES))]
    seen = []

    def rec(t, s):
        seen.append(s)
        return fp8.quantize_act(t, s)
    fp8.forward_fp8(thq, X, sc, quant=rec)
    assert seen == sc


def test_activation_scales_rule():
    """Scales are powers of two, the stacked pairs share one, and each is the
    smallest with 2 amax / s <= 448 (amax from the full-precision network)."""
    thq, X = _net9()
    sc = dict(zip(fp8.ACT_NAMES, fp8.activation_scales(thq, [X])))
    _, cache = cnn.forward(thq, X)
    relu = {nm: r for (nm, _k, _ci, _co, r) in cnn.LAYERS}
    amax = {"X": float(np.abs(X).max())}
    for nm in fp8.ACT_NAMES[1:]:
        z = cache[nm][1]
        amax[nm] = float(np.abs(np.maximum(z, 0.0) if relu[nm] else z).max())
    for a, b in fp8.TIED:
        amax[a] = amax[b] = max(amax[a], amax[b])
        assert sc[a] == sc[b]
    for nm, s in sc.items():
        k = np.log2(s)
        assert k == np.round(k)
        assert 2 * amax[nm] / s <= 448.0 < 2 * amax[nm] / (s / 2)


def test_forward_fp8_error_bound():
    """E4M3 activations and weights stay within the 1e-1 relative (2-norm)
    error budget of an 8-bit network against the full-precision one."""
    thq, X = _net9()
    sc = fp8.activation_scales(thq, [X])
    y8 = fp8.forward_fp8(thq, X, sc)
    y = cnn.forward(thq, X)[0]
    assert np.linalg.norm(y8 - y) / np.linalg.norm(y) <= 1e-1
