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
