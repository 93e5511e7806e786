"""Pins of the oracle U-net (Section 4.2) and training objective (Section 5.1)."""
import itertools
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as Fnn

import synth
from oracle import cnn, fem


def brute_conv(x, w, b, stride):
    n, cin = x.shape[0], x.shape[3]
    cout = w.shape[0]
    no = (n - 1) // stride + 1
    y = np.zeros((no, no, no, cout))
    for pz, py, px in itertools.product(range(no), repeat=3):
        for o in range(cout):
            acc = b[o]
            for t, (tz, ty, tx) in enumerate(cnn.taps3()):
                z, yy, xx = stride * pz + tz - 1, stride * py + ty - 1, stride * px + tx - 1
                if 0 <= z < n and 0 <= yy < n and 0 <= xx < n:
                    for c in range(cin):
                        acc += w[o, t, c] * x[z, yy, xx, c]
            y[pz, py, px, o] = acc
    return y


def brute_tconv(x, w, b):
    n, cin = x.shape[0], x.shape[3]
    cout = w.shape[0]
    no = 2 * n - 1
    y = np.tile(b, (no, no, no, 1)).astype(np.float64)
    for iz, iy, ix in itertools.product(range(n), repeat=3):
        for t, (tz, ty, tx) in enumerate(cnn.taps3()):
            oz, oy, ox = 2 * iz + tz - 1, 2 * iy + ty - 1, 2 * ix + tx - 1
            if 0 <= oz < no and 0 <= oy < no and 0 <= ox < no:
                y[oz, oy, ox] += w[:, t, :] @ x[iz, iy, ix]
    return y


@pytest.fixture
def rng():
    return np.random.default_rng(123)


def test_param_count():
    assert cnn.n_params() == 353713


def test_paper_unet_table_counting():
    """The paper's U_3 table rows 2-5 re-derive as bias-free 27 Cin Cout (convolutions)
    and 8 Cin Cout + Cout + 27 (2 Cout) Cout (transposed conv + skip block)."""
    assert 27 * 32 * 64 == 55296
    assert 27 * 64 * 128 == 221184
    assert 27 * 128 * 128 == 442368
    assert 8 * 128 * 64 + 64 + 27 * 128 * 64 == 286784


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_brute_force(rng, stride):
    x = rng.normal(size=(5, 5, 5, 3))
    w = rng.normal(size=(4, 27, 3))
    b = rng.normal(size=4)
    assert np.allclose(cnn.conv3d(x, w, b, stride), brute_conv(x, w, b, stride), atol=1e-12)


def test_tconv_brute_force(rng):
    x = rng.normal(size=(3, 3, 3, 3))
    w = rng.normal(size=(2, 27, 3))
    b = rng.normal(size=2)
    assert np.allclose(cnn.tconv3d(x, w, b), brute_tconv(x, w, b), atol=1e-12)


def _torch_w(w):
    co, _, ci = w.shape
    return torch.from_numpy(w.reshape(co, 3, 3, 3, ci).transpose(0, 4, 1, 2, 3).copy())


def test_conv_matches_torch_library(rng):
    """Library pin: torch.nn.functional.conv3d / conv_transpose3d in float64 on CPU."""
    x = rng.normal(size=(9, 9, 9, 5))
    w = rng.normal(size=(6, 27, 5))
    b = rng.normal(size=6)
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2)[None].copy())
    for s in (1, 2):
        ref = Fnn.conv3d(xt, _torch_w(w), torch.from_numpy(b), stride=s, padding=1)
        ref = ref[0].numpy().transpose(1, 2, 3, 0)
        assert np.allclose(cnn.conv3d(x, w, b, s), ref, atol=1e-11)
    # conv_transpose3d weight is [Cin, Cout, k, k, k]
    wt = torch.from_numpy(w.reshape(6, 3, 3, 3, 5).transpose(4, 0, 1, 2, 3).copy())
    ref = Fnn.conv_transpose3d(xt, wt, torch.from_numpy(b), stride=2, padding=1)
    ref = ref[0].numpy().transpose(1, 2, 3, 0)
    assert np.allclose(cnn.tconv3d(x, w, b), ref, atol=1e-11)


def test_delta_kernel_is_identity(rng):
    x = rng.normal(size=(7, 7, 7, 3))
    w = np.zeros((3, 27, 3))
    for c in range(3):
        w[c, 13, c] = 1.0
    assert np.array_equal(cnn.conv3d(x, w, np.zeros(3), 1), x)


def test_adjointness(rng):
    """<conv_s(x), y> = <x, conv_s^T(y)>: the stride-2 transposed conv with swapped
    channel roles is the adjoint of the stride-2 conv, and the backward-data
    routines are adjoints of the forward maps."""
    x = rng.normal(size=(9, 9, 9, 4))
    w = rng.normal(size=(3, 27, 4))
    y = rng.normal(size=(5, 5, 5, 3))
    lhs = np.sum(cnn.conv3d(x, w, np.zeros(3), 2) * y)
    wT = np.transpose(w, (2, 1, 0)).copy()          # [Cin, taps, Cout]
    rhs = np.sum(x * cnn.tconv3d(y, wT, np.zeros(4)))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    for stride, yshape in ((1, (9, 9, 9, 3)), (2, (5, 5, 5, 3))):
        y = rng.normal(size=yshape)
        dx, _, _ = cnn.conv3d_backward(x, w, y, stride)
        assert np.sum(cnn.conv3d(x, w, np.zeros(3), stride) * y) == pytest.approx(np.sum(x * dx), rel=1e-12)
    xs = rng.normal(size=(5, 5, 5, 4))
    y = rng.normal(size=(9, 9, 9, 3))
    dx, _, _ = cnn.tconv3d_backward(xs, w, y)
    assert np.sum(cnn.tconv3d(xs, w, np.zeros(3)) * y) == pytest.approx(np.sum(xs * dx), rel=1e-12)


def with_biases(theta, seed, scale=0.2):
    """Random non-zero biases, so that no ReLU pre-activation sits exactly at 0."""
    th = theta.copy()
    off = 0
    for i, (a, b) in enumerate(cnn.layer_sizes()):
        th[off + a:off + a + b] = np.random.default_rng(seed + i).uniform(-scale, scale, b)
        off += a + b
    return th


def relu_signs(theta, X):
    _, c = cnn.forward(theta, X)
    return np.concatenate([(c[name][1] > 0).ravel() for name, _, _, _, relu in cnn.LAYERS if relu])


def test_network_gradient_finite_differences(rng):
    """Central differences (eps 1e-4, FP64) of a scalar functional of U along random
    parameter directions; directions whose perturbation flips a ReLU sign are skipped."""
    theta = with_biases(cnn.init_params(5) * 0.3, 50)
    X = np.stack([rng.normal(size=(9, 9, 9)) / 27.0, rng.uniform(0, 0.5, size=(9, 9, 9))], axis=-1)
    G = rng.normal(size=(9, 9, 9))
    f = lambda th: float(np.sum(cnn.forward(th, X)[0] * G))
    _, cache = cnn.forward(theta, X)
    g, dX = cnn.backward(theta, cache, G)
    eps = 1e-4
    done = 0
    for k in range(16):
        d = rng.normal(size=theta.size)
        d /= np.linalg.norm(d)
        s0 = relu_signs(theta, X)
        if not (np.array_equal(relu_signs(theta + eps * d, X), s0)
                and np.array_equal(relu_signs(theta - eps * d, X), s0)):
            continue
        fd = (f(theta + eps * d) - f(theta - eps * d)) / (2 * eps)
        assert fd == pytest.approx(g @ d, rel=1e-7, abs=1e-10)
        done += 1
    assert done >= 6
    dXd = rng.normal(size=X.shape)
    dXd /= np.linalg.norm(dXd)
    fx = lambda XX: float(np.sum(cnn.forward(theta, XX)[0] * G))
    fd = (fx(X + eps * dXd) - fx(X - eps * dXd)) / (2 * eps)
    assert fd == pytest.approx(np.sum(dX * dXd), rel=1e-5, abs=1e-8)


def _small_system():
    inst = synth.make_instance(7, 8, n_segments=20, elems_per_segment=4, radius=0.01, beta=1.0)
    return fem.assemble(inst)


def _unit_interior(s, seed):
    r = synth.fast_normal(seed, s.n3d)
    r[s.boundary] = 0.0
    return r / np.linalg.norm(r)


def test_zero_network_loss_is_one():
    s = _small_system()
    A00 = s.blocks()[0]
    r = _unit_interior(s, 1)
    loss, g = cnn.sample_loss(np.zeros(cnn.n_params()), A00, r, s.dist, s.alpha, s.boundary)
    assert loss == pytest.approx(1.0, abs=1e-15)


def test_loss_gradient_finite_differences():
    """Gradient of || r - alpha^-1 C U([r, d]) ||^2 on the 8^3-cell copy, eps 1e-3, FP64."""
    s = _small_system()
    A00 = s.blocks()[0]
    r = _unit_interior(s, 2)
    rng = np.random.default_rng(9)
    theta = with_biases(cnn.init_params(2) * 0.3, 70)
    n = 9
    X = np.stack([r.reshape(n, n, n), s.dist.reshape(n, n, n)], axis=-1)
    loss, g = cnn.sample_loss(theta, A00, r, s.dist, s.alpha, s.boundary)
    eps = 1e-3
    ok = 0
    s0 = relu_signs(theta, X)
    for k in range(10):
        d = rng.normal(size=theta.size)
        d /= np.linalg.norm(d)
        if not (np.array_equal(relu_signs(theta + eps * d, X), s0)
                and np.array_equal(relu_signs(theta - eps * d, X), s0)):
            continue
        lp = cnn.sample_loss(theta + eps * d, A00, r, s.dist, s.alpha, s.boundary)[0]
        lm = cnn.sample_loss(theta - eps * d, A00, r, s.dist, s.alpha, s.boundary)[0]
        fd = (lp - lm) / (2 * eps)
        # the loss is quadratic in U: central differences are exact up to third-order terms
        assert fd == pytest.approx(g @ d, rel=1e-6, abs=1e-10)
        ok += 1
    assert ok >= 5


def test_adam_first_step_closed_form():
    """After one step, m_hat = g and v_hat = g^2, so the update is lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = cnn.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


class _TorchUNet(torch.nn.Module):
    """The U-net of Section 4.2 as a torch.nn composition in float64, written
    from the layer table (three levels of 16 / 32 / 64 channels, 3x3x3 kernels
    with padding 1, stride-2 convolutions down, stride-2 transposed
    convolutions up, skip connections by stacking [upsampled | skip] on the
    channel axis, ReLU after every convolution except the transposed ones and
    the 1x1 head).  It shares nothing with the oracle's loops: a library pin of
    the whole wiring."""

    def __init__(self):
        super().__init__()
        C3 = lambda ci, co, s: torch.nn.Conv3d(ci, co, 3, stride=s, padding=1, dtype=torch.float64)
        T3 = lambda ci, co: torch.nn.ConvTranspose3d(ci, co, 3, stride=2, padding=1, dtype=torch.float64)
        self.l0a, self.l0b = C3(2, 16, 1), C3(16, 16, 1)
        self.l1a, self.l1b = C3(16, 32, 2), C3(32, 32, 1)
        self.l2a, self.l2b = C3(32, 64, 2), C3(64, 64, 1)
        self.u1, self.d1 = T3(64, 32), C3(64, 32, 1)
        self.u0, self.d0 = T3(32, 16), C3(32, 16, 1)
        self.head = torch.nn.Conv3d(16, 1, 1, dtype=torch.float64)

    def load_flat(self, theta):
        """Flat order: per layer [Cout][kz][ky][kx][Cin] then the bias."""
        off = 0
        for m in (self.l0a, self.l0b, self.l1a, self.l1b, self.l2a, self.l2b, self.u1, self.d1, self.u0,
                  self.d0, self.head):
            if isinstance(m, torch.nn.ConvTranspose3d):
                ci, co, k = m.weight.shape[0], m.weight.shape[1], m.weight.shape[2]
            else:
                co, ci, k = m.weight.shape[0], m.weight.shape[1], m.weight.shape[2]
            nw = co * k ** 3 * ci
            w = torch.from_numpy(np.asarray(theta[off:off + nw]).reshape(co, k, k, k, ci).copy())
            off += nw
            with torch.no_grad():
                if isinstance(m, torch.nn.ConvTranspose3d):
                    m.weight.copy_(w.permute(4, 0, 1, 2, 3))   # [Cin][Cout][kz][ky][kx]
                else:
                    m.weight.copy_(w.permute(0, 4, 1, 2, 3))   # [Cout][Cin][kz][ky][kx]
                m.bias.copy_(torch.from_numpy(np.asarray(theta[off:off + co]).copy()))
            off += co
        assert off == theta.size

    def forward(self, x):                      # x [B, 2, z, y, x]
        r = torch.relu
        s0 = r(self.l0b(r(self.l0a(x))))
        s1 = r(self.l1b(r(self.l1a(s0))))
        bott = r(self.l2b(r(self.l2a(s1))))
        d1 = r(self.d1(torch.cat([self.u1(bott), s1], dim=1)))
        d0 = r(self.d0(torch.cat([self.u0(d1), s0], dim=1)))
        return self.head(d0)[:, 0]


@pytest.mark.parametrize("n", [5, 9, 13])
def test_network_wiring_matches_torch_composition(n):
    """Whole-network forward of the oracle against the torch.nn composition on
    random weights with non-zero biases (every layer's bias and the
    concatenation order of both skips matter: swapping [up | skip] or dropping
    a ReLU changes the output by far more than the tolerance)."""
    rng = np.random.default_rng(100 + n)
    theta = cnn.init_params(n)
    off = 0
    for nw, nb in cnn.layer_sizes():
        theta[off + nw:off + nw + nb] = rng.uniform(-0.1, 0.1, nb)
        off += nw + nb
    X = np.stack([rng.normal(size=(n, n, n)), rng.uniform(0, 1, (n, n, n))], axis=-1)
    net = _TorchUNet()
    net.load_flat(theta)
    with torch.no_grad():
        ref = net(torch.from_numpy(X.transpose(3, 0, 1, 2)[None].copy()))[0].numpy()
    got = cnn.forward(theta, X)[0]
    assert got.shape == (n, n, n)
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    # a wrong wiring is visible: the composition with swapped skip order differs
    W = net.d0.weight.detach().clone()
    with torch.no_grad():
        net.d0.weight.copy_(torch.cat([W[:, 16:], W[:, :16]], dim=1))
        bad = net(torch.from_numpy(X.transpose(3, 0, 1, 2)[None].copy()))[0].numpy()
    assert np.linalg.norm(bad - got) > 1e-3 * np.linalg.norm(got)


def test_network_gradient_matches_torch_autograd():
    """Backward of the oracle (weights and input) against torch autograd
    through the same torch.nn composition, float64."""
    n = 9
    rng = np.random.default_rng(5)
    theta = cnn.init_params(3)
    off = 0
    for nw, nb in cnn.layer_sizes():
        theta[off + nw:off + nw + nb] = rng.uniform(-0.1, 0.1, nb)
        off += nw + nb
    X = np.stack([rng.normal(size=(n, n, n)), rng.uniform(0, 1, (n, n, n))], axis=-1)
    G = rng.normal(size=(n, n, n))
    net = _TorchUNet()
    net.load_flat(theta)
    xt = torch.from_numpy(X.transpose(3, 0, 1, 2)[None].copy()).requires_grad_(True)
    y = net(xt)[0]
    (y * torch.from_numpy(G)).sum().backward()
    _, cache = cnn.forward(theta, X)
    dtheta, dX = cnn.backward(theta, cache, G)
    assert np.allclose(dX, xt.grad[0].numpy().transpose(1, 2, 3, 0), rtol=1e-10, atol=1e-12)
    off = 0
    for m, (nw, nb) in zip((net.l0a, net.l0b, net.l1a, net.l1b, net.l2a, net.l2b, net.u1, net.d1, net.u0,
                            net.d0, net.head), cnn.layer_sizes()):
        g = m.weight.grad
        g = g.permute(1, 2, 3, 4, 0) if isinstance(m, torch.nn.ConvTranspose3d) else g.permute(0, 2, 3, 4, 1)
        assert np.allclose(dtheta[off:off + nw], g.reshape(-1).numpy(), rtol=1e-10, atol=1e-12)
        assert np.allclose(dtheta[off + nw:off + nw + nb], m.bias.grad.numpy(), rtol=1e-10, atol=1e-12)
        off += nw + nb


def test_round_bf16_matches_torch_conversion():
    """The oracle's bfloat16 rounding against PyTorch's own float32 -> bfloat16
    conversion: 200k random values over many decades, every exact tie between
    two neighbouring bfloat16 values (both parities) and signed zeros."""
    rng = np.random.default_rng(5)
    x = rng.normal(size=200_000) * 10.0 ** rng.uniform(-30, 30, 200_000)
    x = x.astype(np.float32).astype(np.float64)
    hi = rng.integers(0, 0x7F7F, 5000, dtype=np.uint32) << 16                  # finite, below the largest
    ties = (hi | 0x8000).view(np.float32).astype(np.float64)          # halfway between two bf16 values
    vals = np.concatenate([x, ties, -ties, [0.0, -0.0, 1.0, 3.0e38]])
    want = torch.from_numpy(vals.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = cnn.round_bf16(vals)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_bf16_emulation_rounds_where_stated():
    """forward(emulate="bf16"): every stored activation except the head output
    is a bfloat16 value, the network input is rounded, the result stays within
    a few BF16 rounding steps of the FP64 network, and the adjoint of the
    emulated network passes the same central-difference check in the weights
    of the 1x1 head (linear there, so the check is exact up to FP64 rounding)."""
    n = 9
    rng = np.random.default_rng(9)
    th = cnn.init_params(4)
    X = np.stack([rng.normal(size=(n, n, n)), rng.uniform(0, 1, (n, n, n))], axis=-1)
    y64, _ = cnn.forward(th, X)
    y16, cache = cnn.forward(th, X, emulate="bf16")
    assert np.array_equal(cache["X"], cnn.round_bf16(X))
    for name, *_r in cnn.LAYERS[:-1]:
        inp, z = cache[name]
        assert np.array_equal(inp, cnn.round_bf16(inp)), name
    rel = np.linalg.norm(y16 - y64) / np.linalg.norm(y64)
    assert 1e-5 < rel < 5e-2, rel
    G = rng.normal(size=(n, n, n))
    g, _ = cnn.backward(th, cache, G)
    off = cnn.n_params() - 17                      # head weights (16) and bias (1)
    for j in range(17):
        e = np.zeros_like(th)
        e[off + j] = 1e-3
        fp = np.sum(G * cnn.forward(th + e, X, emulate="bf16")[0])
        fm = np.sum(G * cnn.forward(th - e, X, emulate="bf16")[0])
        assert (fp - fm) / 2e-3 == pytest.approx(g[off + j], rel=1e-9, abs=1e-9)
