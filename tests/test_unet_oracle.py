"""Pins of the U-Net reference (oracle/unet_ref.py) against mathematics:
shifts, the convolution theorem, adjoint identities, finite-difference
gradients, bfloat16 rounding values and the closed form of Adam's first step."""
import numpy as np
import pytest

from oracle import unet_ref as U


def test_delta_kernel_is_a_periodic_shift():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((8, 8, 8, 3))
    for t, d in enumerate(U.taps()):
        W = np.zeros((27, 3, 3))
        W[t] = np.eye(3)
        y = U.conv3(x, W)
        # y[i, j, k] = x[i + di, j + dj, k + dk]
        i, j, k = 2, 7, 0
        assert np.allclose(y[i, j, k], x[(i + d[0]) % 8, (j + d[1]) % 8, (k + d[2]) % 8])
    assert U.taps()[0] == (-1, -1, -1) and U.taps()[13] == (0, 0, 0) and U.taps()[26] == (1, 1, 1)


def test_convolution_theorem():
    """Single channel: y[v] = sum_d w[d] x[v + d] is a circular correlation,
    computed independently with FFTs."""
    rng = np.random.default_rng(1)
    n = 8
    x = rng.standard_normal((n, n, n))
    w = rng.standard_normal(27)
    W = w.reshape(27, 1, 1)
    y = U.conv3(x[..., None], W)[..., 0]
    g = np.zeros((n, n, n))
    for t, d in enumerate(U.taps()):
        g[(-d[0]) % n, (-d[1]) % n, (-d[2]) % n] += w[t]
    y_fft = np.real(np.fft.ifftn(np.fft.fftn(x) * np.fft.fftn(g)))
    assert np.max(np.abs(y - y_fft)) < 1e-12


def test_conv_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((8, 8, 8, 5))
    dy = rng.standard_normal((8, 8, 8, 7))
    W = rng.standard_normal((27, 7, 5))
    dW = rng.standard_normal((27, 7, 5))
    lhs = np.sum(U.conv3(x, W) * dy)
    assert abs(lhs - np.sum(x * U.conv3_bwd_data(dy, W))) < 1e-10 * abs(lhs)
    lhs = np.sum(U.conv3(x, dW) * dy)
    assert abs(lhs - np.sum(dW * U.conv3_bwd_weight(x, dy))) < 1e-10 * abs(lhs)


def test_pool_up_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((8, 8, 8, 2))
    y = rng.standard_normal((4, 4, 4, 2))
    assert abs(np.sum(U.pool2(x) * y) - np.sum(x * U.pool2_bwd(y))) < 1e-12
    assert abs(np.sum(U.up2(y) * x) - np.sum(y * U.up2_bwd(x))) < 1e-12
    assert np.allclose(U.pool2(U.up2(y)), y)


def test_bf16_rounding():
    assert U.bf16(1.0) == 1.0
    assert U.bf16(1.0 + 2 ** -8) == 1.0                 # tie -> even
    assert U.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6   # tie -> even (up)
    assert U.bf16(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7
    assert U.bf16(-2.5) == -2.5
    assert U.bf16(3.0e38) == np.float32(3.0e38).astype(np.float64) or np.isfinite(U.bf16(3.0e38))
    assert np.isnan(U.bf16(np.nan))


def test_param_count_and_layout():
    assert U.param_count() == sum(27 * ci * co + co for ci, co in U.CONVS) + 17
    assert 850_000 < U.param_count() < 950_000
    p = np.arange(U.param_count(), dtype=float)
    convs, (wh, bh) = U.split_params(p)
    assert convs[0][0].shape == (27, 16, 16) and convs[8][0].shape == (27, 64, 128)
    assert bh[0] == U.param_count() - 1 and wh[0] == U.param_count() - 17


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    eta = np.exp(rng.standard_normal((n, n, n)))
    cold = np.sqrt(np.maximum(0.0, 1 - 0.2 * eta))
    target = 0.1 * rng.standard_normal((n, n, n))
    return U.make_input(eta, 0.8, cold), target


def test_network_gradient_finite_differences():
    """FP64 gradient of the MSE vs central differences, per parameter block
    and along random directions, with the ReLU pattern frozen at the base
    point (then the loss is a polynomial in the parameters)."""
    n = 8
    x, target = _inputs(n, 4)
    p = U.init_params(5)
    p[-1] = 0.3
    out, cache = U.forward(p, x)
    g = U.backward(p, cache, out, target)

    def loss(pp):
        return U.mse(U.forward(pp, x, masks=cache)[0], target)

    rng = np.random.default_rng(6)
    blocks, off = [], 0
    for ci, co in U.CONVS:
        blocks.append((off, off + 27 * ci * co + co))
        off += 27 * ci * co + co
    blocks.append((off, off + 17))
    blocks.append((0, p.size))
    for a, b in blocks:
        d = np.zeros(p.size)
        d[a:b] = rng.standard_normal(b - a)
        # the loss has degree ~30 along an all-parameter direction: smaller step
        eps = 1e-4 if b - a < p.size else 1e-6
        fd = (loss(p + eps * d) - loss(p - eps * d)) / (2 * eps)
        an = float(g @ d)
        assert abs(fd - an) <= 1e-6 * abs(fd), (a, b, fd, an)


def test_bf16_emulation_is_close_to_fp64():
    n = 8
    x, target = _inputs(n, 7)
    p = U.init_params(8)
    o64, _ = U.forward(p, x)
    o16, _ = U.forward(p, x, bf=True)
    assert np.linalg.norm(o16 - o64) / np.linalg.norm(o64) < 3e-2


def test_adam_first_step_closed_form():
    """With m = v = 0, the bias-corrected first step is lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    p = np.zeros(3)
    p1, m, v = U.adam(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
