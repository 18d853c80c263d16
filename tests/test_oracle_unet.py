"""Pins of the NumPy U-Net reference: convolution vs a brute-force loop,
adjoint identities of pooling/upsampling/convolution, gradients vs finite
differences, and bfloat16 rounding."""
import numpy as np
import pytest

from oracle import unet


def test_conv_matches_bruteforce():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 3))
    W = rng.standard_normal((2, 27, 3))
    b = rng.standard_normal(2)
    assert np.allclose(unet.conv3(x, W, b), unet.conv3_bruteforce(x, W, b), atol=1e-12)


def test_adjoint_identities():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 6, 8, 3))
    y = rng.standard_normal((2, 3, 4, 3))
    assert np.vdot(unet.pool(x), y) == pytest.approx(np.vdot(x, unet.pool_backward(y)))
    assert np.vdot(unet.up(y), x) == pytest.approx(np.vdot(y, unet.up_backward(x)))
    W = rng.standard_normal((5, 27, 3))
    dy = rng.standard_normal((4, 6, 8, 5))
    dx, dW, db = unet.conv3_backward(x, W, dy)
    # <conv(x), dy> is linear in x and in W
    assert np.vdot(unet.conv3(x, W, np.zeros(5)), dy) == pytest.approx(np.vdot(x, dx))
    assert np.vdot(unet.conv3(x, W, np.zeros(5)), dy) == pytest.approx(np.vdot(W, dW))


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    C = 4
    params = unet.init_params(C, seed=3)
    for W, b in params:
        b += 0.1 * rng.standard_normal(b.shape)
    x = rng.standard_normal((4, 8, 8, 2))
    tgt = rng.standard_normal((4, 8, 8, 2))
    net = unet.UNet(params)
    net.loss(x, tgt)
    g = net.backward(tgt)
    eps = 1e-6
    for li in (0, 3, 6, 8, 10):
        W, b = params[li]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            Wp = [(w.copy(), bb.copy()) for w, bb in params]
            Wm = [(w.copy(), bb.copy()) for w, bb in params]
            Wp[li][0][idx] += eps
            Wm[li][0][idx] -= eps
            fd = (unet.UNet(Wp).loss(x, tgt) - unet.UNet(Wm).loss(x, tgt)) / (2 * eps)
            assert g[li][0][idx] == pytest.approx(fd, rel=1e-5, abs=1e-10)
        j = int(rng.integers(0, b.size))
        Bp = [(w.copy(), bb.copy()) for w, bb in params]
        Bm = [(w.copy(), bb.copy()) for w, bb in params]
        Bp[li][1][j] += eps
        Bm[li][1][j] -= eps
        fd = (unet.UNet(Bp).loss(x, tgt) - unet.UNet(Bm).loss(x, tgt)) / (2 * eps)
        assert g[li][1][j] == pytest.approx(fd, rel=1e-5, abs=1e-10)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.14159265, 0.0])
    r = unet.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie rounds to even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6            # tie rounds to even (up)
    assert abs(r[4] - v[4]) <= 2 ** -8 * abs(v[4])
    assert r[5] == 0.0
