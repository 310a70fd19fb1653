"""Pins of the FP64 U-Net oracle against brute-force loops, a library
correlation, adjoint identities, central finite differences and Adam's
closed form (CPU only)."""
import numpy as np
from scipy import signal

import oracle.unet_oracle as U

RNG = np.random.default_rng(1234)
LV = (8, 16, 32)          # a three-level network keeps the FD checks fast


def brute_conv3x3(x, w, b):
    n, h, wd, ci = x.shape
    co = w.shape[0]
    y = np.zeros((n, h, wd, co))
    for a in range(n):
        for yy in range(h):
            for xx in range(wd):
                for o in range(co):
                    s = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            sy, sx = yy + ky - 1, xx + kx - 1
                            if 0 <= sy < h and 0 <= sx < wd:
                                for i in range(ci):
                                    s += w[o, ky, kx, i] * x[a, sy, sx, i]
                    y[a, yy, xx, o] = s
    return y


def test_conv3x3_matches_brute_force_loops():
    x = RNG.normal(size=(2, 4, 5, 3))
    w = RNG.normal(size=(4, 3, 3, 3))
    b = RNG.normal(size=4)
    assert np.allclose(U.conv3x3(x, w, b), brute_conv3x3(x, w, b), rtol=1e-13, atol=1e-13)


def test_conv3x3_matches_scipy_correlation():
    x = RNG.normal(size=(1, 9, 7, 2))
    w = RNG.normal(size=(3, 3, 3, 2))
    y = U.conv3x3(x, w)
    for o in range(3):
        ref = sum(signal.correlate2d(x[0, :, :, i], w[o, :, :, i], mode="same") for i in range(2))
        assert np.allclose(y[0, :, :, o], ref, rtol=1e-12, atol=1e-12)


def test_conv3x3_gradients_are_adjoint():
    """<conv(x), dy> is bilinear: its x- and w-gradients reproduce it."""
    x = RNG.normal(size=(2, 6, 5, 4))
    w = RNG.normal(size=(3, 3, 3, 4))
    dy = RNG.normal(size=(2, 6, 5, 3))
    dx, dw, db = U.conv3x3_grad(x, w, dy)
    s = float((U.conv3x3(x, w) * dy).sum())
    assert np.isclose((dx * x).sum(), s, rtol=1e-12)
    assert np.isclose((dw * w).sum(), s, rtol=1e-12)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


def test_upconv_matches_brute_force_and_is_adjoint():
    x = RNG.normal(size=(2, 3, 4, 5))
    w = RNG.normal(size=(6, 2, 2, 5))
    b = RNG.normal(size=6)
    y = U.upconv2(x, w, b)
    ref = np.zeros_like(y)
    for n in range(2):
        for i in range(3):
            for j in range(4):
                for a in range(2):
                    for c in range(2):
                        ref[n, 2 * i + a, 2 * j + c] = w[:, a, c, :] @ x[n, i, j] + b
    assert np.allclose(y, ref, rtol=1e-13)
    dy = RNG.normal(size=y.shape)
    dx, dw, _ = U.upconv2_grad(x, w, dy)
    s = float((U.upconv2(x, w) * dy).sum())
    assert np.isclose((dx * x).sum(), s, rtol=1e-12)
    assert np.isclose((dw * w).sum(), s, rtol=1e-12)


def test_maxpool_forward_and_first_maximum_rule():
    x = RNG.normal(size=(1, 4, 6, 2))
    y = U.maxpool2(x)
    for i in range(2):
        for j in range(3):
            assert np.allclose(y[0, i, j], x[0, 2 * i:2 * i + 2, 2 * j:2 * j + 2].max(axis=(0, 1)))
    # ties: all four equal -> the gradient goes to the top-left element only
    t = np.ones((1, 2, 2, 1))
    g = U.maxpool2_grad(t, np.full((1, 1, 1, 1), 3.0))
    assert g[0, 0, 0, 0] == 3.0 and g.sum() == 3.0


def _fd(f, x, idx, h=1e-6):
    old = x[idx]
    x[idx] = old + h
    fp = f()
    x[idx] = old - h
    fm = f()
    x[idx] = old
    return (fp - fm) / (2 * h)


def test_bce_gradient_and_value():
    z = RNG.normal(size=(2, 5, 5)) * 3
    t = RNG.uniform(size=z.shape)
    mask = RNG.uniform(size=z.shape) > 0.3
    g = U.masked_bce_grad(z, t, mask)
    for idx in [(0, 1, 2), (1, 4, 4), (0, 0, 0)]:
        fd = _fd(lambda: U.masked_bce(z, t, mask), z, idx)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(g[idx]))
    # value against the direct definition, pixel by pixel
    tot, cnt = 0.0, 0
    for idx in np.ndindex(z.shape):
        if mask[idx]:
            s = 1 / (1 + np.exp(-z[idx]))
            tot -= t[idx] * np.log(s) + (1 - t[idx]) * np.log(1 - s)
            cnt += 1
    assert np.isclose(U.masked_bce(z, t, mask), tot / cnt, rtol=1e-13)


def test_network_gradients_match_central_differences():
    """Every parameter tensor, a few entries each, at FD relative 1e-6."""
    p = U.init_params(7, levels=LV)
    for k in p:
        if k.endswith(".b"):
            p[k] = RNG.normal(0, 0.05, p[k].shape)   # nonzero biases exercise db
    x = RNG.normal(size=(2, 16, 16, U.IN_CHANNELS))
    t = RNG.uniform(size=(2, 16, 16))
    mask = RNG.uniform(size=t.shape) > 0.2

    def loss():
        return U.masked_bce(U.forward(p, x, LV)[0], t, mask)

    z, a = U.forward(p, x, LV)
    g = U.backward(p, a, U.masked_bce_grad(z, t, mask), LV)
    assert set(g) == set(p)
    rng = np.random.default_rng(5)
    worst = 0.0
    for k in sorted(p):
        for _ in range(3):
            idx = tuple(int(rng.integers(s)) for s in p[k].shape)
            fd = _fd(loss, p[k], idx, h=1e-5)
            scale = max(abs(fd), 1e-3 * np.abs(g[k]).max(), 1e-12)
            worst = max(worst, abs(fd - g[k][idx]) / scale)
    assert worst <= 1e-6, worst


def test_adam_closed_form_under_a_constant_gradient():
    """With a constant gradient the bias-corrected moments are g and g^2, so
    every step moves each weight by lr * g / (|g| + eps)."""
    p0 = RNG.normal(size=50)
    g = RNG.normal(size=50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        p, m, v = U.adam_step(p, g, m, v, 1e-3, 0.9, 0.999, 1e-8, step)
        assert np.allclose(p, p0 - step * 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_layer_inventory():
    specs = U.layer_specs()
    assert [s[3] for s in specs if s[1] == "conv"][:8] == [32, 32, 64, 64, 128, 128, 256, 256]
    assert sum(1 for s in specs if s[1] == "up") == 3
    n = sum(co * (9 if kind == "conv" else 4) * ci + co for _, kind, ci, co in specs) + 33
    assert 1.9e6 < n < 2.0e6
