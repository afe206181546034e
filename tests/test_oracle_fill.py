"""Pins of the FP64 learned-fill reference (oracle/fill.py) against things
other than itself: a pure-Python loop of the convolution's definition on tiny
inputs, scipy's 2-D correlation, the identity kernel, central finite
differences of the whole network's loss, the closed form of Adam's first
step, and the masked-MSE gradient."""
import numpy as np
import pytest
from scipy import signal

import eventsim
from oracle import fill


def rand_params(seed, scale=1.0):
    p = eventsim.fill_init_params(seed, zero_last=False).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    # non-zero biases, so that the bias terms are exercised too
    k = 0
    for ws, bs in fill.layer_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        p[k + nw:k + nw + nb] = rng.normal(0, 0.1, nb)
        k += nw + nb
    return p * scale


def test_conv_equals_loop_definition():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 4, 5))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = fill.conv3x3(x, w, b)
    n, cin, h, wd = x.shape
    for i in range(n):
        for o in range(4):
            for r in range(h):
                for c in range(wd):
                    acc = b[o]
                    for ch in range(cin):
                        for dy in range(3):
                            for dx in range(3):
                                rr, cc = r + dy - 1, c + dx - 1
                                if 0 <= rr < h and 0 <= cc < wd:
                                    acc += w[o, ch, dy, dx] * x[i, ch, rr, cc]
                    assert abs(y[i, o, r, c] - acc) < 1e-12


def test_conv_equals_scipy_correlate():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 2, 9, 7))
    w = rng.normal(size=(3, 2, 3, 3))
    b = np.zeros(3)
    y = fill.conv3x3(x, w, b)
    for o in range(3):
        ref = sum(signal.correlate2d(x[0, c], w[o, c], mode="same", boundary="fill", fillvalue=0)
                  for c in range(2))
        np.testing.assert_allclose(y[0, o], ref, rtol=0, atol=1e-12)


def test_identity_kernel_returns_input():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 3, 6, 5))
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1] = 1.0
    np.testing.assert_array_equal(fill.conv3x3(x, w, np.zeros(3)), x)


def test_masked_mse_and_gradient():
    rng = np.random.default_rng(4)
    pred, tgt = rng.normal(size=(2, 5, 5)), rng.normal(size=(2, 5, 5))
    mask = rng.random((2, 5, 5)) < 0.3
    loss, g = fill.masked_mse(pred, tgt, mask)
    assert abs(loss - np.mean((pred[mask] - tgt[mask]) ** 2)) < 1e-14
    assert np.all(g[~mask] == 0)
    np.testing.assert_allclose(g[mask], 2 * (pred[mask] - tgt[mask]) / mask.sum(), rtol=1e-14)


def test_backward_matches_central_differences():
    """Every parameter's gradient of the full network's loss against central
    differences (h = 1e-6, FP64): relative error < 1e-6 where the difference is
    not crossing a ReLU kink."""
    rng = np.random.default_rng(5)
    x = rng.normal(size=(2, 3, 6, 7))
    tgt = rng.normal(size=(2, 6, 7))
    mask = rng.random((2, 6, 7)) < 0.5
    theta = rand_params(7)
    loss, g = fill.loss_and_grad(theta, x, tgt, mask)
    h = 1e-6
    idx = np.arange(fill.N_PARAMS)
    checked = 0
    for k in idx[:: max(1, fill.N_PARAMS // 700)]:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        lp, _ = fill.loss_and_grad(tp, x, tgt, mask)
        lm, _ = fill.loss_and_grad(tm, x, tgt, mask)
        fd = (lp - lm) / (2 * h)
        # a ReLU kink inside [-h, h] shows as a one-sided slope change: skip it
        l0p = (lp - loss) / h
        l0m = (loss - lm) / h
        if abs(l0p - l0m) > 1e-4 * max(1.0, abs(fd)):
            continue
        assert abs(fd - g[k]) <= 1e-6 * max(abs(fd), 1e-3), (k, fd, g[k])
        checked += 1
    assert checked > 600


def test_backward_of_a_single_linear_layer_is_exact_adjoint():
    """<conv(x), gy> = <x, gx> and the weight gradient is the adjoint in w."""
    rng = np.random.default_rng(8)
    x = rng.normal(size=(2, 3, 5, 6))
    w = rng.normal(size=(4, 3, 3, 3))
    gy = rng.normal(size=(2, 4, 5, 6))
    y = fill.conv3x3(x, w, np.zeros(4))
    gx, gw, gb = fill.conv3x3_backward(x, w, gy)
    assert abs((y * gy).sum() - (x * gx).sum()) < 1e-10
    assert abs((y * gy).sum() - (w * gw).sum()) < 1e-10
    np.testing.assert_allclose(gb, gy.sum(axis=(0, 2, 3)), rtol=1e-14)


def test_adam_first_step_closed_form():
    """After one step from zero moments, the bias-corrected update is
    lr * g / (|g| + eps) elementwise."""
    rng = np.random.default_rng(9)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    opt = fill.Adam(50, lr=1e-3)
    new = opt.step(theta, g)
    np.testing.assert_allclose(theta - new, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_second_step_closed_form():
    rng = np.random.default_rng(10)
    theta, g1, g2 = rng.normal(size=(3, 20))
    opt = fill.Adam(20, lr=1e-2)
    t1 = opt.step(theta, g1)
    t2 = opt.step(t1, g2)
    m = (0.1 * 0.9 * g1 + 0.1 * g2) / (1 - 0.81)
    v = (0.001 * 0.999 * g1 * g1 + 0.001 * g2 * g2) / (1 - 0.999 ** 2)
    np.testing.assert_allclose(t1 - t2, 1e-2 * m / (np.sqrt(v) + 1e-8), rtol=1e-10)


def test_parameter_count_and_flat_layout():
    assert fill.N_PARAMS == 16 * 3 * 9 + 16 + 2 * (16 * 16 * 9 + 16) + 16 * 9 + 1 == 5233
    theta = np.arange(fill.N_PARAMS, dtype=np.float64)
    np.testing.assert_array_equal(fill.flatten(fill.unflatten(theta)), theta)
    w0, b0 = fill.unflatten(theta)[0]
    assert w0[0, 0, 0, 0] == 0 and w0[0, 0, 0, 1] == 1 and w0[0, 1, 0, 0] == 9 and b0[0] == 432


def test_forward_flops_per_pixel():
    """The per-pixel multiply-add count of the network (two flops each)."""
    macs = sum(9 * a * b for a, b in zip(fill.CHANNELS[:-1], fill.CHANNELS[1:]))
    assert 2 * macs == 10368


def test_fill_target_and_psnr():
    rng = np.random.default_rng(11)
    gt = rng.normal(size=(20, 30))
    L = 3.0 * gt - 0.5
    active = rng.random((20, 30)) < 0.4
    t = eventsim.fill_target(gt, L, active)
    np.testing.assert_allclose(t, L, rtol=1e-5, atol=1e-5)
    mask = ~active
    assert eventsim.fill_psnr(t, L, mask) > 90
    noisy = L + 0.1 * (L.max() - L.min())
    assert abs(eventsim.fill_psnr(noisy, L, mask) - 20.0) < 1e-6


def test_zero_last_layer_gives_back_L():
    rng = np.random.default_rng(12)
    x = rng.normal(size=(2, 3, 7, 9))
    theta = rand_params(13)
    w3, b3 = fill.unflatten(theta)[3]
    theta[-(w3.size + b3.size):] = 0.0
    pred, _ = fill.forward(fill.unflatten(theta), x)
    np.testing.assert_array_equal(pred, x[:, 0])
