"""Pins of the FP64 reference U-Net (the warm-start network) against mathematics outside it.

* conv3x3 equals scipy's 2-D cross-correlation summed over input channels (a library routine).
* Pooling / upsampling backward passes are the adjoints of their forward passes.
* Directional finite differences of the loss match the analytic gradient of every layer on a 32^2 input
  (all four levels: 32, 16, 8 and the 4^2 bottleneck), relative error <= 1e-6.
* Adam's first step moves every parameter by lr against the sign of its gradient (bias correction).
* With every convolution zeroed the network is the identity (residual output).
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet
from paper_1512_04564_amd import synth


def test_parameter_layout_matches_generator():
    assert unet.n_params() == synth.unet_params(0).size
    assert [s for s in synth.UNET_SHAPES] == [tuple(s) for s in unet.LAYERS]


def test_conv_is_channel_summed_cross_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 9, 7))
    W = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    z = unet.conv3x3(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, i], W[o, i], mode="same") for i in range(3))
            np.testing.assert_allclose(z[n, o], ref, rtol=1e-12, atol=1e-12)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 8, 6))
    y = rng.normal(size=(2, 3, 4, 3))
    assert np.isclose(np.sum(unet.pool2(x) * y), np.sum(x * unet.pool2_backward(y)), rtol=1e-12)
    assert np.isclose(np.sum(unet.up2(y) * x), np.sum(y * unet.up2_backward(x)), rtol=1e-12)
    # average pooling undoes nearest upsampling
    np.testing.assert_allclose(unet.pool2(unet.up2(y)), y, rtol=1e-14)


def _problem(seed=2, n=2, size=32):
    rng = np.random.default_rng(seed)
    theta = synth.unet_params(seed, out_std=0.3).astype(np.float64)
    # non-zero biases so that their gradients are exercised
    P = unet.unpack(theta)
    for W, b in P:
        b[:] = rng.normal(0.0, 0.05, b.shape)
    theta = unet.pack(P)
    x = rng.uniform(0.0, 1.5, (n, size, size))
    target = x + rng.normal(0.0, 0.05, x.shape)
    yy, xx = np.mgrid[:size, :size]
    mask = (yy - size / 2 + 0.5) ** 2 + (xx - size / 2 + 0.5) ** 2 <= (0.45 * size) ** 2
    return theta, x, target, mask


def _loss(theta, x, target, mask):
    out, _ = unet.forward(theta, x)
    return unet.loss(out, target, mask)


def test_gradient_matches_directional_finite_differences_per_layer():
    theta, x, target, mask = _problem()
    out, cache = unet.forward(theta, x)
    g = unet.backward(theta, cache, unet.loss_grad(out, target, mask))
    rng = np.random.default_rng(3)
    offs = np.cumsum([0] + [co * ci * k * k + co for ci, co, k in unet.LAYERS])
    for i in range(len(unet.LAYERS)):
        d = np.zeros_like(theta)
        d[offs[i]:offs[i + 1]] = rng.normal(size=offs[i + 1] - offs[i])
        h = 1e-6 / np.linalg.norm(d) * max(np.linalg.norm(theta[offs[i]:offs[i + 1]]), 1.0)
        fd = (_loss(theta + h * d, x, target, mask) - _loss(theta - h * d, x, target, mask)) / (2 * h)
        an = float(g @ d)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.linalg.norm(g)), f"layer {i}: fd {fd} analytic {an}"


def test_adam_first_step_is_signed_learning_rate():
    rng = np.random.default_rng(4)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    t1, m, v = unet.adam(theta, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_allclose(t1, theta - 1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_zero_network_is_identity():
    theta = np.zeros(unet.n_params())
    x = np.random.default_rng(5).uniform(size=(1, 16, 16))
    out, _ = unet.forward(theta, x)
    np.testing.assert_array_equal(out, x)
