"""FP64 reference of the warm-start U-Net: forward, backward, loss and Adam (test infrastructure).

Only tests, the entry point's smoke check and the benchmark's CPU leg use this module; the library never
imports it. Plain numpy in NCHW layout, float64 throughout, every step written out as its definition:

* 3x3 convolution with zero padding ("same" size), cross-correlation form:
  z[n, o, y, x] = b[o] + sum_{i, dy, dx} W[o, i, dy, dx] * in[n, i, y + dy - 1, x + dx - 1]
* ReLU after every 3x3 convolution.
* 2x2 average pooling between encoder levels; nearest-neighbour 2x upsampling in the decoder, whose first
  convolution at each level reads [upsampled lower level, encoder skip] concatenated along channels.
* A 1x1 output convolution added to the input (residual form): out = in + b + sum_c w[c] a[c].
* Loss: mean over masked pixels of (1000 (out - target))^2, i.e. the squared error in HU when images
  are expressed in units of mu_water.
* Adam with bias correction (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

The warm start itself (not the paper's; an extension) feeds this network the FBP-like image of the scan
in units of mu_water (the network adds a correction to it). Parameters are one flat vector in canonical order: per layer the weight
[c_out][c_in][k][k] then the bias [c_out], layers as listed in LAYERS.
"""
from __future__ import annotations

import numpy as np

#: (c_in, c_out, kernel) in canonical order: enc1a, enc1b, enc2a, enc2b, enc3a, enc3b, bottleneck a, b,
#: dec3a (256 up + 128 skip), dec3b, dec2a (128 up + 64 skip), dec2b, dec1a (64 up + 32 skip), dec1b, out.
LAYERS = ((1, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3), (64, 128, 3), (128, 128, 3), (128, 256, 3),
          (256, 256, 3), (384, 128, 3), (128, 128, 3), (192, 64, 3), (64, 64, 3), (96, 32, 3), (32, 32, 3),
          (32, 1, 1))


def n_params() -> int:
    return sum(co * ci * k * k + co for ci, co, k in LAYERS)


def unpack(theta):
    """Flat parameter vector -> list of (W [co][ci][k][k], b [co]) views."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for ci, co, k in LAYERS:
        nw = co * ci * k * k
        W = theta[o:o + nw].reshape(co, ci, k, k)
        o += nw
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == theta.size, "parameter vector has the wrong length"
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in layers])


# ---------------------------------------------------------------- building blocks ---------------------

def conv3x3(x, W, b):
    """Zero-padded 3x3 cross-correlation: x [n][ci][h][w] -> [n][co][h][w]."""
    n, ci, h, w = x.shape
    xp = np.zeros((n, ci, h + 2, w + 2))
    xp[:, :, 1:-1, 1:-1] = x
    z = np.broadcast_to(b[None, :, None, None], (n, W.shape[0], h, w)).copy()
    for dy in range(3):
        for dx in range(3):
            z += np.einsum("oi,nihw->nohw", W[:, :, dy, dx], xp[:, :, dy:dy + h, dx:dx + w], optimize=True)
    return z


def conv3x3_backward(x, W, dz):
    """Gradients of conv3x3 w.r.t. its input, weight and bias, given dz = dL/dz."""
    n, ci, h, w = x.shape
    xp = np.zeros((n, ci, h + 2, w + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for dy in range(3):
        for dx in range(3):
            dW[:, :, dy, dx] = np.einsum("nohw,nihw->oi", dz, xp[:, :, dy:dy + h, dx:dx + w], optimize=True)
            dxp[:, :, dy:dy + h, dx:dx + w] += np.einsum("oi,nohw->nihw", W[:, :, dy, dx], dz, optimize=True)
    return dxp[:, :, 1:-1, 1:-1], dW, dz.sum(axis=(0, 2, 3))


def pool2(x):
    """2x2 average pooling (h, w even)."""
    return 0.25 * (x[:, :, 0::2, 0::2] + x[:, :, 1::2, 0::2] + x[:, :, 0::2, 1::2] + x[:, :, 1::2, 1::2])


def pool2_backward(d):
    n, c, h, w = d.shape
    out = np.zeros((n, c, 2 * h, 2 * w))
    for a in range(2):
        for b in range(2):
            out[:, :, a::2, b::2] = 0.25 * d
    return out


def up2(x):
    """Nearest-neighbour 2x upsampling."""
    return x.repeat(2, axis=2).repeat(2, axis=3)


def up2_backward(d):
    return d[:, :, 0::2, 0::2] + d[:, :, 1::2, 0::2] + d[:, :, 0::2, 1::2] + d[:, :, 1::2, 1::2]


# ---------------------------------------------------------------- network ------------------------------

def forward(theta, x):
    """x: [n][h][w] (h, w divisible by 8). Returns (out [n][h][w], cache for backward)."""
    P = unpack(theta)
    a0 = np.asarray(x, dtype=np.float64)[:, None]
    cache = {"x": a0, "z": [], "inp": []}

    def layer(i, inp):
        z = conv3x3(inp, *P[i])
        cache["inp"].append(inp)
        cache["z"].append(z)
        return np.maximum(z, 0.0)

    e1 = layer(1, layer(0, a0))
    e2 = layer(3, layer(2, pool2(e1)))
    e3 = layer(5, layer(4, pool2(e2)))
    bt = layer(7, layer(6, pool2(e3)))
    d3 = layer(9, layer(8, np.concatenate([up2(bt), e3], axis=1)))
    d2 = layer(11, layer(10, np.concatenate([up2(d3), e2], axis=1)))
    d1 = layer(13, layer(12, np.concatenate([up2(d2), e1], axis=1)))
    Wo, bo = P[14]
    out = a0[:, 0] + bo[0] + np.einsum("c,nchw->nhw", Wo[0, :, 0, 0], d1)
    cache["d1"] = d1
    return out, cache


def backward(theta, cache, dout):
    """Gradient of a scalar loss w.r.t. the flat parameters, given dout = dL/dout [n][h][w]."""
    P = unpack(theta)
    grads = [None] * len(LAYERS)
    Wo, _ = P[14]
    d1 = cache["d1"]
    grads[14] = (np.einsum("nhw,nchw->c", dout, d1).reshape(1, -1, 1, 1), np.array([dout.sum()]))
    da = Wo[0, :, 0, 0][None, :, None, None] * dout[:, None]

    def layer_back(i, da):
        dz = da * (cache["z"][i] > 0)
        dx, dW, db = conv3x3_backward(cache["inp"][i], P[i][0], dz)
        grads[i] = (dW, db)
        return dx

    def dec_level(ia, da, c_up):
        dcat = layer_back(ia, layer_back(ia + 1, da))
        return up2_backward(dcat[:, :c_up]), dcat[:, c_up:]

    dd2, de1 = dec_level(12, da, 64)
    dd3, de2 = dec_level(10, dd2, 128)
    dbt, de3 = dec_level(8, dd3, 256)
    de3 = de3 + pool2_backward(layer_back(6, layer_back(7, dbt)))
    de2 = de2 + pool2_backward(layer_back(4, layer_back(5, de3)))
    de1 = de1 + pool2_backward(layer_back(2, layer_back(3, de2)))
    layer_back(0, layer_back(1, de1))
    return pack(grads)


def loss(out, target, mask):
    """Mean over masked pixels of the squared error in HU (images in units of mu_water)."""
    m = np.broadcast_to(np.asarray(mask, dtype=bool), out.shape)
    d = 1000.0 * (out - target)
    return float(np.sum(d[m] ** 2) / m.sum())


def loss_grad(out, target, mask):
    m = np.broadcast_to(np.asarray(mask, dtype=bool), out.shape)
    return np.where(m, 2.0e6 * (out - target), 0.0) / m.sum()


def adam(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t = 1 for the first); returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
