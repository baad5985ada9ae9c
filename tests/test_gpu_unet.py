"""GPU: the BF16 matrix-core U-Net of the learned warm start against the FP64 reference network.

Bars (BF16 storage of weights, activations and gradients, FP32 sums), norm-wise relative to the FP64
reference running on the same FP32 master weights:
* forward: the network's contribution (output minus the residual input) within 2e-2;
* gradients: within 5e-2 per layer. Every stored BF16 value carries a relative rounding of at most 2^-9;
  between the loss and the deepest layer's weight gradient lie about 25 such roundings (activations
  and weights on the way down, gradients on the way back), so 25 * 2^-9 = 4.9% bounds the aligned
  worst case; independent roundings give far less, which is what is measured (1-2%);
* one Adam step within FP32 rounding of the FP64 update computed from the GPU's own gradient.
Shapes include ragged ones whose deepest level holds a few pixels (8 x 8 input: one pixel; 24 x 40: 15
pixels, so partial 64-pixel waves and a partial 32-pixel chunk of the weight-gradient sum). Gradients
are compared where each weight's gradient sums enough products for the rounding bound to apply; at
a single 8 x 8 image (64 products) one ReLU sign flipped by rounding can move a layer's gradient by
several percent, so that shape is checked in the forward pass only. The learned start of a solve
equals a given start made from the same network output, bit for bit.
"""
import numpy as np
import pytest

import oracle
from oracle import unet as ref
from paper_1512_04564_amd import synth

from gpu_util import rel_norm, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1512_04564_amd import api, unet
    return api, unet


def params(seed=7):
    th = synth.unet_params(seed, out_std=0.3)
    rng = np.random.default_rng(seed)
    P = ref.unpack(th.astype(np.float64))
    for _, b in P:
        b[:] = rng.normal(0.0, 0.05, b.shape)
    return ref.pack(P).astype(np.float32)


def images(n, h, w, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.5, (n, h, w))
    t = x + rng.normal(0.0, 0.1, x.shape)
    yy, xx = np.mgrid[:h, :w]
    mask = ((yy - h / 2 + 0.5) / (0.45 * h)) ** 2 + ((xx - w / 2 + 0.5) / (0.45 * w)) ** 2 <= 1.0
    return x.astype(np.float32), t.astype(np.float32), mask


def dev3(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda:0")


def layer_slices():
    offs = np.cumsum([0] + [co * ci * k * k + co for ci, co, k in ref.LAYERS])
    return [slice(offs[i], offs[i + 1]) for i in range(len(ref.LAYERS))]


@pytest.mark.parametrize("n,h,w", [(1, 8, 8), (2, 24, 40), (2, 64, 64), (3, 96, 128), (1, 512, 512)])
def test_forward_parity(mods, n, h, w):
    _, unet = mods
    th = params()
    x, _, _ = images(n, h, w, 11)
    net = unet.UNet(th, n, h, w)
    out = to_np(net.forward(dev3(x)))
    ro, _ = ref.forward(th.astype(np.float64), x.astype(np.float64))
    e = rel_norm(out - x, ro - x)
    say(f"  [unet fwd {n}x{h}x{w}] rel err of the network term {e:.2e}")
    assert e <= 2e-2


# 2 x 256^2 runs the LDS-tiled convolution in both directions with 16-row tiles (with and without the
# chunk prefetch) and 8-row tiles, and the pooling fused into its forward epilogue; the smaller images
# run the untiled forms. The weight gradient takes its nine-tap form at levels whose width is a multiple
# of 64 (256: four 64-pixel segments per row, 128: two, 64: one; 1 x 64 x 192: three, then 96 and 48 wide
# levels in the single-tap form) and the single-tap form elsewhere (2 x 24 x 40 throughout).
@pytest.mark.parametrize("n,h,w", [(2, 64, 64), (2, 24, 40), (2, 256, 256), (1, 64, 192)])
def test_gradient_parity_every_layer(mods, n, h, w):
    import torch
    _, unet = mods
    th = params()
    x, t, mask = images(n, h, w, 12)
    net = unet.UNet(th, n, h, w)
    m = torch.as_tensor(mask.astype(np.uint8), device="cuda:0")
    loss, g = net.gradient(dev3(x), dev3(t), m)
    out, cache = ref.forward(th.astype(np.float64), x.astype(np.float64))
    lo = ref.loss(out, t, mask)
    go = ref.backward(th.astype(np.float64), cache, ref.loss_grad(out, t.astype(np.float64), mask))
    say(f"  loss gpu {loss:.6g} ref {lo:.6g}")
    assert abs(loss - lo) <= 2e-2 * lo
    worst = 0.0
    for i, sl in enumerate(layer_slices()):
        e = rel_norm(g[sl], go[sl])
        worst = max(worst, e)
        say(f"  layer {i:2d} {ref.LAYERS[i]}: gradient rel err {e:.2e}")
        assert e <= 5e-2, f"layer {i}"
    say(f"  worst layer {worst:.2e}")


def test_adam_step_matches_reference_update(mods):
    import torch
    _, unet = mods
    th = params(8)
    x, t, mask = images(2, 32, 32, 13)
    net = unet.UNet(th, 2, 32, 32)
    m = torch.as_tensor(mask.astype(np.uint8), device="cuda:0")
    _, g = net.gradient(dev3(x), dev3(t), m)
    net.train_step(dev3(x), dev3(t), m, lr=1e-3)
    th1 = net.params()
    ref1, _, _ = ref.adam(th.astype(np.float64), g.astype(np.float64), np.zeros(th.size), np.zeros(th.size), 1, 1e-3)
    err = np.abs(th1 - ref1)
    say(f"  Adam step max abs err {err.max():.2e} (step size 1e-3)")
    assert err.max() <= 1e-6 + 1e-6 * np.abs(ref1).max()


def test_training_reduces_the_loss(mods):
    import torch
    _, unet = mods
    th = synth.unet_params(9)
    x, t, mask = images(4, 64, 64, 14)
    # a learnable map: target = smoothed input
    t = (x + np.roll(x, 1, 1) + np.roll(x, -1, 1) + np.roll(x, 1, 2) + np.roll(x, -1, 2)) / 5.0
    net = unet.UNet(th, 4, 64, 64)
    m = torch.as_tensor(mask.astype(np.uint8), device="cuda:0")
    xd, td = dev3(x), dev3(t.astype(np.float32))
    losses = [net.train_step(xd, td, m, lr=1e-3) for _ in range(40)]
    say(f"  loss {losses[0]:.4g} -> {losses[-1]:.4g}")
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.3 * losses[0]


def test_network_input_and_learned_start(mods):
    import torch
    api, unet = mods
    g = synth.CFG1
    s = synth.noisy_scan(g, 5, truth=False)
    G = api.Geometry(g)
    y, w = to_dev(s.y), to_dev(s.w)
    xin = unet.network_input(G, y)
    xo = oracle.fbp(g, s.y.astype(np.float64)) / 0.02
    e = rel_norm(to_np(xin), xo)
    say(f"  network input rel err {e:.2e}")
    assert e <= 1e-5
    net = unet.UNet(synth.unet_params(3), 1, g.ny, g.nx)
    x0 = 0.02 * torch.clamp(net.forward(xin[None].contiguous())[0], min=0.0)
    p_l = api.Params(alpha=1.999, niters=3, subset_order="bitrev", start="learned", unet=net)
    x_l = torch.zeros((g.ny, g.nx), device="cuda:0")
    api.rlalm_solve(G, p_l, y, w, x_l)
    x_g = x0.clone()
    api.rlalm_solve(G, api.Params(alpha=1.999, niters=3, subset_order="bitrev"), y, w, x_g)
    torch.cuda.synchronize()
    assert torch.equal(x_l, x_g)
    with pytest.raises(api.CtError):
        api.rlalm_solve(G, api.Params(niters=1, start="learned"), y, w, x_l)   # no network given
