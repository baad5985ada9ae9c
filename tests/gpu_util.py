"""Helpers shared by the GPU tests (not collected as tests)."""
import math
import sys

import numpy as np


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def torch_dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=torch_dev())


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_norm(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def hu_rmsd(a, b, mask=None, mu_w=0.02):
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    if mask is not None:
        d = d[mask]
    return float(1000.0 / mu_w * np.sqrt(np.mean(d * d)))


def tiny_geom(**kw):
    from paper_1512_04564_amd import synth
    base = dict(nx=6, ny=5, dx=1.3, dy=0.9, nb=7, du=2.0, u_offset=0.0, det="flat", nviews=8, beta0=0.0,
                span=2 * math.pi, dso=20.0, dsd=40.0, nsubsets=2)
    base.update(kw)
    return synth.ScanGeometry(**base)


# Image parity bars (HU, mu_water = 0.02 mm^-1): the RMS bar applies over the field-of-view disk and over
# the whole image; the largest pixel difference may reach MAX_OVER_RMS times the RMS bar -- twice the
# expected extreme, sqrt(2 ln N) ~ 5 for N = 512^2 pixels, of a Gaussian error field whose RMS just meets
# the bar.
MAX_OVER_RMS = 10.0


def image_parity(xg, xo, g, bar_rms=0.5, tag=""):
    """Asserts RMSD(FOV) <= bar_rms, RMSD(whole image) <= bar_rms and max |dx| <= MAX_OVER_RMS * bar_rms (HU).
    Returns (rmsd_fov, rmsd_all, max_abs)."""
    from paper_1512_04564_amd import synth
    import oracle
    mask = oracle.fov_mask(g, synth.fov_radius(g))
    d_fov = hu_rmsd(xg, xo, mask)
    d_all = hu_rmsd(xg, xo)
    mx = float(1000.0 / 0.02 * np.max(np.abs(np.asarray(xg, np.float64) - np.asarray(xo, np.float64))))
    say(f"  {tag} RMSD(gpu, oracle): FOV {d_fov:.4f} HU, whole image {d_all:.4f} HU, max |dx| {mx:.3f} HU")
    assert d_fov <= bar_rms, d_fov
    assert d_all <= bar_rms, d_all
    assert mx <= MAX_OVER_RMS * bar_rms, mx
    return d_fov, d_all, mx
