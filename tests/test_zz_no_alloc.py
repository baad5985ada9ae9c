"""GPU: ct_forward_noalloc -- the forward projection for callers that cannot allocate -- against ct_forward.

Called through the C ABI on two geometries in a row, the second with a smaller image (the shared scratch
array keeps the first call's contents), each result compared bit for bit with ct_forward on a fresh
handle; an image above the scratch maximum is rejected before anything is launched.
"""
import numpy as np
import pytest

from paper_1512_04564_amd import synth

pytestmark = pytest.mark.gpu


def test_forward_noalloc_matches_forward_twice():
    import torch
    from paper_1512_04564_amd import api
    rng = np.random.default_rng(21)
    for g in (synth.CFG2, synth.CFG1.replace(nx=100, ny=77)):   # second call: smaller, ragged image
        x = torch.as_tensor(rng.uniform(0.0, 0.03, (g.ny, g.nx)).astype(np.float32), device="cuda:0")
        for subset in (-1, 3):
            G = api.Geometry(g)
            nv = G.views_in(subset)
            out = torch.full((nv, g.nb), float("nan"), device="cuda:0")
            api.forward_noalloc(G, x, out, subset=subset)
            ref = api.forward(api.Geometry(g), x, subset=subset)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (g.nx, g.ny, subset)


def test_forward_noalloc_rejects_oversized_images():
    import torch
    from paper_1512_04564_amd import api
    g = synth.CFG1.replace(nx=2049, ny=2048, dx=0.1, dy=0.1)   # 2049 x 2048 > 4 Mi pixels
    G = api.Geometry(g)
    x = torch.zeros((g.ny, g.nx), device="cuda:0")
    out = torch.zeros((g.nviews, g.nb), device="cuda:0")
    with pytest.raises(api.CtError) as ei:
        api.forward_noalloc(G, x, out)
    assert ei.value.status == 1 and "scratch" in str(ei.value)
