"""GPU: 16-bit storage (float16 / bfloat16) of the solver's y, w, residual block and projector image copies.

The oracle (FP64) is run on the very 16-bit values the GPU receives (one CPU conversion feeds both), so
the remaining difference is the GPU's own rounding: every forward projection reads the image rounded to
16 bits and every back-projection reads a 16-bit residual. Tolerances follow from the rounding of the
image copy, the dominant term. Every phantom value is below 0.04 mm^-1 < 2^-4, so a pixel's rounding error
is at most half a unit in the last place of the binade [2^-5, 2^-4): 2^-5 * 2^-11 = 1.5e-5 mm^-1 = 0.76 HU
in float16 and 2^-5 * 2^-8 = 1.2e-4 mm^-1 = 6.1 HU in bfloat16. Uniform rounding has RMS 1/sqrt(3) of
that (0.44 / 3.52 HU; body values, one binade lower, give half), and at the fixed point the image differs
from the oracle's by its own rounding residual (the projector sees the rounded copy). Bars: float16 0.5 HU
(the float32 bar), bfloat16 3.6 HU, as RMSD over the field-of-view disk and over the whole image; the
largest pixel difference may reach ten times the RMS bar (as for float32). float16 needs the weights in range: w and beta are scaled by 2^-6,
which leaves the iterates unchanged (pinned on the oracle in test_oracle_algorithm).

The 512^2 cases use the bit-reversed subset order: with the sequential order at M = 41 the iteration
itself is unstable on this workload (the FP64 oracle's own error to the phantom grows from 73 to 1080 HU
over four iterations), so any perturbation, float32 rounding included, is amplified without bound and
no rounding-derived bar applies.
"""
import numpy as np
import pytest

import oracle
from paper_1512_04564_amd import synth

from gpu_util import image_parity, rel_norm, say, to_dev, to_np

pytestmark = pytest.mark.gpu

SCALE = {"f16": 2.0 ** -6, "bf16": 1.0}
BAR_HU = {"f16": 0.5, "bf16": 3.6}


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1512_04564_amd import api as a
    return a


def rounded(a, storage):
    """The 16-bit tensor (CPU) and its exact float64 value."""
    import torch
    dt = {"f16": torch.float16, "bf16": torch.bfloat16}[storage]
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dt)
    return t, t.to(torch.float64).numpy()


def inputs(g, seed, storage):
    s = synth.noisy_scan(g, seed)
    c = SCALE[storage]
    y16, y64 = rounded(s.y, storage)
    w16, w64 = rounded(s.w * c, storage)
    return s, y16.cuda(), w16.cuda(), y64, w64, c


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_solve_parity_16bit_cfg1(api, storage):
    import torch
    g = synth.CFG1
    s, y, w, y64, w64, c = inputs(g, 0, storage)
    say(f"[16-bit cfg1] {storage}")
    G = api.Geometry(g, storage)
    x = torch.zeros((g.ny, g.nx), device="cuda:0")
    api.rlalm_solve(G, api.Params(alpha=1.999, niters=20, subset_order="bitrev", beta=1024.0 * c), y, w, x)
    po = oracle.params(alpha=1.999, niters=20, nsubsets=g.nsubsets, subset_order="bitrev", beta=1024.0 * c)
    xo, _, _ = oracle.rlalm_solve(g, po, y64, w64, np.zeros((g.ny, g.nx)))
    image_parity(to_np(x), xo, g, bar_rms=BAR_HU[storage], tag=storage)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_solve_parity_16bit_cfg2_first_iterations(api, storage):
    """Full size (512^2, 984 views, M = 41), the benchmarked shape, for 2 iterations."""
    import torch
    g = synth.CFG2
    s, y, w, y64, w64, c = inputs(g, 100, storage)
    say(f"[16-bit cfg2] {storage}")
    G = api.Geometry(g, storage)
    x = torch.zeros((g.ny, g.nx), device="cuda:0")
    api.rlalm_solve(G, api.Params(alpha=1.999, niters=2, subset_order="bitrev", beta=1024.0 * c), y, w, x)
    po = oracle.params(alpha=1.999, niters=2, nsubsets=g.nsubsets, subset_order="bitrev", beta=1024.0 * c)
    xo, _, _ = oracle.rlalm_solve(g, po, y64, w64, np.zeros((g.ny, g.nx)))
    image_parity(to_np(x), xo, g, bar_rms=BAR_HU[storage], tag=storage)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_majorizer_and_fbp_from_16bit_inputs(api, storage):
    """D_L and the FBP-like start read 16-bit y / w but sum in float32 (FBP in FP64): the float32 bars hold."""
    import torch
    g = synth.CFG1
    s, y, w, y64, w64, c = inputs(g, 1, storage)
    G = api.Geometry(g, storage)
    dl = torch.empty((g.ny, g.nx), device="cuda:0")
    api.rlalm_prepare(G, api.Params(), w, dl)
    e_dl = rel_norm(to_np(dl), oracle.dl(g, w64))
    e_fbp = rel_norm(to_np(api.fbp(G, y)), oracle.fbp(g, y64))
    say(f"  {storage}: D_L rel err {e_dl:.2e}, FBP rel err {e_fbp:.2e}")
    assert e_dl <= 1e-5 and e_fbp <= 1e-5


def test_storage_dtype_is_checked(api):
    import torch
    g = synth.CFG1
    G = api.Geometry(g, "bf16")
    y = torch.zeros((g.nviews, g.nb), device="cuda:0")   # float32, not bfloat16
    x = torch.zeros((g.ny, g.nx), device="cuda:0")
    with pytest.raises(TypeError):
        api.rlalm_solve(G, api.Params(niters=1), y, y, x)
