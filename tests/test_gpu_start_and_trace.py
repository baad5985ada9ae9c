"""GPU: the FBP-like start (against the oracle's), solver error reporting, trace rows and kernel timing."""
import numpy as np
import pytest

import oracle
from paper_1512_04564_amd import synth

from gpu_util import hu_rmsd, image_parity, rel_norm, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1512_04564_amd import api as a
    return a


@pytest.mark.parametrize("cfg", ["cfg1", "cfg2"])
def test_fbp_parity(api, cfg):
    g = {"cfg1": synth.CFG1, "cfg2": synth.CFG2}[cfg]
    s = synth.noisy_scan(g, 1 if cfg == "cfg1" else 101, truth=False)
    say(f"[fbp] {cfg}")
    G = api.Geometry(g)
    xg = to_np(api.fbp(G, to_dev(s.y)))
    xo = oracle.fbp(g, s.y.astype(np.float64))
    e = rel_norm(xg, xo)
    say(f"  rel err {e:.2e}")
    assert e <= 1e-5


def test_fbp_rejects_arc_detector(api):
    g = synth.CFG1.replace(det="arc")
    G = api.Geometry(g)
    y = to_dev(np.zeros((g.nviews, g.nb), dtype=np.float32))
    with pytest.raises(api.CtError) as ei:
        api.fbp(G, y)
    assert ei.value.status == 4   # CT_ERR_UNSUPPORTED


def test_solve_from_fbp_start(api):
    import torch
    g = synth.CFG1
    s = synth.noisy_scan(g, 0)
    G = api.Geometry(g)
    x = torch.zeros((g.ny, g.nx), device="cuda:0")
    p = api.Params(alpha=1.999, niters=10, subset_order="bitrev", start="fbp")
    api.rlalm_solve(G, p, to_dev(s.y), to_dev(s.w), x)
    po = oracle.params(alpha=1.999, niters=10, nsubsets=g.nsubsets, subset_order="bitrev")
    x0 = oracle.fbp(g, s.y.astype(np.float64))
    xo, _, _ = oracle.rlalm_solve(g, po, s.y.astype(np.float64), s.w.astype(np.float64), x0)
    image_parity(to_np(x), xo, g, tag="from FBP start")


def test_too_small_majorizer_is_reported_as_divergence(api):
    """D_L scaled far below the majorizer (the paper notes that too small a D_L diverges): the solve
    returns CT_ERR_DIVERGED instead of a silent non-finite image."""
    import torch
    g = synth.CFG1
    s = synth.noisy_scan(g, 0, truth=False)
    G = api.Geometry(g)
    x = torch.zeros((g.ny, g.nx), device="cuda:0")
    p = api.Params(alpha=1.999, niters=20, dl_scale=1e-8, start="zero")
    with pytest.raises(api.CtError) as ei:
        api.rlalm_solve(G, p, to_dev(s.y), to_dev(s.w), x)
    assert ei.value.status == 5   # CT_ERR_DIVERGED


def test_nan_in_data_is_reported(api):
    import torch
    g = synth.CFG1
    s = synth.noisy_scan(g, 0, truth=False)
    y = s.y.copy()
    y[3, 100] = np.nan
    G = api.Geometry(g)
    x = torch.zeros((g.ny, g.nx), device="cuda:0")
    with pytest.raises(api.CtError) as ei:
        api.rlalm_solve(G, api.Params(niters=2, start="zero"), to_dev(y), to_dev(s.w), x)
    assert ei.value.status == 5


def test_trace_rows_match_recomputed_rmsd(api):
    import torch
    g = synth.CFG1
    s = synth.noisy_scan(g, 0)
    G = api.Geometry(g)
    ref = to_dev(s.truth)
    rf = synth.fov_radius(g)
    p = api.Params(alpha=1.999, niters=6, subset_order="bitrev", start="zero", fov_radius=rf)
    x = torch.zeros((g.ny, g.nx), device="cuda:0")
    rows = api.rlalm_solve(G, p, to_dev(s.y), to_dev(s.w), x, x_ref=ref, trace=True)
    assert [r["iter"] for r in rows] == list(range(1, 7))
    assert all(r["finite"] for r in rows)
    assert all(rows[k]["seconds"] <= rows[k + 1]["seconds"] for k in range(5))
    mask = oracle.fov_mask(g, rf)
    for k in (1, 4, 6):
        xk = torch.zeros_like(x)
        api.rlalm_solve(G, api.Params(alpha=1.999, niters=k, subset_order="bitrev", start="zero"), to_dev(s.y),
                        to_dev(s.w), xk)
        d = hu_rmsd(to_np(xk), s.truth, mask)
        assert abs(rows[k - 1]["rmsd_hu"] - d) <= 1e-3 * d + 1e-3
    # the traced solve's final image equals the untraced one
    assert torch.equal(x, xk)


def test_kernel_timing(api):
    import torch
    g = synth.CFG1
    s = synth.noisy_scan(g, 0, truth=False)
    G = api.Geometry(g)
    x = torch.zeros((g.ny, g.nx), device="cuda:0")
    with pytest.raises(api.CtError):
        api.kernel_times(G)
    api.rlalm_solve(G, api.Params(niters=2, start="zero", time_kernels=True), to_dev(s.y), to_dev(s.w), x)
    kt = api.kernel_times(G)
    assert kt["n_forward"] == 50 and kt["n_update"] == 50
    assert 0 < kt["ms_forward"] < 1000 and 0 < kt["ms_update"] < 1000
    # timing does not change the result
    x2 = torch.zeros_like(x)
    api.rlalm_solve(G, api.Params(niters=2, start="zero"), to_dev(s.y), to_dev(s.w), x2)
    assert torch.equal(x, x2)
