"""GPU solver parity: the HIP relaxed OS-LALM (through the C ABI) against the FP64 oracle's Algorithm 1.

Bar: image RMSD <= 0.5 HU (mu_water = 0.02 mm^-1) over the field-of-view disk and over the whole image,
and max |x_gpu - x_oracle| <= 5 HU over the whole image, after a fixed number of iterations. Cases: the
128^2 scan (220 views, M = 10, 20 iterations) for alpha = 1 and 1.999 and the options; the 512^2 scan
(984 views, M = 41) for a few iterations at full size, and long runs at M = 41, 12 and 1; one
subiteration at full size compared norm-wise on x, g and h; the state interface (init / iterate,
checkpoint-resume) and graph replay compared bitwise against the plain launches.
"""
import math

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


_SCANS = {}


def scan(g, seed):
    key = (g, seed)
    if key not in _SCANS:
        _SCANS[key] = synth.noisy_scan(g, seed)
    return _SCANS[key]


def gpu_solve(api, g, s, x0, **kw):
    import torch
    G = api.Geometry(g)
    p = api.Params(**kw)
    x = to_dev(x0)
    api.rlalm_solve(G, p, to_dev(s.y), to_dev(s.w), x)
    torch.cuda.synchronize()
    return to_np(x)


def oracle_solve(g, s, x0, **kw):
    kw = dict(kw)
    kw.pop("use_graph", None)
    kw.pop("forward_split", None)   # how the GPU forms the residual, not what it computes
    start = kw.pop("start", "given")
    p = oracle.params(nsubsets=g.nsubsets, **kw)
    x, _, _ = oracle.rlalm_solve(g, p, s.y.astype(np.float64), s.w.astype(np.float64),
                                 np.zeros((g.ny, g.nx)) if start == "zero" else x0)
    return x


CFG1_CASES = [
    dict(alpha=1.0, subset_order="sequential"),
    dict(alpha=1.999, subset_order="bitrev"),
    dict(alpha=1.999, subset_order="bitrev", kappa=True),
    dict(alpha=1.999, subset_order="bitrev", algorithm=2),
    dict(alpha=1.999, subset_order="sequential", kappa=True),
    # fixed AL penalty (Section IV, rho = 0.05) with the proposed and the simple relaxation
    dict(alpha=1.999, subset_order="bitrev", rho_mode="fixed", rho_fixed=0.05),
    dict(alpha=1.999, subset_order="bitrev", rho_mode="fixed", rho_fixed=0.05, algorithm=2),
    # the Fair potential of the paper's XCAT run, the maximum-curvature D_R, the full-gradient start
    dict(alpha=1.5, subset_order="bitrev", potential="fair"),
    dict(alpha=1.999, subset_order="bitrev", huber=False),
    dict(alpha=1.999, subset_order="bitrev", init_full=True),
    # the forward projection split over two workgroups per block (the default at this size) and not
    dict(alpha=1.999, subset_order="bitrev", forward_split=0),
    dict(alpha=1.999, subset_order="bitrev", forward_split=1),
]


@pytest.mark.parametrize("case", CFG1_CASES, ids=lambda c: "-".join(f"{k}={v}" for k, v in c.items()))
def test_solve_parity_cfg1(api, case):
    g = synth.CFG1
    s = scan(g, 0)
    x0 = np.zeros((g.ny, g.nx), dtype=np.float32)
    say(f"[solve cfg1] {case}")
    xg = gpu_solve(api, g, s, x0, niters=20, **case)
    xo = oracle_solve(g, s, x0.astype(np.float64), niters=20, **case)
    image_parity(xg, xo, g)


def test_solve_parity_cfg1_divergent_default(api):
    """alpha = 1.999 with the sequential subset order (the default readings) diverges at cfg1 in FP64
    as well; the GPU follows the oracle over the first iterations, before the divergence amplifies the
    FP32 / FP64 difference."""
    g = synth.CFG1
    s = scan(g, 0)
    x0 = np.zeros((g.ny, g.nx), dtype=np.float32)
    for k in (1, 2):
        xg = gpu_solve(api, g, s, x0, niters=k, alpha=1.999)
        xo = oracle_solve(g, s, x0.astype(np.float64), niters=k, alpha=1.999)
        image_parity(xg, xo, g, tag=f"k={k}")


def test_state_interface_matches_solve_and_resumes_bitwise(api):
    import torch
    g = synth.CFG1
    s = scan(g, 0)
    G = api.Geometry(g)
    p = api.Params(alpha=1.999, niters=5, subset_order="bitrev")
    y, w = to_dev(s.y), to_dev(s.w)
    x_solve = torch.zeros((g.ny, g.nx), device="cuda:0")
    api.rlalm_solve(G, p, y, w, x_solve)
    dl = torch.empty_like(x_solve)
    api.rlalm_prepare(G, p, w, dl)
    T = p.niters * g.nsubsets
    # straight run through the state interface
    x = torch.zeros_like(x_solve)
    gv, h = torch.empty_like(x), torch.empty_like(x)
    api.rlalm_init(G, p, y, w, dl, x, gv, h)
    api.rlalm_iterate(G, p, y, w, dl, x, gv, h, 0, T)
    torch.cuda.synchronize()
    assert torch.equal(x, x_solve)
    # checkpoint after 13 subiterations (mid-iteration), resume
    x2 = torch.zeros_like(x)
    g2, h2 = torch.empty_like(x), torch.empty_like(x)
    api.rlalm_init(G, p, y, w, dl, x2, g2, h2)
    api.rlalm_iterate(G, p, y, w, dl, x2, g2, h2, 0, 13)
    ckpt = [t.clone() for t in (x2, g2, h2)]
    x3, g3, h3 = [t.clone() for t in ckpt]
    api.rlalm_iterate(G, p, y, w, dl, x3, g3, h3, 13, T - 13)
    torch.cuda.synchronize()
    assert torch.equal(x3, x_solve)
    assert torch.equal(g3, gv) and torch.equal(h3, h)
    # graph replay and plain launches give the same bits
    p_plain = api.Params(alpha=1.999, niters=5, subset_order="bitrev", use_graph=False)
    x_plain = torch.zeros_like(x)
    api.rlalm_solve(G, p_plain, y, w, x_plain)
    torch.cuda.synchronize()
    assert torch.equal(x_plain, x_solve)


def test_init_and_one_subiteration_parity_cfg2(api):
    """The 512^2 scan: the initial state and one subiteration from it, norm-wise against the oracle (1e-5)."""
    import torch
    g = synth.CFG2
    s = scan(g, 100)
    say("[solve cfg2] init + one subiteration")
    G = api.Geometry(g)
    p = api.Params(alpha=1.999, niters=1)
    y, w = to_dev(s.y), to_dev(s.w)
    dl = torch.empty((g.ny, g.nx), device="cuda:0")
    api.rlalm_prepare(G, p, w, dl)
    dl_ref = oracle.dl(g, s.w.astype(np.float64))
    assert rel_norm(to_np(dl), dl_ref) <= 1e-5
    x0 = (s.truth * 0.9).astype(np.float32)
    x = to_dev(x0)
    gv, h = torch.empty_like(x), torch.empty_like(x)
    api.rlalm_init(G, p, y, w, dl, x, gv, h)
    po = oracle.params(alpha=1.999, niters=1, nsubsets=g.nsubsets)
    xo, go, ho = oracle.rlalm_init(g, po, s.y.astype(np.float64), s.w.astype(np.float64), dl_ref,
                                   x0.astype(np.float64))
    assert rel_norm(to_np(gv), go) <= 1e-5
    assert rel_norm(to_np(h), ho) <= 1e-5
    api.rlalm_iterate(G, p, y, w, dl, x, gv, h, 0, 1)
    oracle.rlalm_iterate(g, po, s.y.astype(np.float64), s.w.astype(np.float64), dl_ref, xo, go, ho, 0, 1)
    ex, eg, eh = rel_norm(to_np(x), xo), rel_norm(to_np(gv), go), rel_norm(to_np(h), ho)
    say(f"  one subiteration rel err x {ex:.2e} g {eg:.2e} h {eh:.2e}")
    assert ex <= 1e-5 and eg <= 1e-5 and eh <= 1e-5


@pytest.mark.parametrize("alpha", [1.999, 1.0])
def test_solve_parity_cfg2_first_iterations(api, alpha):
    """Full-size cfg2 (M = 41, the benchmarked launch configuration) for 2 iterations."""
    g = synth.CFG2
    s = scan(g, 100)
    x0 = np.zeros((g.ny, g.nx), dtype=np.float32)
    say(f"[solve cfg2] alpha={alpha}, 2 iterations")
    xg = gpu_solve(api, g, s, x0, niters=2, alpha=alpha)
    xo = oracle_solve(g, s, x0.astype(np.float64), niters=2, alpha=alpha)
    image_parity(xg, xo, g)


RAGGED = {
    # sizes that are not multiples of the 16 x 16 update tile or of the 64-bin projection block, an
    # off-centre detector, and 6 subsets of 6 views
    "ragged": synth.ScanGeometry(nx=77, ny=53, dx=1.1, dy=0.8, nb=131, du=1.3, u_offset=-0.25, det="flat",
                                 nviews=36, beta0=0.05, span=2 * math.pi, dso=300.0, dsd=600.0, nsubsets=6),
    "arc_cfg1": synth.CFG1.replace(det="arc"),
}


@pytest.mark.parametrize("name", list(RAGGED))
def test_solve_parity_ragged_and_arc(api, name):
    g = RAGGED[name]
    s = scan(g, 7)
    x0 = np.zeros((g.ny, g.nx), dtype=np.float32)
    case = dict(alpha=1.999, subset_order="bitrev", niters=10)
    xg = gpu_solve(api, g, s, x0, **case)
    xo = oracle_solve(g, s, x0.astype(np.float64), **case)
    mask = oracle.fov_mask(g, synth.fov_radius(g))
    assert mask.sum() > 100
    image_parity(xg, xo, g, tag=name)


def test_solve_parity_exp_weights(api):
    """Statistical weights w = exp(-y) (the paper's simulated scan), about 1/I0 of the default weights, with
    beta scaled alike (1024 / 1e5)."""
    g = synth.CFG1
    s = synth.noisy_scan(g, 3, weights="exp")
    x0 = np.zeros((g.ny, g.nx), dtype=np.float32)
    case = dict(alpha=1.999, subset_order="bitrev", niters=20, beta=1024.0 / 1e5)
    xg = gpu_solve(api, g, s, x0, **case)
    xo = oracle_solve(g, s, x0.astype(np.float64), **case)
    image_parity(xg, xo, g, tag="exp weights")


def test_solve_parity_potentials(api):
    """The three potentials (hyperbola, Fair, q-GGMRF with p = 2, q = 1.2) with a strong regularizer
    (beta = 1e6), where their images differ from each other by more than 0.3 HU: the GPU must match the
    oracle's result for the same potential to 0.05 HU, well inside that separation (the 0.5 HU bar of the
    other cases would not tell the potentials apart)."""
    g = synth.CFG1
    s = scan(g, 0)
    x0 = np.zeros((g.ny, g.nx), dtype=np.float32)
    mask = oracle.fov_mask(g, synth.fov_radius(g))
    xo = {}
    for pot in ("hyperbola", "fair", "qggmrf"):
        case = dict(alpha=1.999, subset_order="bitrev", niters=20, beta=1e6, potential=pot)
        xg = gpu_solve(api, g, s, x0, **case)
        xo[pot] = oracle_solve(g, s, x0.astype(np.float64), **case)
        image_parity(xg, xo[pot], g, bar_rms=0.05, tag=f"potential {pot}, beta 1e6")
    for a, b in (("hyperbola", "fair"), ("hyperbola", "qggmrf"), ("fair", "qggmrf")):
        assert hu_rmsd(xo[a], xo[b], mask) > 0.3, (a, b)


def test_forward_split_setting(api):
    """The split and the unsplit residual differ by rounding only; an unknown setting is an argument error."""
    g = synth.CFG1
    s = scan(g, 0)
    x0 = np.zeros((g.ny, g.nx), dtype=np.float32)
    mask = oracle.fov_mask(g, synth.fov_radius(g))
    xs = {k: gpu_solve(api, g, s, x0, niters=5, alpha=1.999, subset_order="bitrev", forward_split=k) for k in (0, 1)}
    d = hu_rmsd(xs[0], xs[1], mask)
    say(f"  RMSD(split, unsplit) = {d:.2e} HU")
    assert 0.0 < d <= 0.01
    with pytest.raises(api.CtError):
        gpu_solve(api, g, s, x0, niters=1, forward_split=2)


def test_forward_split_with_unstaged_windows(api):
    """Bins much finer than pixels: a 16 x 16 tile's bin window exceeds what the update kernel stages, so it
    reads the residual from memory, both planes of a split projection included. Split and unsplit solves
    agree to rounding and with the oracle."""
    g = synth.ScanGeometry(nx=64, ny=64, dx=1.0, dy=1.0, nb=512, du=0.25, u_offset=0.0, det="flat", nviews=60,
                           beta0=0.0, span=2 * math.pi, dso=541.0, dsd=949.0, nsubsets=6)
    s = scan(g, 3)
    x0 = np.zeros((g.ny, g.nx), dtype=np.float32)
    mask = oracle.fov_mask(g, synth.fov_radius(g))
    xs = {k: gpu_solve(api, g, s, x0, niters=4, alpha=1.999, subset_order="bitrev", forward_split=k) for k in (0, 1)}
    xo = oracle_solve(g, s, x0.astype(np.float64), niters=4, alpha=1.999, subset_order="bitrev")
    d01 = hu_rmsd(xs[0], xs[1], mask)
    say(f"  RMSD(split, unsplit) = {d01:.2e} HU")
    assert d01 <= 0.01
    image_parity(xs[1], xo, g, tag="split")


LONG_CASES = [
    # the named 41-subset configuration over 100 iterations, unrelaxed (alpha = 1 stays stable at 41 subsets
    # on this scan; alpha = 1.999 falls into a limit cycle hundreds of HU wide there, whose phase the
    # rounding difference between FP32 and FP64 decides, so it has only the short runs above)
    dict(nsubsets=41, alpha=1.0, niters=100),
    # the 12-subset configurations behind the time-to-1-HU, relaxation and ablation numbers
    dict(nsubsets=12, alpha=1.999, niters=30),
    dict(nsubsets=12, alpha=1.0, niters=30),
    # one subset of all 984 views
    dict(nsubsets=1, alpha=1.999, niters=20),
]


@pytest.mark.parametrize("case", LONG_CASES, ids=lambda c: "-".join(f"{k}={v}" for k, v in c.items()))
def test_solve_parity_cfg2_long(api, case):
    """The 512^2 scan over many iterations (bit-reversed subset order, FBP-like start computed by the
    oracle for both sides), against the oracle over the whole image."""
    case = dict(case)
    M = case.pop("nsubsets")
    g = synth.CFG2.replace(nsubsets=M)
    s = scan(synth.CFG2, 100)
    x0 = oracle.fbp(g, s.y.astype(np.float64)).astype(np.float32)
    say(f"[solve 512^2 long] M={M} {case}")
    xg = gpu_solve(api, g, s, x0, subset_order="bitrev", **case)
    xo = oracle_solve(g, s, x0.astype(np.float64), subset_order="bitrev", **case)
    image_parity(xg, xo, g, tag=f"M={M}")


def test_graph_cache_follows_forward_split(api):
    """Two solves on one handle that differ only in forward_split: the second must not replay the graph
    captured for the first (its result equals that of a fresh handle, bit for bit)."""
    import torch
    g = synth.CFG1
    s = scan(g, 0)
    y, w = to_dev(s.y), to_dev(s.w)
    G = api.Geometry(g)
    outs = {}
    for k in (1, 0):
        x = torch.zeros((g.ny, g.nx), device="cuda:0")
        api.rlalm_solve(G, api.Params(alpha=1.999, niters=4, subset_order="bitrev", forward_split=k), y, w, x)
        outs[k] = x
    x_fresh = torch.zeros((g.ny, g.nx), device="cuda:0")
    api.rlalm_solve(api.Geometry(g), api.Params(alpha=1.999, niters=4, subset_order="bitrev", forward_split=0), y, w,
                    x_fresh)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], x_fresh)
    assert not torch.equal(outs[0], outs[1])
