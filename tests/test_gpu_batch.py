"""GPU: batched solve of uneven slices in lockstep (one launch per kernel per subiteration for all slices,
one graph replay per iteration).

* With the default launch shape the batched kernels run the same per-slice arithmetic as the single
  solve, so every slice equals its own ct_rlalm_solve bit for bit (uneven sizes, M odd so that a graph of
  2M subiterations and a plain tail both run).
* The three full-size slice classes (256^2 / 492 views, 384^2 / 738, 512^2 / 984; constant 500 mm field,
  M = 41, bit-reversed order) against the oracle per slice, autotuned, in float32 (0.5 HU bar) and
  bfloat16 storage (3.6 HU, the rounding-derived bar of the precision tests), RMS over the field of view
  and the whole image, max |dx| within ten times that: float32 over 20 iterations unrelaxed, both storage
  types over the first 2 iterations (relaxed and unrelaxed). At 41 subsets the relaxed iteration is chaotic
  on the 256^2 class (12 views per subset): the FP64 oracle runs away from the phantom, and two oracle runs
  whose starts differ by 0.005 HU end more than 1 HU apart after 20 iterations (pinned on the CPU in
  test_oracle_recursion), so no rounding-derived bar holds after 20 relaxed iterations there; the unrelaxed
  iteration stays contractive. The bfloat16 bar is the fixed-point rounding residual of the projector's
  image copy; over 20 iterations of 12-view subsets the per-step rounding accumulates past it on the 256^2
  class (3.9 HU RMS measured), so the 20-iteration bfloat16 errors are reported per class on the benchmark
  line rather than asserted.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1512_04564_amd import synth

from gpu_util import hu_rmsd, image_parity, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1512_04564_amd import api as a
    return a


def small_classes(M):
    def cls(n, nv, nb):
        s = 128.0 / n
        return synth.ScanGeometry(n, n, 1.0 * s, 1.0 * s, nb, 256.0 / nb, 0.0, "flat", nv, 0.0, 2 * math.pi, 541.0,
                                  949.0, M)
    return [cls(48, 110, 96), cls(80, 150, 160), cls(128, 220, 256), cls(64, 130, 128)]


@pytest.mark.parametrize("M,niters,split,storage", [(5, 3, -1, "f32"), (10, 2, -1, "f32"), (10, 2, 0, "f32"),
                                                     (10, 2, 1, "f32"), (10, 2, -1, "bf16"), (10, 2, 0, "bf16"),
                                                     (10, 2, 1, "bf16"), (10, 2, -1, "f16")])
def test_batched_equals_single_solves_bitwise(api, M, niters, split, storage):
    """Same bits with the same forward_split setting: automatic (these small batches underfill the device,
    so the batch and every single launch split), never, always; float32 and bfloat16 storage (a split
    projection's residual planes are float32 in both)."""
    import torch
    geoms = small_classes(M)
    scans = [synth.noisy_scan(g, 40 + i, truth=False) for i, g in enumerate(geoms)]
    p = api.Params(alpha=1.999, niters=niters, subset_order="bitrev", start="zero", forward_split=split)
    Gs = [api.Geometry(g, storage) for g in geoms]
    dt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[storage]
    wscale = 2.0 ** -6 if storage == "f16" else 1.0   # counts-sized weights into float16 range (same inputs on both sides)
    ys = [to_dev(s.y).to(dt) for s in scans]
    ws = [(to_dev(s.w) * wscale).to(dt) for s in scans]
    xs = [torch.zeros((g.ny, g.nx), device="cuda:0") for g in geoms]
    cfg = api.rlalm_solve_batched(Gs, p, ys, ws, xs)
    assert cfg["fp_waves"] == 16 and not cfg["largest_first"]
    for i, g in enumerate(geoms):
        xr = torch.zeros((g.ny, g.nx), device="cuda:0")
        api.rlalm_solve(api.Geometry(g, storage), p, ys[i], ws[i], xr)
        torch.cuda.synchronize()
        assert torch.equal(xs[i], xr), f"slice {i} ({g.nx}^2) differs from its single solve"


def test_batched_given_start_and_order_invariance(api):
    """x0 given per slice; the autotuned shape (any slice order) matches the oracle; the batch result does
    not depend on the slice order in the grid (a reordered call gives the same bits)."""
    import torch
    geoms = small_classes(10)[:3]
    scans = [synth.noisy_scan(g, 60 + i) for i, g in enumerate(geoms)]
    p = api.Params(alpha=1.999, niters=4, subset_order="bitrev")
    x0s = [(0.8 * s.truth).astype(np.float32) for s in scans]
    ys = [to_dev(s.y) for s in scans]
    ws = [to_dev(s.w) for s in scans]
    Gs = [api.Geometry(g) for g in geoms]
    xs = [to_dev(x0) for x0 in x0s]
    cfg = api.rlalm_solve_batched(Gs, p, ys, ws, xs, autotune=True)
    say(f"  tuned: {cfg}")
    assert cfg["fp_waves"] in (8, 16) and cfg["ms_subiteration"] > 0
    for i, g in enumerate(geoms):
        po = oracle.params(alpha=1.999, niters=4, nsubsets=g.nsubsets, subset_order="bitrev")
        xo, _, _ = oracle.rlalm_solve(g, po, scans[i].y.astype(np.float64), scans[i].w.astype(np.float64),
                                      x0s[i].astype(np.float64))
        image_parity(to_np(xs[i]), xo, g, tag=f"slice {i} ({g.nx}^2)")
    # same slices, reversed order in the call: same bits per slice (same launch shape via the cache
    # is not guaranteed for a new shape key, so force the default shape on both)
    xa = [to_dev(x0) for x0 in x0s]
    api.rlalm_solve_batched(Gs, p, ys, ws, xa)
    xb = [to_dev(x0) for x0 in x0s[::-1]]
    Gr = [api.Geometry(g) for g in geoms[::-1]]
    api.rlalm_solve_batched(Gr, p, ys[::-1], ws[::-1], xb)
    torch.cuda.synchronize()
    for i in range(3):
        assert torch.equal(xa[i], xb[2 - i])


@pytest.mark.parametrize("storage,alpha,niters", [("f32", 1.0, 20), ("f32", 1.999, 2), ("bf16", 1.999, 2),
                                                  ("bf16", 1.0, 2)])
def test_batched_full_size_classes_against_oracle(api, storage, alpha, niters):
    """One slice of each full-size class (the uneven batch's shapes, M = 41) from zero."""
    import torch
    geoms = list(synth.BATCH_CLASSES)
    scans = [synth.noisy_scan(g, 300 + i, truth=False) for i, g in enumerate(geoms)]
    dt = {"f32": torch.float32, "bf16": torch.bfloat16}[storage]
    cpu = [(torch.from_numpy(s.y).to(dt), torch.from_numpy(s.w).to(dt)) for s in scans]
    Gs = [api.Geometry(g, storage) for g in geoms]
    xs = [torch.zeros((g.ny, g.nx), device="cuda:0") for g in geoms]
    p = api.Params(alpha=alpha, niters=niters, subset_order="bitrev", start="zero")
    cfg = api.rlalm_solve_batched(Gs, p, [y.cuda() for y, _ in cpu], [w.cuda() for _, w in cpu], xs, autotune=True)
    say(f"[batch {storage}] tuned: {cfg}")
    bar = {"f32": 0.5, "bf16": 3.6}[storage]   # bfloat16: the rounding-derived bar of test_gpu_precision
    for i, g in enumerate(geoms):
        po = oracle.params(alpha=alpha, niters=niters, nsubsets=g.nsubsets, subset_order="bitrev")
        y64, w64 = (t.to(torch.float64).numpy() for t in cpu[i])
        xo, _, _ = oracle.rlalm_solve(g, po, y64, w64, np.zeros((g.ny, g.nx)))
        image_parity(to_np(xs[i]), xo, g, bar_rms=bar,
                     tag=f"slice {i} ({g.nx}^2, {g.nviews} views, {storage}, alpha {alpha}, {niters} iterations)")


def test_batched_argument_errors(api):
    import torch
    a, b = small_classes(5)[0], small_classes(10)[1]
    Ga, Gb = api.Geometry(a), api.Geometry(b)
    ya = torch.zeros((a.nviews, a.nb), device="cuda:0")
    yb = torch.zeros((b.nviews, b.nb), device="cuda:0")
    xa = torch.zeros((a.ny, a.nx), device="cuda:0")
    xb = torch.zeros((b.ny, b.nx), device="cuda:0")
    with pytest.raises(api.CtError) as ei:
        api.rlalm_solve_batched([Ga, Gb], api.Params(niters=1), [ya, yb], [ya, yb], [xa, xb])
    assert ei.value.status == 1   # different M
    with pytest.raises(api.CtError) as ei:
        api.rlalm_solve_batched([Ga, Ga], api.Params(niters=1), [ya, ya], [ya, ya], [xa, xa])
    assert ei.value.status == 1   # one handle twice
    with pytest.raises(api.CtError) as ei:
        api.rlalm_solve_batched([Ga], api.Params(niters=1, time_kernels=True), [ya], [ya], [xa])
    assert ei.value.status == 4


@pytest.mark.parametrize("M,niters", [(10, 3), (5, 3)])
def test_persistent_launch_matches_lockstep_and_oracle(api, M, niters):
    """The single persistent launch (grid barriers between the phases, 8-wave forward workgroups) against
    the lockstep launches and the oracle; M odd gives an odd number of subiterations."""
    import torch
    geoms = small_classes(M)
    scans = [synth.noisy_scan(g, 80 + i) for i, g in enumerate(geoms)]
    p = api.Params(alpha=1.999, niters=niters, subset_order="bitrev", start="zero")
    ys = [to_dev(s.y) for s in scans]
    ws = [to_dev(s.w) for s in scans]
    xp = [torch.zeros((g.ny, g.nx), device="cuda:0") for g in geoms]
    cfg = api.rlalm_solve_batched([api.Geometry(g) for g in geoms], p, ys, ws, xp, autotune="persistent")
    say(f"  persistent: {cfg}")
    assert cfg["persistent"] and cfg["blocks_per_cu"] >= 1 and cfg["fp_waves"] == 8
    xl = [torch.zeros((g.ny, g.nx), device="cuda:0") for g in geoms]
    api.rlalm_solve_batched([api.Geometry(g) for g in geoms], p, ys, ws, xl)
    torch.cuda.synchronize()
    for i, g in enumerate(geoms):
        d = hu_rmsd(to_np(xp[i]), to_np(xl[i]))
        say(f"  slice {i} ({g.nx}^2): RMSD(persistent, lockstep) = {d:.2e} HU")
        assert d <= 0.01
        po = oracle.params(alpha=1.999, niters=niters, nsubsets=M, subset_order="bitrev")
        xo, _, _ = oracle.rlalm_solve(g, po, scans[i].y.astype(np.float64), scans[i].w.astype(np.float64),
                                      np.zeros((g.ny, g.nx)))
        image_parity(to_np(xp[i]), xo, g, tag=f"persistent slice {i} ({g.nx}^2)")


def test_persistent_full_size_classes_against_oracle(api):
    """The three full-size classes in one persistent launch, 20 unrelaxed iterations at 41 subsets."""
    import torch
    geoms = list(synth.BATCH_CLASSES)
    scans = [synth.noisy_scan(g, 300 + i, truth=False) for i, g in enumerate(geoms)]
    xs = [torch.zeros((g.ny, g.nx), device="cuda:0") for g in geoms]
    p = api.Params(alpha=1.0, niters=20, subset_order="bitrev", start="zero")
    api.rlalm_solve_batched([api.Geometry(g) for g in geoms], p, [to_dev(s.y) for s in scans],
                            [to_dev(s.w) for s in scans], xs, autotune="persistent")
    for i, g in enumerate(geoms):
        po = oracle.params(alpha=1.0, niters=20, nsubsets=g.nsubsets, subset_order="bitrev")
        xo, _, _ = oracle.rlalm_solve(g, po, scans[i].y.astype(np.float64), scans[i].w.astype(np.float64),
                                      np.zeros((g.ny, g.nx)))
        image_parity(to_np(xs[i]), xo, g, tag=f"persistent slice {i} ({g.nx}^2, {g.nviews} views)")


def test_tuned_shape_is_cached_on_disk(api, tmp_path, monkeypatch):
    """autotune = 1 writes the chosen shape to the on-disk cache, one text file per GPU architecture and set
    of slice shapes."""
    import torch
    monkeypatch.setenv("CTRLALM_TUNE_DIR", str(tmp_path))
    geoms = small_classes(10)[:2]
    scans = [synth.noisy_scan(g, 90 + i, truth=False) for i, g in enumerate(geoms)]
    p = api.Params(alpha=1.999, niters=1, subset_order="bitrev", start="zero")
    xs = [torch.zeros((g.ny, g.nx), device="cuda:0") for g in geoms]
    cfg = api.rlalm_solve_batched([api.Geometry(g) for g in geoms], p, [to_dev(s.y) for s in scans],
                                  [to_dev(s.w) for s in scans], xs, autotune=True)
    files = list(tmp_path.rglob("*.txt"))
    say(f"  tuned {cfg}; cache files {[str(f.relative_to(tmp_path)) for f in files]}")
    assert len(files) == 1 and files[0].parent.name.startswith("gfx")
    text = files[0].read_text()
    assert f"persistent {int(cfg['persistent'])}" in text and f"fp_waves {cfg['fp_waves']}" in text
    assert f"forward_split {cfg['forward_split']}" in text
