"""Pins of the oracle's distance-driven projector against things other than itself.

The paper cites its projector without defining it; the operator is the distance-driven one (weights
defined in the oracle's header). Pins: a brute-force O(pixels x bins) evaluation of every weight from
the definition (a different algorithm from the oracle's sequential merge), the adjoint identity, exact
identities (ones image = analytic chord of the central ray through the image square; partition of
unity; 90-degree rotation and mirror symmetries), and analytic line integrals through ellipses.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1512_04564_amd import synth


def tiny_geom(det="flat", u_offset=0.0, nviews=8, beta0=0.0):
    # 6x5 image, 7 bins; nviews = 8 puts views exactly on 45 degrees (sweep-mode ties)
    return synth.ScanGeometry(nx=6, ny=5, dx=1.3, dy=0.9, nb=7, du=2.0, u_offset=u_offset, det=det,
                              nviews=nviews, beta0=beta0, span=2 * math.pi, dso=20.0, dsd=40.0, nsubsets=1)


def brute_force_matrix(g):
    """Dense A [nviews*nb, ny*nx] straight from the weight definition, pixel by bin."""
    A = np.zeros((g.nviews * g.nb, g.ny * g.nx))
    u = (np.arange(g.nb + 1) - g.nb / 2.0 + g.u_offset) * g.du
    um = (np.arange(g.nb) + 0.5 - g.nb / 2.0 + g.u_offset) * g.du
    for v in range(g.nviews):
        beta = g.beta0 + g.span * v / g.nviews
        row = abs(math.sin(beta)) >= abs(math.cos(beta)) - 1e-12
        src, P = synth.ray_points(g, v, u)          # boundary rays
        _, C = synth.ray_points(g, v, um)           # bin-centre rays
        S = src[0]
        nl, nq = (g.ny, g.nx) if row else (g.nx, g.ny)
        dl, dq = (g.dy, g.dx) if row else (g.dx, g.dy)
        ax_l, ax_q = (1, 0) if row else (0, 1)      # coordinate index of the line normal / along-line axis
        for l in range(nl):
            cl = (l - (nl - 1) / 2.0) * dl
            # intersection of ray S -> P_k with the line {coord[ax_l] = cl}
            t = (cl - S[ax_l]) / (P[:, ax_l] - S[ax_l])
            pos = S[ax_q] + t * (P[:, ax_q] - S[ax_q])
            b = pos / dq + nq / 2.0
            for k in range(g.nb):
                r = C[k] - S
                scale = dl * np.hypot(r[0], r[1]) / abs(r[ax_l])
                lo, hi = min(b[k], b[k + 1]), max(b[k], b[k + 1])
                for q in range(nq):
                    ov = min(hi, q + 1) - max(lo, q)
                    if ov > 0:
                        i, j = (l, q) if row else (q, l)
                        A[v * g.nb + k, i * g.nx + j] += scale * ov / (hi - lo)
    return A


def oracle_matrix(g):
    cols = []
    for p in range(g.ny * g.nx):
        e = np.zeros(g.ny * g.nx)
        e[p] = 1.0
        cols.append(oracle.forward(g, e.reshape(g.ny, g.nx)).reshape(-1))
    return np.stack(cols, axis=1)


def oracle_matrix_T(g):
    rows = []
    for p in range(g.nviews * g.nb):
        e = np.zeros(g.nviews * g.nb)
        e[p] = 1.0
        rows.append(oracle.back(g, e.reshape(g.nviews, g.nb)).reshape(-1))
    return np.stack(rows, axis=0)


@pytest.mark.parametrize("det,u_offset,beta0", [("flat", 0.0, 0.0), ("flat", 0.37, 0.1), ("arc", 0.0, 0.0),
                                                 ("arc", -0.25, 0.3)])
def test_bruteforce_weights(det, u_offset, beta0):
    g = tiny_geom(det, u_offset, beta0=beta0)
    A_bf = brute_force_matrix(g)
    A_or = oracle_matrix(g)
    assert np.count_nonzero(A_bf) > 100
    np.testing.assert_allclose(A_or, A_bf, rtol=0, atol=1e-13)
    # the back-projector is the exact transpose
    np.testing.assert_allclose(oracle_matrix_T(g), A_or, rtol=0, atol=1e-13)


def test_sweep_mode_ties_are_row_sweep():
    g = tiny_geom()
    # views at 45 + 90 k degrees are exact ties and go to the row sweep
    assert [oracle.row_sweep(g, v) for v in range(8)] == [False, True, True, True, False, True, True, True]


def test_adjoint_identity_cfg1():
    g = synth.CFG1
    rng = np.random.default_rng(5)
    x = rng.random((g.ny, g.nx))
    r = rng.standard_normal((g.nviews, g.nb))
    lhs = float(np.sum(oracle.forward(g, x) * r))
    rhs = float(np.sum(x * oracle.back(g, r)))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # subsets are blocks of the same operator
    views = oracle.subset_views(g.nviews, g.nsubsets, 3)
    np.testing.assert_allclose(oracle.forward(g, x, views), oracle.forward(g, x)[views], rtol=0, atol=1e-12)


def _slab_chord(src, det, half_w, half_h):
    """Length of the segment of the line src->det inside [-half_w, half_w] x [-half_h, half_h]."""
    d = det - src
    n = d / np.linalg.norm(d)
    t_lo, t_hi = -np.inf, np.inf
    for ax, h in ((0, half_w), (1, half_h)):
        if abs(n[ax]) < 1e-300:
            if abs(src[ax]) > h:
                return 0.0
            continue
        a, b = (-h - src[ax]) / n[ax], (h - src[ax]) / n[ax]
        t_lo, t_hi = max(t_lo, min(a, b)), min(t_hi, max(a, b))
    return max(t_hi - t_lo, 0.0)


def test_ones_image_equals_central_chord():
    """For bins whose footprint stays inside the image on every line, A 1 = N_lines * spacing / |cos theta|,
    which is the exact chord of the bin-centre ray through the image rectangle."""
    g = synth.CFG1
    ones = oracle.forward(g, np.ones((g.ny, g.nx)))
    hw, hh = g.nx * g.dx / 2, g.ny * g.dy / 2
    checked = 0
    u = (np.arange(g.nb + 1) - g.nb / 2.0) * g.du
    um = (np.arange(g.nb) + 0.5 - g.nb / 2.0) * g.du
    for v in range(0, g.nviews, 7):
        src, P = synth.ray_points(g, v, u)
        _, C = synth.ray_points(g, v, um)
        row = oracle.row_sweep(g, v)
        ax_l, ax_q = (1, 0) if row else (0, 1)
        half_q = hw if row else hh
        half_l = hh if row else hw
        for k in range(g.nb):
            inside = True
            for kk in (k, k + 1):
                S, D = src[0], P[kk]
                for edge in (-half_l, half_l):
                    t = (edge - S[ax_l]) / (D[ax_l] - S[ax_l])
                    pos = S[ax_q] + t * (D[ax_q] - S[ax_q])
                    inside &= abs(pos) < half_q - 1e-6
            if not inside:
                continue
            chord = _slab_chord(src[0], C[k], hw, hh)
            assert abs(ones[v, k] - chord) <= 1e-12 * chord
            checked += 1
    assert checked > 500


def test_partition_of_unity():
    """Every pixel inside the detector shadow of a line is covered exactly once by the bins' footprints."""
    g = tiny_geom(beta0=0.2)
    A = oracle_matrix(g)
    for v in range(g.nviews):
        scale, row = oracle.view_scale(g, v)
        nl = g.ny if row else g.nx
        for l in range(nl):
            b = oracle.line_boundaries(g, v, l)
            width = np.abs(np.diff(b))
            lo, hi = b.min(), b.max()
            nq = g.nx if row else g.ny
            for q in range(nq):
                if q < lo or q + 1 > hi:
                    continue
                i, j = (l, q) if row else (q, l)
                cover = np.sum(A[v * g.nb:(v + 1) * g.nb, i * g.nx + j] * width / scale)
                assert abs(cover - 1.0) < 1e-12


def _disk_image(g, cx, cy, rad, mu=0.02, a=None, b=None, phi=0.0):
    e = synth.Ellipse(cx, cy, a or rad, b or rad, phi, mu)
    return e, synth.phantom_image(g, [e], supersample=8)


def test_rotation_and_mirror_symmetry_exact():
    """A centred disk: projections at 0/90/180/270 degrees agree and are mirror-symmetric, to rounding."""
    g = synth.CFG1
    _, img = _disk_image(g, 0.0, 0.0, 40.0)
    q = g.nviews // 4
    p = oracle.forward(g, img, [0, q, 2 * q, 3 * q])
    for a in range(4):
        np.testing.assert_allclose(p[a], p[a][::-1], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(p[a], p[0], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("cx,cy,a,b,phi", [(12.0, -20.0, 30.0, 30.0, 0.0), (-25.0, 8.0, 35.0, 18.0, 0.7)])
def test_analytic_chords(cx, cy, a, b, phi):
    """DD of a pixelised (8x8 supersampled) off-centre ellipse vs exact line integrals averaged over
    16 sub-rays per bin: pixelisation-limited agreement. A wrong angle direction, detector sign, bin
    offset or magnification fails by O(1)."""
    g = synth.CFG1
    e, img = _disk_image(g, cx, cy, None, a=a, b=b, phi=phi)
    p = oracle.forward(g, img)
    ref = synth.analytic_sinogram(g, [e], subrays=16)
    sel = ref > 5 * g.dx * e.mu
    assert sel.sum() > 5000
    rel = np.sqrt(np.mean((p[sel] - ref[sel]) ** 2)) / np.sqrt(np.mean(ref[sel] ** 2))
    assert rel < 0.01
    # the same comparison with the detector flipped is far off (the check has teeth)
    bad = np.sqrt(np.mean((p[:, ::-1][sel] - ref[sel]) ** 2)) / np.sqrt(np.mean(ref[sel] ** 2))
    assert bad > 0.2


def test_analytic_chords_arc_detector():
    g = synth.CFG1.replace(det="arc", du=1.0)
    e, img = _disk_image(g, 10.0, 15.0, 30.0)
    p = oracle.forward(g, img)
    ref = synth.analytic_sinogram(g, [e], subrays=16)
    sel = ref > 5 * g.dx * e.mu
    rel = np.sqrt(np.mean((p[sel] - ref[sel]) ** 2)) / np.sqrt(np.mean(ref[sel] ** 2))
    assert rel < 0.01


def test_synth_chords_against_sampling():
    """The analytic ellipse line integral itself, against dense sampling along a few rays."""
    g = synth.CFG1
    e = synth.Ellipse(7.0, -11.0, 33.0, 21.0, 0.4, 1.0)
    rng = np.random.default_rng(0)
    for _ in range(20):
        v = int(rng.integers(g.nviews))
        uu = float(rng.uniform(-60, 60))
        src, det = synth.ray_points(g, v, uu)
        exact = synth._chords(src[None], det[None], [e])[0]
        t = np.linspace(0, 1, 400001)
        pts = src[None] + t[:, None] * (det - src)[None]
        inside = synth._inside(pts[:, 0], pts[:, 1], e.cx, e.cy, e.a, e.b, e.phi)
        approx = inside.mean() * np.linalg.norm(det - src)
        assert abs(exact - approx) < 2e-3 * max(1.0, exact)
