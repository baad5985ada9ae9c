"""Pins of the 3-D helical cone-beam oracle (oracle/ct_oracle3.c) against facts it does not compute itself.

Projector (separable distance-driven, helical source, flat detector panel):
* the merge-based projector equals a brute-force evaluation of every weight from the definition, entry by
  entry, on tiny grids (45-degree tie views, offsets, rows leaving the volume);
* adjoint identity <A x, r> = <x, A' r>;
* ones volume: a detector cell whose rays stay inside the volume gets exactly the length of its central ray
  between the first and last plane, computed here from the 3-D ray vector;
* analytic line integrals through an ellipsoid match the projection of its finely voxelised image to 1%
  RMS over cells with long chords, while the same comparison with the helix run backwards or the rows
  flipped fails by far;
* mirror symmetry of a centred sphere under an axial (feed 0) scan;
* the helix: a single voxel's projection sits on the detector row predicted by the source height.
Regularizer (13 directions, 26 neighbours): finite differences, SQS majorization, the isolated-voxel closed
form, the large-delta weighted graph Laplacian. Iteration: the alpha = 1 identity D_L x - h = zeta, SQS
descent with one subset, and a one-voxel recursion stepped by hand (subset order and rho index included).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import helical as H
from paper_1512_04564_amd import synth

TINY = [
    # 1.5 turns of 8 views from beta0 = 0: views 1, 3, ... sit exactly at 45 degrees (sweep-mode ties)
    synth.HelicalGeometry(5, 4, 3, 1.3, 0.9, 1.1, 0.2, 7, 2.0, 0.3, 4, 1.7, -0.2, 12, 8, 0.0, -2.0, 3.0, 20.0, 40.0, 3),
    # an axial-ish helix with rows reaching past the volume and a wider detector
    synth.HelicalGeometry(4, 6, 5, 1.0, 1.2, 0.7, -0.3, 9, 1.5, -0.4, 6, 1.4, 0.5, 10, 10, 0.3, -1.0, 1.2, 25.0, 45.0, 2),
]


def dense_forward(g, v):
    nvox = g.nx * g.ny * g.nz
    A = np.zeros((g.nr * g.nb, nvox))
    for n in range(nvox):
        e = np.zeros(nvox)
        e[n] = 1.0
        A[:, n] = H.forward(g, e.reshape(g.nz, g.ny, g.nx), views=[v]).reshape(-1)
    return A


@pytest.mark.parametrize("gi", range(len(TINY)))
def test_merge_equals_brute_force_weights(gi):
    g = TINY[gi]
    sweeps = set()
    for v in range(g.nviews):
        A = dense_forward(g, v)
        B = H.weights_dense(g, v)
        assert np.max(np.abs(A - B)) <= 1e-14 * max(1.0, np.max(np.abs(B))), v
        sweeps.add(H.row_sweep(g, v))
    assert sweeps == {True, False}
    assert np.count_nonzero(B) > 0


@pytest.mark.parametrize("gi", range(len(TINY)))
def test_adjoint_identity(gi):
    g = TINY[gi]
    rng = np.random.default_rng(gi)
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    r = rng.standard_normal((g.nviews, g.nr, g.nb))
    lhs = float(np.vdot(H.forward(g, x), r))
    rhs = float(np.vdot(x, H.back(g, r)))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)
    # and views subsets
    vs = [1, 4, 7]
    lhs = float(np.vdot(H.forward(g, x, views=vs), r[vs]))
    rhs = float(np.vdot(x, H.back(g, r[vs], views=vs)))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


def _central_ray(g, v, k, l):
    uc = (k + 0.5 - g.nb / 2.0 + g.u_offset) * g.du
    wc = (l + 0.5 - g.nr / 2.0 + g.w_offset) * g.dw
    src, det = synth.helical_ray_points(g, v, uc, wc)
    return src, det - src


def test_ones_volume_gives_the_central_ray_length():
    """Cells whose boundary rays cross every plane inside the volume: A 1 = length of the central ray from
    the first to the last plane (|R| / |R_normal| times the volume's extent along the plane normal)."""
    g = synth.HelicalGeometry(24, 20, 40, 1.0, 1.1, 0.5, 0.0, 11, 1.0, 0.0, 5, 0.8, 0.0, 16, 16, 0.05, -0.5, 1.0,
                              60.0, 110.0, 1)
    p = H.forward(g, np.ones((g.nz, g.ny, g.nx)))
    checked = 0
    for v in range(g.nviews):
        row = H.row_sweep(g, v)
        nl, nq = (g.ny, g.nx) if row else (g.nx, g.ny)
        half_normal = 0.5 * nl * (g.dy if row else g.dx)
        half_along = 0.5 * nq * (g.dx if row else g.dy)
        for k in range(g.nb):
            for l in range(g.nr):
                # every ray of the cell (its four corner rays bound it) must cross both outer planes inside
                # the volume's transaxial extent and its z extent
                ok = True
                for du in (0.0, 1.0):
                    for dw in (0.0, 1.0):
                        u = (k + du - g.nb / 2.0 + g.u_offset) * g.du
                        w = (l + dw - g.nr / 2.0 + g.w_offset) * g.dw
                        s, d = synth.helical_ray_points(g, v, u, w)
                        r = d - s
                        ax_n, ax_a = (1, 0) if row else (0, 1)
                        for plane in (-half_normal, half_normal):
                            t = (plane - s[ax_n]) / r[ax_n]
                            pt = s + t * r
                            if abs(pt[ax_a]) > half_along - 1e-9 or abs(pt[2] - g.zc) > 0.5 * g.nz * g.dz - 2 * g.dz:
                                ok = False
                if not ok:
                    continue
                s, r = _central_ray(g, v, k, l)
                n_ax = 1 if row else 0
                expect = 2 * half_normal * np.linalg.norm(r) / abs(r[n_ax])
                assert abs(p[v, l, k] - expect) <= 1e-12 * expect, (v, k, l, p[v, l, k], expect)
                checked += 1
    assert checked > 100


def _sphere_scan(g, ell, subrays=4):
    return synth.analytic_helical_sinogram(g, ell, subrays=subrays)


def test_analytic_ellipsoid_chords_and_negative_controls():
    """1 mm voxels (the error is first order in the voxel size: 1.2% at 2 mm, 0.6% at 1 mm)."""
    g = synth.helical_geometry(96, 48, 1.0, 1.0, 128, 1.3, 16, 24, 2, 1.0, 1)
    e = synth.random_ellipsoids(g, 5, n=1)[0]
    vol = synth.phantom_volume(g, [e], supersample=2)
    p = H.forward(g, vol)
    li = _sphere_scan(g, [e])
    long = li > 5 * g.dx * e.mu
    assert long.sum() > 1000
    err = np.sqrt(np.mean((p[long] - li[long]) ** 2)) / np.sqrt(np.mean(li[long] ** 2))
    assert err <= 0.01, err
    # the helix run backwards (table moving the other way) or the detector rows flipped: far off
    gb = g.replace(z0=-g.z0, feed=-g.feed)
    li_b = _sphere_scan(gb, [e])
    err_b = np.sqrt(np.mean((p[long] - li_b[long]) ** 2)) / np.sqrt(np.mean(li[long] ** 2))
    err_f = np.sqrt(np.mean((p[:, ::-1][long] - li[long]) ** 2)) / np.sqrt(np.mean(li[long] ** 2))
    assert err_b > 10 * err and err_f > 10 * err, (err, err_b, err_f)


def test_axial_scan_mirror_symmetry():
    """A centred sphere, feed 0 and the source at the volume's mid-plane: the projection is symmetric in w
    about the detector's centre row, and at 90 degrees symmetric in u (to rounding)."""
    g = synth.helical_geometry(32, 16, 2.0, 2.0, 40, 2.5, 10, 8, 1, 0.0, 1)
    e = synth.Ellipsoid(0.0, 0.0, 0.0, 20.0, 20.0, 9.0, 0.0, 0.02)
    vol = synth.phantom_volume(g, [e], supersample=2)
    p = H.forward(g, vol)
    assert np.max(np.abs(p - p[:, ::-1, :])) <= 1e-12 * np.max(p)
    v90 = 2   # beta = 90 degrees
    assert np.max(np.abs(p[v90] - p[v90, :, ::-1])) <= 1e-12 * np.max(p)
    assert np.max(p) > 10.0 * 0.02


def test_helix_moves_a_voxel_across_rows():
    """One voxel at height z_p: in each view its projection's row centroid is at the row coordinate of the
    ray through it, w = (z_p - S_z(v)) dsd / ell, to within a fraction of a row."""
    g = synth.helical_geometry(16, 40, 1.0, 0.5, 41, 1.0, 16, 12, 2, 0.6, 1)
    vol = np.zeros((g.nz, g.ny, g.nx))
    kz, i, j = 23, 9, 4
    vol[kz, i, j] = 1.0
    p = H.forward(g, vol)
    xp, yp = (j - (g.nx - 1) / 2.0) * g.dx, (i - (g.ny - 1) / 2.0) * g.dy
    zp = g.zc + (kz - (g.nz - 1) / 2.0) * g.dz
    seen = 0
    for v in range(g.nviews):
        rows = p[v].sum(axis=1)
        if rows.sum() <= 0:
            continue
        beta = g.beta0 + 2 * math.pi * v / g.views_per_turn
        sz = g.z0 + g.feed * v / g.views_per_turn
        ell = xp * math.cos(beta) + yp * math.sin(beta) + g.dso
        w = (zp - sz) * g.dsd / ell
        wl = (np.arange(g.nr) + 0.5 - g.nr / 2.0 + g.w_offset) * g.dw
        if abs(w) > (0.5 * g.nr - 1.5) * g.dw:
            continue   # the voxel's shadow is cut by the detector's edge
        cent = float(np.sum(rows * wl) / rows.sum())
        assert abs(cent - w) <= 0.2 * g.dw, (v, cent, w)
        seen += 1
    assert seen >= g.nviews // 2


# ---- regularizer -------------------------------------------------------------------------------------

RG = synth.HelicalGeometry(6, 5, 4, 1.0, 1.0, 1.0, 0.0, 4, 1.0, 0.0, 2, 1.0, 0.0, 4, 4, 0.0, 0.0, 0.0, 20.0, 40.0, 1)


@pytest.mark.parametrize("pot", ["hyperbola", "fair", "qggmrf"])
def test_regularizer_gradient_by_finite_differences(pot):
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 3e-4, (RG.nz, RG.ny, RG.nx))
    gr, _ = H.reg_grad(RG, x, potential=pot)
    h = 1e-9
    for n in rng.choice(x.size, 25, replace=False):
        e = np.zeros(x.size)
        e[n] = h
        e = e.reshape(x.shape)
        fd = (H.reg_cost(RG, x + e, potential=pot) - H.reg_cost(RG, x - e, potential=pot)) / (2 * h)
        assert abs(fd - gr.reshape(-1)[n]) <= 1e-7 * max(abs(fd), 1e-3)


@pytest.mark.parametrize("huber", [True, False])
def test_regularizer_sqs_majorizes(huber):
    rng = np.random.default_rng(4)
    for _ in range(20):
        x = rng.uniform(0.0, 5e-4, (RG.nz, RG.ny, RG.nx))
        z = x + rng.normal(0.0, 3e-4, x.shape)
        gr, dr = H.reg_grad(RG, x, huber=huber)
        quad = H.reg_cost(RG, x) + np.vdot(gr, z - x) + 0.5 * np.sum(dr * (z - x) ** 2)
        assert H.reg_cost(RG, z) <= quad + 1e-12 * abs(quad)


def test_isolated_voxel_closed_form():
    """One interior voxel of value t in a zero volume: R = beta phi(t) (6 + 12/sqrt 2 + 8/sqrt 3) -- each of
    the 26 neighbour pairs once, weighted by 1 / offset length."""
    g = RG.replace(nx=5, ny=5, nz=5)
    x = np.zeros((5, 5, 5))
    t = 2.5e-4
    x[2, 2, 2] = t
    d = 1e-4
    phi = d * d * (math.sqrt(1 + (t / d) ** 2) - 1)
    expect = 1024.0 * phi * (6 + 12 / math.sqrt(2) + 8 / math.sqrt(3))
    assert abs(H.reg_cost(g, x) - expect) <= 1e-12 * expect
    gr, dr = H.reg_grad(g, x)
    assert abs(gr[2, 2, 2] - 1024.0 * (t / math.sqrt(1 + (t / d) ** 2)) * (6 + 12 / math.sqrt(2) + 8 / math.sqrt(3))) \
        <= 1e-12 * abs(gr[2, 2, 2])


def test_large_delta_gives_the_weighted_laplacian():
    """delta -> infinity: phi(t) -> t^2 / 2, so grad R = L x with the 26-neighbour graph Laplacian of
    weights beta / ||s|| (built here from the neighbour offsets)."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((RG.nz, RG.ny, RG.nx))
    gr, dr = H.reg_grad(RG, x, delta=1e8, beta=2.0)
    lap = np.zeros_like(x)
    for dz in (-1, 0, 1):
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                if dz == di == dj == 0:
                    continue
                wgt = 2.0 / math.sqrt(dz * dz + di * di + dj * dj)
                for kz in range(RG.nz):
                    for i in range(RG.ny):
                        for j in range(RG.nx):
                            k2, i2, j2 = kz + dz, i + di, j + dj
                            if 0 <= k2 < RG.nz and 0 <= i2 < RG.ny and 0 <= j2 < RG.nx:
                                lap[kz, i, j] += wgt * (x[kz, i, j] - x[k2, i2, j2])
    assert np.max(np.abs(gr - lap)) <= 1e-9 * np.max(np.abs(lap))


# ---- iteration --------------------------------------------------------------------------------------

def _tiny_problem(seed=0, M=3):
    g = TINY[0].replace(nsubsets=M)
    rng = np.random.default_rng(seed)
    xt = rng.uniform(0.0, 0.02, (g.nz, g.ny, g.nx))
    y = H.forward(g, xt) + rng.normal(0.0, 0.002, (g.nviews, g.nr, g.nb))
    w = rng.uniform(0.5, 2.0, y.shape)
    return g, y, w


def test_alpha_one_identity():
    """alpha = 1: h = D_L x - zeta after every subiteration (the unrelaxed h recursion)."""
    g, y, w = _tiny_problem()
    p = H.params(alpha=1.0, nsubsets=g.nsubsets, beta=1e-3)
    dl = H.dl(g, w)
    x, gv, h = H.rlalm_init(g, p, y, w, dl, np.full((g.nz, g.ny, g.nx), 0.01))
    for t in range(6):
        H.rlalm_iterate(g, p, y, w, dl, x, gv, h, t, 1)
        m = t % g.nsubsets
        views = np.arange(m, g.nviews, g.nsubsets)
        r = g.nsubsets * w[views] * (H.forward(g, x, views=views) - y[views])
        zeta = H.back(g, r, views=views)
        assert np.max(np.abs(dl * x - h - zeta)) <= 1e-10 * np.max(np.abs(zeta))


def test_sqs_case_descends():
    """One subset, alpha = 1, fixed rho = 1: the iteration is SQS, so the cost never increases."""
    g, y, w = _tiny_problem(M=1)
    p = H.params(alpha=1.0, nsubsets=1, rho_mode="fixed", rho_fixed=1.0, beta=1e-2)
    dl = H.dl(g, w)
    x, gv, h = H.rlalm_init(g, p, y, w, dl, np.zeros((g.nz, g.ny, g.nx)))
    c = H.cost(g, y, w, x, beta=1e-2)
    for t in range(15):
        H.rlalm_iterate(g, p, y, w, dl, x, gv, h, t, 1)
        c2 = H.cost(g, y, w, x, beta=1e-2)
        assert c2 <= c + 1e-12 * abs(c)
        c = c2


def test_one_voxel_recursion_by_hand():
    """A one-voxel volume with R = 0: every quantity is a scalar. With two subsets in bit-reversed order,
    the initial gradient comes from the last subset of the order and subiteration t uses rho_t in the x-step
    and in g+; the oracle must follow that recursion to 1e-12."""
    g = synth.HelicalGeometry(1, 1, 1, 2.0, 2.0, 2.0, 0.0, 6, 1.0, 0.0, 3, 1.0, 0.0, 8, 4, 0.3, -1.0, 1.0,
                              20.0, 40.0, 2)
    a = H.forward(g, np.ones((1, 1, 1)))
    assert np.all(a.sum(axis=(1, 2)) > 0)
    rng = np.random.default_rng(9)
    y = 0.7 * a + rng.normal(0.0, 0.05, a.shape)
    w = rng.uniform(0.5, 2.0, a.shape)
    alpha, M = 1.999, 2
    order = oracle.subset_order(M, "bitrev")
    L = float(np.sum(w * a * a))
    Lm = [float(np.sum((w * a * a)[m::M])) for m in range(M)]
    bm = [float(np.sum((w * a * y)[m::M])) for m in range(M)]

    def rho(t):
        if t == 0:
            return 1.0
        c = math.pi / (alpha * (t + 1))
        return c * math.sqrt(1 - (c / 2) ** 2)

    x = 0.2
    z = M * (Lm[order[-1]] * x - bm[order[-1]])
    gg, h = z, L * x - z
    p = H.params(alpha=alpha, nsubsets=M, beta=0.0, subset_order="bitrev")
    dl = H.dl(g, w)
    xo, go, ho = H.rlalm_init(g, p, y, w, dl, np.full((1, 1, 1), 0.2))
    for t in range(8):
        r = rho(t)
        x = max((r - 1) * gg / (r * L) + h / L, 0.0)
        m = order[t % M]
        z = M * (Lm[m] * x - bm[m])
        gg = r / (r + 1) * (alpha * z + (1 - alpha) * gg) + gg / (r + 1)
        h = alpha * (L * x - z) + (1 - alpha) * h
        H.rlalm_iterate(g, p, y, w, dl, xo, go, ho, t, 1)
        for got, want in ((xo, x), (go, gg), (ho, h)):
            assert abs(float(got.reshape(-1)[0]) - want) <= 1e-12 * max(1.0, abs(want)), (t, got, want)
