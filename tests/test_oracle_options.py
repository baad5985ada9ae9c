"""Pins of the oracle's optional pieces: certainty weights kappa in R (Section III, eq. def_reg, where
kappa_n weights each pair term), the bit-reversed subset order (the paper leaves the order open), and
the FBP-like start image (Algorithm 1 starts from an FBP image)."""
import math

import numpy as np
import pytest

import oracle
from paper_1512_04564_amd import synth


def test_kappa_of_uniform_weights():
    """w = c everywhere gives kappa = sqrt(c) wherever a ray meets the pixel."""
    g = synth.CFG1
    kap = oracle.kappa(g, np.full((g.nviews, g.nb), 9.0))
    assert np.all(kap > 0)
    np.testing.assert_allclose(kap, 3.0, rtol=1e-12)


def test_kappa_weighted_regularizer():
    rng = np.random.default_rng(11)
    x = rng.uniform(0.01, 0.03, (7, 9))
    kap = rng.uniform(0.5, 2.0, (7, 9))
    delta, beta = 1e-3, 100.0
    gr, dr = oracle.reg_grad_kappa(x, kap, "hyperbola", delta, beta)
    eps = 1e-8
    for _ in range(25):
        i, j = rng.integers(7), rng.integers(9)
        xp, xm = x.copy(), x.copy()
        xp[i, j] += eps
        xm[i, j] -= eps
        fd = (oracle.reg_cost_kappa(xp, kap, "hyperbola", delta, beta)
              - oracle.reg_cost_kappa(xm, kap, "hyperbola", delta, beta)) / (2 * eps)
        assert abs(fd - gr[i, j]) <= 1e-6 * max(abs(gr[i, j]), beta * delta)
    # kappa = 1 reproduces the plain regularizer
    g1, d1 = oracle.reg_grad_kappa(x, np.ones_like(x), "hyperbola", delta, beta)
    g0, d0 = oracle.reg_grad(x, "hyperbola", delta, beta)
    np.testing.assert_allclose(g1, g0, rtol=1e-14)
    np.testing.assert_allclose(d1, d0, rtol=1e-14)
    # majorization still holds with the weights
    z = x + rng.normal(0, 1e-3, x.shape)
    rhs = oracle.reg_cost_kappa(x, kap, "hyperbola", delta, beta) + np.sum(gr * (z - x)) + 0.5 * np.sum(dr * (z - x) ** 2)
    assert oracle.reg_cost_kappa(z, kap, "hyperbola", delta, beta) <= rhs + 1e-12 * abs(rhs)


def test_subset_orders():
    assert list(oracle.subset_order(8, "bitrev")) == [0, 4, 2, 6, 1, 5, 3, 7]
    assert list(oracle.subset_order(5, "sequential")) == [0, 1, 2, 3, 4]
    for M in (1, 3, 10, 12, 41):
        o = oracle.subset_order(M, "bitrev")
        assert sorted(o) == list(range(M))
        assert o[0] == 0


def test_bitrev_order_visits_every_subset_once_per_iteration():
    """Position m of an iteration uses the interleaved view set of subset order[m]; over one iteration
    every view is used exactly once."""
    M, nviews = 41, 984
    order = oracle.subset_order(M, "bitrev")
    seen = np.concatenate([oracle.subset_views(nviews, M, int(m)) for m in order])
    assert sorted(seen) == list(range(nviews))
    # consecutive subsets are far apart in angle (the point of the order), unlike the sequential one
    gaps = np.abs(np.diff(order.astype(int)))
    assert gaps.min() >= 2 and np.median(gaps) >= 8


def test_fbp_recovers_the_phantom():
    """The FBP-like start inverts noise-free analytic data: small error inside the field of view, and the
    mean attenuation of the body is right (a scale or geometry error fails this)."""
    g = synth.CFG1
    s = synth.noisy_scan(g, 3)
    x = oracle.fbp(g, s.line_integrals)
    mask = oracle.fov_mask(g, 0.9 * synth.fov_radius(g))
    err = np.abs(x - s.truth)[mask]
    assert np.median(err) < 0.02 * s.truth[mask].mean()
    assert abs(x[mask].mean() - s.truth[mask].mean()) < 0.02 * s.truth[mask].mean()
