"""Pins of the oracle's regularizer R(x) = sum_i beta_i sum_n phi([C_i x]_n) (Section III, eq. def_reg),
its gradient and its Huber-curvature majorizer D_R (Section III-A): finite differences, the SQS
majorization inequality, the large-delta limit (weighted graph Laplacian) and closed forms at a
constant image."""
import math

import numpy as np
import pytest

import oracle


def laplacian(x, beta):
    """sum over the 4 directions of beta_i (2 x_j - x_{j+s} - x_{j-s}), only for in-image neighbours."""
    ny, nx = x.shape
    out = np.zeros_like(x)
    for (di, dj), b in (((0, 1), beta), ((1, 0), beta), ((1, 1), beta / math.sqrt(2)), ((1, -1), beta / math.sqrt(2))):
        for sgn in (1, -1):
            sh = np.full_like(x, np.nan)
            src = x[max(0, sgn * di):ny + min(0, sgn * di), max(0, sgn * dj):nx + min(0, sgn * dj)]
            sh[max(0, -sgn * di):ny + min(0, -sgn * di), max(0, -sgn * dj):nx + min(0, -sgn * dj)] = src
            m = ~np.isnan(sh)
            out[m] += b * (x[m] - sh[m])
    return out


@pytest.mark.parametrize("potential", ["hyperbola", "fair", "qggmrf"])
def test_gradient_matches_finite_differences(potential):
    rng = np.random.default_rng(1)
    x = rng.uniform(0.01, 0.03, (9, 11))
    delta, beta = 1e-3, 1024.0
    gr, _ = oracle.reg_grad(x, potential, delta, beta)
    eps = 1e-8
    for _ in range(40):
        i, j = rng.integers(9), rng.integers(11)
        xp, xm = x.copy(), x.copy()
        xp[i, j] += eps
        xm[i, j] -= eps
        fd = (oracle.reg_cost(xp, potential, delta, beta) - oracle.reg_cost(xm, potential, delta, beta)) / (2 * eps)
        assert abs(fd - gr[i, j]) <= 1e-6 * max(abs(gr[i, j]), beta * delta)


@pytest.mark.parametrize("potential", ["hyperbola", "fair", "qggmrf"])
@pytest.mark.parametrize("huber", [True, False])
def test_sqs_majorizes(potential, huber):
    """R(z) <= R(x) + grad R(x)'(z - x) + 1/2 ||z - x||^2_{D_R(x)} (Section II, majorization condition)."""
    rng = np.random.default_rng(2)
    delta, beta = 1e-3, 1024.0
    for _ in range(50):
        x = rng.uniform(0.0, 0.04, (8, 8))
        z = x + rng.normal(0, rng.choice([1e-4, 1e-3, 1e-2]), x.shape)
        gr, dr = oracle.reg_grad(x, potential, delta, beta, huber=huber)
        rhs = oracle.reg_cost(x, potential, delta, beta) + np.sum(gr * (z - x)) + 0.5 * np.sum(dr * (z - x) ** 2)
        lhs = oracle.reg_cost(z, potential, delta, beta)
        assert lhs <= rhs + 1e-12 * abs(rhs)


def test_large_delta_limit_is_laplacian():
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 0.04, (7, 10))
    beta = 512.0
    gr, dr = oracle.reg_grad(x, "hyperbola", 1e6, beta)
    np.testing.assert_allclose(gr, laplacian(x, beta), rtol=1e-9, atol=1e-12)


def test_curvature_closed_form_at_constant_image():
    beta = 1024.0
    _, dr = oracle.reg_grad(np.full((6, 6), 0.02), "hyperbola", 1e-4, beta)
    interior = 2 * (2 * beta + 2 * beta + 4 * beta / math.sqrt(2))
    corner = 2 * (beta + beta + beta / math.sqrt(2))
    edge = 2 * (2 * beta + beta + 2 * beta / math.sqrt(2))
    assert abs(dr[2, 3] - interior) < 1e-9 * interior
    assert abs(dr[0, 0] - corner) < 1e-9 * corner
    assert abs(dr[0, 3] - edge) < 1e-9 * edge


def pair_gradient(potential, delta, t):
    """phi'(t) through the oracle: R of the 1 x 2 image (0, t) is beta phi(-t) over the one horizontal pair,
    so its gradient at the second pixel is beta phi'(t)."""
    gr, dr = oracle.reg_grad(np.array([[0.0, t]]), potential, delta, 1.0)
    return gr[0, 1], dr[0, 1]


@pytest.mark.parametrize("potential", ["hyperbola", "fair", "qggmrf"])
def test_potentials_are_quadratic_near_zero(potential):
    """Every potential is t^2 / 2 to second order (Huber curvature 1 at t = 0): the same scale of delta."""
    d = 1e-3
    g, dr = pair_gradient(potential, d, 1e-9 * d)
    assert abs(g / (1e-9 * d) - 1.0) < 1e-6
    assert abs(dr - 2.0) < 1e-6   # D_R = 2 beta omega for the one pair


def test_qggmrf_tail_exponent():
    """q-GGMRF with p = 2, q = 1.2: phi'(t) grows like t^(q-1) for |t| >> delta (the published form's
    large-difference behaviour, q the exponent of the edge-preserving tail)."""
    d = 1e-3
    g1, _ = pair_gradient("qggmrf", d, 1e6 * d)
    g2, _ = pair_gradient("qggmrf", d, 1e7 * d)
    slope = math.log(g2 / g1) / math.log(10.0)
    assert abs(slope - 0.2) < 2e-3
