"""Pins of the oracle's Algorithm 1 / Algorithm 2 (Section III-A) and the continuation rho_k(alpha)
(Section III-B, eq. dec_rho; rationale in the supplement, section "Continuation with over-relaxation").

Against: the supplement's transition matrix T_i (critical damping at rho_k and the damping frequency),
exact algebraic identities of the recursion at alpha = 1, the closed-form minimiser of the x-step's prox
objective (eq. relaxed_lal_iter_quad), the fixed point at a KKT point, monotone descent in the SQS special
case, and the dense Cholesky solution of the unregularized problem.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1512_04564_amd import synth


def small_geom(M=4):
    return synth.ScanGeometry(nx=8, ny=8, dx=1.0, dy=1.0, nb=24, du=1.0, u_offset=0.0, det="flat", nviews=24,
                              beta0=0.1, span=2 * math.pi, dso=30.0, dsd=60.0, nsubsets=M)


def small_problem(M=4, seed=0, noise=0.01):
    g = small_geom(M)
    rng = np.random.default_rng(seed)
    x_true = rng.uniform(0.5, 1.5, (g.ny, g.nx))
    y = oracle.forward(g, x_true) + rng.normal(0, noise, (g.nviews, g.nb))
    w = rng.uniform(0.5, 2.0, (g.nviews, g.nb))
    return g, x_true, y, w


def dense_A(g):
    cols = []
    for p in range(g.ny * g.nx):
        e = np.zeros(g.ny * g.nx)
        e[p] = 1.0
        cols.append(oracle.forward(g, e.reshape(g.ny, g.nx)).reshape(-1))
    return np.stack(cols, axis=1)


# ---------------------------------------------------------------- continuation ---------------------

def transition(alpha, rho, lam_over_L):
    """T_i of the supplement (L_A = 1, lambda_i = lam_over_L)."""
    lam, L = lam_over_L, 1.0
    t11 = alpha * rho * lam / (rho + 1) * (rho - 1) / (rho * L) + ((1 - alpha) * rho + 1) / (rho + 1)
    t12 = alpha * rho * lam / (rho + 1) * rho / (rho * L)
    t21 = alpha * (L - lam) * (rho - 1) / (rho * L)
    t22 = alpha * (L - lam) * rho / (rho * L) + (1 - alpha)
    return np.array([[t11, t12], [t21, t22]])


@pytest.mark.parametrize("alpha", [1.0, 1.5, 1.999])
@pytest.mark.parametrize("k", [1, 2, 5, 40, 409, 4099])
def test_rho_is_critical_damping(alpha, k):
    """rho_k(alpha) is the critical AL penalty of the eigencomponent with lambda/L = (pi/(2 alpha (k+1)))^2:
    the characteristic polynomial of T has a double root there, for every alpha."""
    rho = oracle.rho(k, alpha)
    lam = (math.pi / (2 * alpha * (k + 1))) ** 2
    T = transition(alpha, rho, lam)
    tr, det = np.trace(T), np.linalg.det(T)
    disc = tr * tr - 4 * det
    assert abs(disc) <= 1e-12 * max(tr * tr, 1e-300)
    # slightly larger rho: real distinct roots (overdamped); slightly smaller: complex (underdamped)
    T_hi, T_lo = transition(alpha, rho * 1.01, lam), transition(alpha, rho * 0.99, lam)
    assert np.trace(T_hi) ** 2 - 4 * np.linalg.det(T_hi) > 0
    assert np.trace(T_lo) ** 2 - 4 * np.linalg.det(T_lo) < 0


def test_rho_start_and_monotone():
    for alpha in (1.0, 1.5, 1.999):
        assert oracle.rho(0, alpha) == 1.0
        vals = [oracle.rho(k, alpha) for k in range(1, 2000)]
        assert all(a > b for a, b in zip(vals, vals[1:]))
        assert vals[-1] <= math.pi / (alpha * 2000)


@pytest.mark.parametrize("alpha", [1.0, 1.999])
def test_damping_frequency_scales_with_alpha(alpha):
    """As rho -> 0, the smallest eigencomponent rotates at omega_1 ~ alpha sqrt(lambda_1 / L)."""
    lam = 1e-4
    T = transition(alpha, 1e-7, lam)
    cosw = np.trace(T) / math.sqrt(4 * np.linalg.det(T))
    omega = math.acos(cosw)
    assert abs(omega - alpha * math.sqrt(lam)) < 0.01 * alpha * math.sqrt(lam)


# ---------------------------------------------------------------- recursion algebra ----------------

def subset_gradient(g, y, w, x, m, M):
    views = oracle.subset_views(g.nviews, M, m)
    r = M * w[views] * (oracle.forward(g, x, views) - y[views])
    return oracle.back(g, r, views)


def test_alpha1_h_tracks_the_last_gradient():
    """With alpha = 1, h = D_L x - zeta holds exactly after every step, zeta the last subset gradient."""
    M = 4
    g, _, y, w = small_problem(M)
    p = oracle.params(alpha=1.0, niters=1, nsubsets=M, beta=10.0, delta=1e-2)
    dl = oracle.dl(g, w)
    x, gv, h = oracle.rlalm_init(g, p, y, w, dl, np.zeros((g.ny, g.nx)) + 0.3)
    np.testing.assert_allclose(dl * x - h, subset_gradient(g, y, w, x, M - 1, M), rtol=1e-12, atol=1e-12)
    for t in range(7):
        oracle.rlalm_iterate(g, p, y, w, dl, x, gv, h, t, 1)
        zeta = subset_gradient(g, y, w, x, t % M, M)
        np.testing.assert_allclose(dl * x - h, zeta, rtol=1e-10, atol=1e-10 * np.abs(zeta).max())


def test_alpha1_algorithms_coincide():
    """At alpha = 1 the proposed and the simple relaxation are both unrelaxed OS-LALM."""
    M = 4
    g, _, y, w = small_problem(M)
    x0 = np.full((g.ny, g.nx), 0.2)
    xa, _, _ = oracle.rlalm_solve(g, oracle.params(alpha=1.0, niters=10, nsubsets=M, algorithm=1), y, w, x0)
    xb, _, _ = oracle.rlalm_solve(g, oracle.params(alpha=1.0, niters=10, nsubsets=M, algorithm=2), y, w, x0)
    np.testing.assert_allclose(xa, xb, rtol=1e-9, atol=1e-12)  # differ only by rounding of D_L x - (D_L x - zeta)
    # and at alpha = 1.999 they differ
    xc, _, _ = oracle.rlalm_solve(g, oracle.params(alpha=1.999, niters=10, nsubsets=M, algorithm=1), y, w, x0)
    xd, _, _ = oracle.rlalm_solve(g, oracle.params(alpha=1.999, niters=10, nsubsets=M, algorithm=2), y, w, x0)
    assert np.abs(xc - xd).max() > 1e-6


def golden_min(f, lo, hi, iters=200):
    phi = (math.sqrt(5) - 1) / 2
    a, b = lo.copy(), hi.copy()
    c, d = b - phi * (b - a), a + phi * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(iters):
        left = fc < fd
        b = np.where(left, d, b)
        a = np.where(left, a, c)
        c2, d2 = b - phi * (b - a), a + phi * (b - a)
        c, d = c2, d2
        fc, fd = f(c), f(d)
    return 0.5 * (a + b)


@pytest.mark.parametrize("alpha,t0", [(1.999, 0), (1.999, 9), (1.5, 3)])
def test_xstep_minimises_the_prox_objective(alpha, t0):
    """x+ = argmin_{z >= 0} <grad R(x), z - x> + 1/2 ||z - x||^2_{D_R} + 1/2 ||z - (rho D_L)^-1 gamma||^2_{rho D_L}
    with gamma = (rho - 1) g + rho h (eq. relaxed_lal_iter_quad), evaluated per pixel by golden section."""
    M = 4
    g, _, y, w = small_problem(M, seed=3)
    p = oracle.params(alpha=alpha, niters=1, nsubsets=M, beta=20.0, delta=5e-2)
    dl = oracle.dl(g, w)
    x, gv, h = oracle.rlalm_init(g, p, y, w, dl, np.full((g.ny, g.nx), 0.4))
    oracle.rlalm_iterate(g, p, y, w, dl, x, gv, h, 0, t0)
    rho = oracle.rho(t0, alpha)
    gamma = (rho - 1) * gv + rho * h
    gr, dr = oracle.reg_grad(x, "hyperbola", 5e-2, 20.0)
    xk = x.copy()

    def F(z):
        return gr * (z - xk) + 0.5 * dr * (z - xk) ** 2 + 0.5 * rho * dl * (z - gamma / (rho * dl)) ** 2

    z = golden_min(F, np.zeros_like(x), np.full_like(x, 10.0))
    oracle.rlalm_iterate(g, p, y, w, dl, x, gv, h, t0, 1)
    np.testing.assert_allclose(x, z, rtol=1e-8, atol=1e-9)


def test_kkt_point_is_a_fixed_point():
    """With M = 1, (x_hat, g = grad L(x_hat), h = D_L x_hat - grad L(x_hat)) is left unchanged for any rho, alpha."""
    g, _, y, w = small_problem(1, seed=4, noise=0.3)
    delta, beta = 5e-2, 20.0
    xs, its, kkt = oracle.xstar(g, y, w, np.zeros((g.ny, g.nx)), delta=delta, beta=beta, maxit=40000,
                                step_tol=1e-16, kkt_tol=1e-14)
    assert kkt < 1e-12
    dl = oracle.dl(g, w)
    zeta = oracle.data_grad(g, y, w, xs)
    x, gv, h = xs.copy(), zeta.copy(), dl * xs - zeta
    p = oracle.params(alpha=1.999, niters=1, nsubsets=1, beta=beta, delta=delta)
    oracle.rlalm_iterate(g, p, y, w, dl, x, gv, h, 17, 5)
    np.testing.assert_allclose(x, xs, rtol=1e-8, atol=1e-9)


def test_sqs_special_case_descends():
    """M = 1, alpha = 1, rho = 1: the x-step is the SQS step, so the PWLS cost never increases."""
    g, _, y, w = small_problem(1, seed=5, noise=0.2)
    delta, beta = 1e-2, 30.0
    p = oracle.params(alpha=1.0, niters=1, nsubsets=1, rho_mode="fixed", rho_fixed=1.0, beta=beta, delta=delta,
                      init_full=True)
    dl = oracle.dl(g, w)
    x, gv, h = oracle.rlalm_init(g, p, y, w, dl, np.zeros((g.ny, g.nx)))
    costs = [oracle.cost(g, y, w, x, delta=delta, beta=beta)]
    for t in range(40):
        oracle.rlalm_iterate(g, p, y, w, dl, x, gv, h, t, 1)
        costs.append(oracle.cost(g, y, w, x, delta=delta, beta=beta))
    costs = np.array(costs)
    assert np.all(np.diff(costs) <= 1e-12 * np.abs(costs[:-1]))
    assert costs[-1] < 0.5 * costs[0]


@pytest.mark.parametrize("alpha", [1.0, 1.999])
def test_unregularized_solution_is_weighted_least_squares(alpha):
    """beta = 0, M = 1, interior solution: the iteration converges to (A'WA)^-1 A'W y (dense Cholesky)."""
    g, _, y, w = small_problem(1, seed=6, noise=0.02)
    A = dense_A(g)
    Wd = w.reshape(-1)
    H = A.T @ (Wd[:, None] * A)
    L = np.linalg.cholesky(H)
    xhat = np.linalg.solve(L.T, np.linalg.solve(L, A.T @ (Wd * y.reshape(-1)))).reshape(g.ny, g.nx)
    assert xhat.min() > 0.1
    p = oracle.params(alpha=alpha, niters=3000, nsubsets=1, rho_mode="fixed", rho_fixed=0.5, beta=0.0,
                      init_full=True)
    x, _, _ = oracle.rlalm_solve(g, p, y, w, np.zeros((g.ny, g.nx)))
    np.testing.assert_allclose(x, xhat, rtol=1e-8)
    xs, _, _ = oracle.xstar(g, y, w, np.zeros((g.ny, g.nx)), beta=0.0, maxit=20000, step_tol=1e-16, kkt_tol=1e-14)
    np.testing.assert_allclose(xs, xhat, rtol=1e-8)


def test_relaxation_speeds_up_early_iterations():
    """M = 1 on a small data-dominated CT problem: alpha = 1.999 reaches 100, 30 and 10 HU from x* in clearly
    fewer iterations than alpha = 1. The paper claims about twice as fast "at least in early iterations",
    with the speed-up diminishing near the solution (Sections I, IV)."""
    g = synth.ScanGeometry(nx=32, ny=32, dx=1.0, dy=1.0, nb=64, du=1.0, u_offset=0.0, det="flat", nviews=60,
                           beta0=0.0, span=2 * math.pi, dso=60.0, dsd=120.0, nsubsets=1)
    rng = np.random.default_rng(7)
    ell = [synth.Ellipse(0, 0, 12, 10, 0.3, 0.02), synth.Ellipse(3, -2, 3, 4, 0.0, 0.01)]
    counts = np.maximum(rng.poisson(1e4 * np.exp(-synth.analytic_sinogram(g, ell))).astype(float), 1.0)
    y, w = np.log(1e4 / counts), counts
    xs, _, kkt = oracle.xstar(g, y, w, np.zeros((g.ny, g.nx)), delta=1e-3, beta=1.0, maxit=20000,
                              step_tol=1e-14, kkt_tol=1e-12)
    assert kkt < 1e-12
    first = {}
    for alpha in (1.0, 1.999):
        p = oracle.params(alpha=alpha, niters=60, nsubsets=1, beta=1.0, delta=1e-3)
        _, _, tr = oracle.rlalm_solve(g, p, y, w, np.zeros((g.ny, g.nx)), xref=xs, mu_w=0.02)
        first[alpha] = [int(np.argmax(tr < th)) + 1 for th in (100.0, 30.0, 10.0)]
        assert all(f <= 60 and tr[f - 1] < th for f, th in zip(first[alpha], (100.0, 30.0, 10.0)))
    for f_relaxed, f_plain in zip(first[1.999], first[1.0]):
        assert f_relaxed <= 0.7 * f_plain


# ---------------------------------------------------------------- weight scaling -------------------

@pytest.mark.parametrize("kappa", [False, True])
def test_iterates_invariant_under_joint_scaling_of_weights_and_beta(kappa):
    """Scaling W and beta by one constant c scales the cost by c; in Algorithm 1 it scales D_L, zeta, g, h,
    grad R and D_R alike, so the x-step (numerator over denominator) and every x iterate are unchanged.
    With c a power of two the FP64 arithmetic is scaled exactly, so the iterates agree to rounding-free
    precision. With certainty weights kappa = sqrt(A'w / A'1) the regularizer already scales with W
    (kappa_j kappa_k scales by c), so beta stays. (Half-precision storage relies on this to bring
    count-sized weights into range.)"""
    g, _, y, w = small_problem(M=4, seed=3)
    w = w * 4000.0
    c = 2.0 ** -6
    x0 = np.zeros((g.ny, g.nx))
    p1 = oracle.params(alpha=1.999, niters=6, nsubsets=g.nsubsets, beta=2.0, delta=0.05, kappa=kappa)
    p2 = oracle.params(alpha=1.999, niters=6, nsubsets=g.nsubsets, beta=2.0 if kappa else 2.0 * c, delta=0.05,
                       kappa=kappa)
    x1, _, _ = oracle.rlalm_solve(g, p1, y, w, x0)
    x2, _, _ = oracle.rlalm_solve(g, p2, y, w * c, x0)
    assert np.abs(x1).max() > 0.1
    np.testing.assert_allclose(x2, x1, rtol=0, atol=1e-13 * np.abs(x1).max())
    # the other choice of beta changes the iterates (the test is not vacuous)
    p3 = oracle.params(alpha=1.999, niters=6, nsubsets=g.nsubsets, beta=2.0 * c if kappa else 2.0, delta=0.05,
                       kappa=kappa)
    x3, _, _ = oracle.rlalm_solve(g, p3, y, w * c, x0)
    assert np.abs(x3 - x1).max() > 1e-3 * np.abs(x1).max()
