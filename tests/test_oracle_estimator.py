"""Closed-form pins of the oracle's perturbation draw and gradient combination.

The renderer is replaced by scalar objectives L(x) whose Gaussian-smoothed
gradients are known exactly: a step (erf), a product of steps, a quadratic.
Each estimate must agree with the closed form within 4 standard errors.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

Phi, phi = stats.norm.cdf, stats.norm.pdf


def estimate(mode, theta, sigma, P, seed, Lfun):
    theta = np.asarray(theta, np.float32)
    sigma = np.asarray(sigma, np.float32)
    tau, c = O.draw_tau(mode, sigma, P, seed)
    Xp = (theta[None, :] + tau).astype(np.float32)
    Xm = (theta[None, :] - tau).astype(np.float32)
    L = np.empty(2 * P)
    L[0::2] = Lfun(Xp.astype(np.float64))
    L[1::2] = Lfun(Xm.astype(np.float64))
    g, q = O.combine(c, L)
    terms = c * (L[0::2] - L[1::2])[:, None]          # per-pair contributions
    se = terms.std(axis=0, ddof=1) / math.sqrt(P)
    return g, q, se, terms, tau, L


def step(a):
    return lambda X: (X[:, 0] > a).astype(np.float64)


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS, O.IS_PERDIM])
@pytest.mark.parametrize("theta,a,sigma", [(0.3, 0.0, 0.5), (-0.7, 0.2, 0.25), (1.5, 0.0, 1.0)])
def test_erf_step_1d(mode, theta, a, sigma):
    # Q(theta) = Phi((theta - a)/sigma), dQ/dtheta = phi((theta - a)/sigma)/sigma
    g, q, se, *_ = estimate(mode, [theta], [sigma], 40000, 17, step(a))
    truth = phi((theta - a) / sigma) / sigma
    assert abs(g[0] - truth) <= 4 * se[0] + 1e-12, (g, truth, se)


def test_is_constant_and_sign_against_paper_algorithm():
    # For d = 1 the importance-sampled pair term is sqrt(2/pi)/sigma times the
    # paper's per-iteration increment (L(theta+tau) - L(theta-tau)) / 2 with
    # tau = sqrt(-2 sigma^2 ln xi) > 0 (up to the pair's random sign).
    sigma = float(np.float32(0.4))          # the estimator receives binary32 sigma
    g, q, se, terms, tau, L = estimate(O.IS, [0.1], [sigma], 2000, 3, step(0.0))
    tau_abs = np.abs(tau[:, 0].astype(np.float64))
    sgn = np.sign(tau[:, 0])
    alg1_increment = (L[0::2] - L[1::2]) * sgn          # L(theta+|tau|) - L(theta-|tau|)
    np.testing.assert_allclose(terms[:, 0], math.sqrt(2 / math.pi) / (2 * sigma) * alg1_increment,
                               rtol=1e-15, atol=0)
    assert (tau_abs > 0).all()


def test_zero_variance_at_the_step():
    # theta = a: every importance-sampled pair gives exactly 1/(sigma sqrt(2 pi))
    sigma = float(np.float32(0.3))
    _, _, _, terms, _, _ = estimate(O.IS, [0.0], [sigma], 5000, 23, step(0.0))
    truth = 1.0 / (sigma * math.sqrt(2 * math.pi))
    assert np.all(terms[:, 0] == terms[0, 0])
    assert abs(terms[0, 0] - truth) <= 2 * np.spacing(truth)


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS, O.IS_PERDIM])
@pytest.mark.parametrize("d", [1, 3, 12])
def test_antithetic_zero_for_symmetric_objective(mode, d):
    # L symmetric about theta = 0: L(tau) = L(-tau) exactly, so the estimate is 0
    sigma = np.linspace(0.1, 0.9, d)
    g, *_ = estimate(mode, np.zeros(d), sigma, 257, 5, lambda X: (X * X).sum(axis=1))
    assert np.all(g == 0.0)


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS])
def test_product_of_steps_2d(mode):
    theta = np.array([0.2, -0.1])
    a = np.array([0.5, -0.3])
    sigma = np.array([0.3, 0.5])
    L = lambda X: ((X[:, 0] > a[0]) & (X[:, 1] > a[1])).astype(np.float64)
    g, q, se, *_ = estimate(mode, theta, sigma, 60000, 99, L)
    z = (theta - a) / sigma
    truth = np.array([phi(z[0]) / sigma[0] * Phi(z[1]), phi(z[1]) / sigma[1] * Phi(z[0])])
    assert np.all(np.abs(g - truth) <= 4 * se), (g, truth, se)


def test_per_dimension_reading_is_biased_in_2d():
    # The literal per-axis Rayleigh sampler is exact for d = 1 but not for a
    # non-separable objective in d = 2 (documented reading; default is the radial one).
    theta = np.array([0.2, -0.1])
    a = np.array([0.5, -0.3])
    sigma = np.array([0.3, 0.5])
    L = lambda X: ((X[:, 0] > a[0]) & (X[:, 1] > a[1])).astype(np.float64)
    g, q, se, *_ = estimate(O.IS_PERDIM, theta, sigma, 60000, 99, L)
    z = (theta - a) / sigma
    truth = np.array([phi(z[0]) / sigma[0] * Phi(z[1]), phi(z[1]) / sigma[1] * Phi(z[0])])
    assert np.any(np.abs(g - truth) > 8 * se)


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS])
@pytest.mark.parametrize("d", [6, 12, 150, 256])
def test_quadratic(mode, d):
    # L = |x - c|^2: Q = |theta - c|^2 + sum sigma^2, grad Q = 2 (theta - c)
    rng = np.random.default_rng(d)
    theta = rng.uniform(-1, 1, d)
    cc = rng.uniform(-1, 1, d)
    sigma = rng.uniform(0.1, 0.6, d)
    L = lambda X: ((X - cc[None, :]) ** 2).sum(axis=1)
    g, q, se, *_ = estimate(mode, theta.astype(np.float32), sigma.astype(np.float32), 30000, 7, L)
    th32 = theta.astype(np.float32).astype(np.float64)
    truth = 2.0 * (th32 - cc)
    assert np.all(np.abs(g - truth) <= 4 * se + 1e-6), (g, truth, se)


def test_gauss_loss_mean_is_smoothed_objective():
    # GAUSS draws: mean of L over the 2P images estimates Q; for the quadratic
    # Q = |theta - c|^2 + sum sigma^2
    d = 4
    theta = np.array([0.1, -0.2, 0.3, 0.0], np.float32)
    sigma = np.array([0.2, 0.3, 0.4, 0.5], np.float32)
    cc = np.array([0.5, 0.5, -0.5, 0.0])
    L = lambda X: ((X - cc[None, :]) ** 2).sum(axis=1)
    g, q, se, terms, tau, Ls = estimate(O.GAUSS, theta, sigma, 50000, 8, L)
    truth = ((theta.astype(np.float64) - cc) ** 2).sum() + (sigma.astype(np.float64) ** 2).sum()
    pair_mean = 0.5 * (Ls[0::2] + Ls[1::2])
    assert abs(q - truth) <= 4 * pair_mean.std(ddof=1) / math.sqrt(pair_mean.size)


def test_rayleigh_magnitude_matches_supplement_cdf():
    # d = 1 importance sampling: |tau| has CDF 1 - exp(-t^2 / (2 sigma^2)) on each
    # half-space (supplement CDF with C+ = 1, C- = 0); sign is balanced.
    sigma = 0.7
    tau, c = O.draw_tau(O.IS, [sigma], 50000, 41)
    t = tau[:, 0].astype(np.float64)
    p = stats.kstest(np.abs(t) / sigma, stats.rayleigh.cdf).pvalue
    assert p > 1e-3
    assert abs(np.mean(np.abs(t)) - sigma * math.sqrt(math.pi / 2)) < 4 * np.std(np.abs(t)) / math.sqrt(t.size)
    assert abs(np.mean(t * t) - 2 * sigma**2) < 4 * np.std(t * t) / math.sqrt(t.size)
    assert abs(np.mean(t > 0) - 0.5) < 4 * 0.5 / math.sqrt(t.size)
    # signed CDF: F = 1 - exp(-t^2/2s^2)/2 for t > 0, exp(-t^2/2s^2)/2 for t < 0
    F = lambda x: np.where(x > 0, 1 - 0.5 * np.exp(-x**2 / (2 * sigma**2)),
                           0.5 * np.exp(-x**2 / (2 * sigma**2)))
    assert stats.kstest(t, F).pvalue > 1e-3
    assert stats.kstest(O.draw_tau(O.IS_PERDIM, [sigma], 50000, 43)[0][:, 0], F).pvalue > 1e-3


@pytest.mark.parametrize("d", [2, 3, 6, 12, 150, 256])
def test_radial_sampler_is_chi_d_plus_1(d):
    sigma = np.full(d, 0.5, np.float32)
    tau, c = O.draw_tau(O.IS, sigma, 20000, 100 + d)
    r = np.linalg.norm(tau.astype(np.float64) / 0.5, axis=1)
    assert stats.kstest(r, stats.chi(d + 1).cdf).pvalue > 1e-3
    u = tau / np.linalg.norm(tau, axis=1, keepdims=True)
    cov = (u.T @ u) / u.shape[0]
    assert np.abs(cov - np.eye(d) / d).max() < 0.03
    # pair weight C_d u_j / (2 sigma_j)
    np.testing.assert_allclose(c, O.chi_mean(d) * u / (2 * 0.5), rtol=2e-6, atol=1e-7)


@pytest.mark.parametrize("d", [1, 2, 5])
def test_gauss_sampler_is_normal(d):
    sigma = np.full(d, 0.3, np.float32)
    tau, c = O.draw_tau(O.GAUSS, sigma, 20000, 200 + d)
    for j in range(d):
        assert stats.kstest(tau[:, j] / 0.3, stats.norm.cdf).pvalue > 1e-3
    np.testing.assert_allclose(c, tau.astype(np.float64) / 0.3 / (2 * 0.3), rtol=1e-6)


@pytest.mark.parametrize("d", [32, 33, 70])
def test_per_axis_signs_past_32_axes(d):
    # one sign word per 32 axes: every axis is balanced, and axes 32 apart do
    # not share their signs; the radii are Rayleigh on every axis
    P = 20000
    tau, c = O.draw_tau(O.IS_PERDIM, np.full(d, 0.5, np.float32), P, 300 + d)
    sg = tau > 0
    assert np.all(np.abs(sg.mean(0) - 0.5) < 4 * 0.5 / math.sqrt(P))
    for j in range(d - 32):
        assert abs((sg[:, j] == sg[:, j + 32]).mean() - 0.5) < 4 * 0.5 / math.sqrt(P)
    assert stats.kstest(np.abs(tau[:, d - 1]) / 0.5, stats.rayleigh.cdf).pvalue > 1e-3
    np.testing.assert_array_equal(np.sign(c), np.sign(tau))


def test_draw_is_a_function_of_seed_and_pair_only():
    t1, _ = O.draw_tau(O.IS, [0.5, 0.5, 0.5], 8, 1234)
    t2, _ = O.draw_tau(O.IS, [0.5, 0.5, 0.5], 16, 1234)
    assert np.array_equal(t1, t2[:8])
    t3, _ = O.draw_tau(O.IS, [0.5, 0.5, 0.5], 8, 1235)
    assert not np.array_equal(t1, t3)


def test_sigma_schedule_and_adam():
    assert O.sigma_schedule(1.0, 0.05, 0, 200) == 1.0
    assert abs(O.sigma_schedule(1.0, 0.05, 199, 200) - 0.05) < 1e-15
    assert abs(O.sigma_schedule(1.0, 0.05, 100, 200) - (1.0 - 0.95 * 100 / 199)) < 1e-15
    # constant gradient: bias-corrected moments equal g and g^2, every step is
    # lr g / (|g| + eps)
    th = np.array([0.0, 1.0, -2.0])
    m, v = np.zeros(3), np.zeros(3)
    g = np.array([0.3, -2.0, 1e-3])
    for t in range(1, 6):
        before = th.copy()
        O.adam_step(th, g, m, v, t, 0.01)
        np.testing.assert_allclose(before - th, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_plateau_loss_is_flat_without_overlap():
    # Sec. 2.1: a black sphere over a constant background; while its silhouette
    # does not overlap the reference one, small moves leave the point-sampled
    # image loss exactly unchanged (the plateau: zero gradient almost
    # everywhere, level up to the disk's pixel coverage), and it drops once
    # they overlap
    from paper_2211_17263_amd import scenes as S
    osc = O.OracleScene(S.plateau_scene())
    ref = osc.reference(np.zeros(2, np.float32), seed=5)

    def loss(th):
        img = osc.reference(np.array(th, np.float32), seed=5)
        return float(((img - ref) ** 2).mean())

    here = loss((0.9, 0.9))
    assert here > 0 and loss((0.9001, 0.9)) == here and loss((0.9, 0.9001)) == here
    flat = [loss(th) for th in ((0.9, 0.9), (0.95, 0.9), (-1.2, 0.3), (0.2, -1.3))]
    assert max(flat) / min(flat) - 1.0 < 0.05
    assert loss((0.5, 0.5)) < 0.9 * min(flat)
    assert loss((0.3, 0.3)) < loss((0.5, 0.5))
    assert loss((0.0, 0.0)) == 0.0


def estimate_independent(mode, theta, sigma, N, seed, Lfun):
    """Independent draws (no antithetic partner): g = mean of c_i L(theta + tau_i)."""
    theta = np.asarray(theta, np.float32)
    sigma = np.asarray(sigma, np.float32)
    tau, c = O.draw_tau(mode | O.INDEPENDENT, sigma, N, seed)
    X = (theta[None, :] + tau).astype(np.float32)
    L = Lfun(X.astype(np.float64))
    g, q = O.combine_independent(c, L)
    terms = c * L[:, None]
    se = terms.std(axis=0, ddof=1) / math.sqrt(N)
    return g, q, se, terms


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS])
@pytest.mark.parametrize("theta,a,sigma", [(0.3, 0.0, 0.5), (-0.7, 0.2, 0.25)])
def test_independent_erf_step_1d(mode, theta, a, sigma):
    # without antithetic partners the estimator stays unbiased (the noAT arm of Sec. 4.4, Tab. 4)
    g, q, se, _ = estimate_independent(mode, [theta], [sigma], 80000, 23, step(a))
    truth = phi((theta - a) / sigma) / sigma
    assert abs(g[0] - truth) <= 4 * se[0], (g, truth, se)


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS])
def test_independent_product_of_steps_and_quadratic(mode):
    theta = np.array([0.2, -0.1])
    a = np.array([0.5, -0.3])
    sigma = np.array([0.3, 0.5])
    L = lambda X: ((X[:, 0] > a[0]) & (X[:, 1] > a[1])).astype(np.float64)
    g, q, se, _ = estimate_independent(mode, theta, sigma, 120000, 31, L)
    z = (theta - a) / sigma
    truth = np.array([phi(z[0]) / sigma[0] * Phi(z[1]), phi(z[1]) / sigma[1] * Phi(z[0])])
    assert np.all(np.abs(g - truth) <= 4 * se), (g, truth, se)
    rng = np.random.default_rng(3)
    d = 6
    th = rng.uniform(-1, 1, d).astype(np.float32)
    cc = rng.uniform(-1, 1, d)
    sg = rng.uniform(0.1, 0.6, d).astype(np.float32)
    Lq = lambda X: ((X - cc[None, :]) ** 2).sum(axis=1)
    g, q, se, _ = estimate_independent(mode, th, sg, 200000, 5, Lq)
    truth = 2.0 * (th.astype(np.float64) - cc)
    assert np.all(np.abs(g - truth) <= 4 * se), (g, truth, se)


def test_independent_weights_are_twice_the_pair_weights_and_lose_zero_variance():
    # same draws; single-sample score weights = 2 x antithetic pair weights; at the
    # step (theta = a) the antithetic estimate has zero variance, the
    # independent one does not
    for mode in (O.GAUSS, O.IS, O.IS_PERDIM):
        t1, c1 = O.draw_tau(mode, [0.5, 0.3, 0.2], 64, 9)
        t2, c2 = O.draw_tau(mode | O.INDEPENDENT, [0.5, 0.3, 0.2], 64, 9)
        assert np.array_equal(t1, t2) and np.array_equal(2.0 * c1, c2)
    *_, terms_at, _, _ = estimate(O.IS, [0.0], [0.5], 2000, 3, step(0.0))
    _, _, _, terms_ind = estimate_independent(O.IS, [0.0], [0.5], 2000, 3, step(0.0))
    assert np.ptp(terms_at) == 0.0
    assert terms_ind.std() > 0.5 * np.abs(terms_ind.mean())


# ---- stratified draws (the alternative to antithetic pairs of Sec. 3.2) ----

@pytest.mark.parametrize("mode", [O.IS, O.IS_PERDIM])
@pytest.mark.parametrize("N", [2, 7, 64])
def test_stratified_draws_cover_each_stratum_once(mode, N):
    # d = 1: |v_i| = sqrt(-2 ln xi_i), so xi_i = exp(-v_i^2 / 2) recovers the
    # draw's first uniform, which must lie in stratum i of N
    sigma = 0.4
    tau, c = O.draw_tau(mode | O.INDEPENDENT | O.STRATIFIED, [sigma], N, 17)
    xi = np.exp(-0.5 * (tau[:, 0].astype(np.float64) / sigma) ** 2)
    pos = xi * N - np.arange(N)
    assert np.all(pos > -1e-4) and np.all(pos < 1.0 + 1e-4), pos
    # the plain independent draws of the same seed are not stratified
    t2, _ = O.draw_tau(mode | O.INDEPENDENT, [sigma], N, 17)
    if N == 64:
        x2 = np.exp(-0.5 * (t2[:, 0].astype(np.float64) / sigma) ** 2)
        assert np.any(np.abs(x2 * N - np.arange(N) - 0.5) > 1.0)


def test_stratified_needs_independent_draws():
    with pytest.raises(ValueError):
        O.draw_tau(O.IS | O.STRATIFIED, [0.3], 4, 1)


def stratified_estimates(mode, theta, sigma, N, seeds, Lfun):
    out = []
    for s in seeds:
        tau, c = O.draw_tau(mode, np.asarray(sigma, np.float32), N, s)
        X = (np.asarray(theta, np.float32)[None, :] + tau).astype(np.float64)
        g, _ = O.combine_independent(c, Lfun(X))
        out.append(g)
    return np.array(out)


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS])
def test_stratified_erf_step_1d_unbiased_and_less_variable(mode):
    # each stratum is sampled from its own conditional law, so the mean over
    # seeds is grad Q exactly as for plain independent draws; stratifying the
    # radius (IS) or the Box-Muller radius (GAUSS) lowers the variance here
    theta, a, sigma, N = 0.3, 0.0, 0.5, 16
    truth = phi((theta - a) / sigma) / sigma
    seeds = range(3000)
    gs = stratified_estimates(mode | O.INDEPENDENT | O.STRATIFIED, [theta], [sigma], N, seeds,
                              step(a))[:, 0]
    gi = stratified_estimates(mode | O.INDEPENDENT, [theta], [sigma], N, seeds, step(a))[:, 0]
    se = gs.std(ddof=1) / math.sqrt(len(gs))
    assert abs(gs.mean() - truth) <= 4 * se, (gs.mean(), truth, se)
    assert gs.var() < gi.var(), (gs.var(), gi.var())


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS, O.IS_PERDIM])
def test_stratified_unbiased_in_several_dimensions(mode):
    # d > 1: only the first uniform of each draw is stratified, and each
    # stratum keeps its conditional law, so the estimate stays unbiased: the
    # mean over seeds of the product-of-steps and quadratic gradients equals
    # the closed form (the per-axis sampler is biased for the non-separable
    # product of steps, so it is checked on the separable quadratic only)
    seeds = range(1500)
    if mode != O.IS_PERDIM:
        theta = np.array([0.2, -0.1])
        a = np.array([0.5, -0.3])
        sigma = np.array([0.3, 0.5])
        L = lambda X: ((X[:, 0] > a[0]) & (X[:, 1] > a[1])).astype(np.float64)
        gs = stratified_estimates(mode | O.INDEPENDENT | O.STRATIFIED, theta, sigma, 16, seeds, L)
        z = (theta - a) / sigma
        truth = np.array([phi(z[0]) / sigma[0] * Phi(z[1]), phi(z[1]) / sigma[1] * Phi(z[0])])
        se = gs.std(axis=0, ddof=1) / math.sqrt(len(gs))
        assert np.all(np.abs(gs.mean(axis=0) - truth) <= 4 * se), (gs.mean(axis=0), truth, se)
    rng = np.random.default_rng(11)
    d = 6
    th = rng.uniform(-1, 1, d).astype(np.float32)
    cc = rng.uniform(-1, 1, d)
    sg = rng.uniform(0.1, 0.6, d).astype(np.float32)
    Lq = lambda X: ((X - cc[None, :]) ** 2).sum(axis=1)
    gq = stratified_estimates(mode | O.INDEPENDENT | O.STRATIFIED, th, sg, 16, seeds, Lq)
    truth = 2.0 * (th.astype(np.float64) - cc)
    se = gq.std(axis=0, ddof=1) / math.sqrt(len(gq))
    assert np.all(np.abs(gq.mean(axis=0) - truth) <= 4 * se + 1e-9), (gq.mean(axis=0), truth, se)
