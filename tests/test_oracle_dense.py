"""Pins of O1 (oracle/dense.py) against closed forms and library routines."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import dense, kernels


def test_loglik_matches_scipy_mvn():
    rng = np.random.default_rng(0)
    x = np.sort(rng.uniform(0, 1, 40))
    y = rng.normal(size=40)
    K = 1.7 * kernels.K1_dense(kernels.SE, 0.2, 1e-6, x)
    ref = stats.multivariate_normal(mean=np.zeros(40), cov=K + np.eye(40) / 3.0).logpdf(y)
    assert dense.loglik(K, 3.0, y) == pytest.approx(ref, rel=1e-12)


def test_posterior_diagonal_closed_form():
    # ell -> 0: K = sigma^2 (1 + eta) I, so each coordinate is the scalar conjugate
    # posterior: var = k / (tau k + 1), mean = tau var y
    x = np.linspace(0, 1, 7)
    y = np.arange(7.0) - 3.0
    K = 2.0 * kernels.K1_dense(kernels.SE, 1e-6, 1e-6, x)
    k = 2.0 * (1 + 1e-6)
    mu, S = dense.posterior_f(K, 5.0, y)
    var = k / (5.0 * k + 1.0)
    np.testing.assert_allclose(np.diag(S), var, rtol=1e-14)
    np.testing.assert_allclose(mu, 5.0 * var * y, rtol=1e-14)
    assert np.abs(S - np.diag(np.diag(S))).max() < 1e-300 + 1e-15


def test_constant_kernel_logdet_closed_form():
    # ell -> infinity: K_1 = 1 1' + eta I, det = eta^(n-1) (eta + n)
    n, eta = 50, 1e-3
    x = np.linspace(0, 1, n)
    K1 = kernels.K1_dense(kernels.SE, 1e9, eta, x)
    assert dense.logdet_spd(K1) == pytest.approx((n - 1) * math.log(eta) + math.log(eta + n),
                                                 rel=1e-9)


def test_tau_conditional_brute_force():
    # p(tau | y, f) from prior x likelihood, normalised numerically
    rng = np.random.default_rng(1)
    n = 30
    y, f = rng.normal(size=n), rng.normal(size=n) * 0.5
    a1, b1 = 1.0, 1.0
    sse = float((y - f) @ (y - f))

    def logp(t):
        return ((a1 / 2 - 1) * math.log(t) - b1 * t / 2 + n / 2 * math.log(t) - t * sse / 2)

    grid_max = 20.0 * n / sse
    lo = math.exp(logp(1.0))
    Z = integrate.quad(lambda t: math.exp(logp(t) - logp(n / sse)), 0, grid_max, limit=200)[0]
    m = integrate.quad(lambda t: t * math.exp(logp(t) - logp(n / sse)), 0, grid_max, limit=200)[0]
    shape, rate = dense.tau_conditional(a1, b1, y, f)
    assert lo > 0
    assert m / Z == pytest.approx(shape / rate, rel=1e-8)


def test_rho_conditional_brute_force():
    # the discrete conditional equals the normalised N(0, K) densities of f
    rng = np.random.default_rng(2)
    n = 24
    x = np.sort(rng.uniform(0, 1, n))
    ells = [0.05, 0.1, 0.2, 0.4]
    f = rng.normal(size=n)
    p = dense.rho_conditional(kernels.SE, ells, 1e-4, x, 1.3, f)
    logs = np.array([stats.multivariate_normal(np.zeros(n), 1.3 * kernels.K1_dense(
        kernels.SE, e, 1e-4, x)).logpdf(f) for e in ells])
    ref = np.exp(logs - logs.max())
    np.testing.assert_allclose(p, ref / ref.sum(), rtol=1e-9)


def test_kl_zero_and_scalar():
    S = np.array([[2.0, 0.3], [0.3, 1.0]])
    assert abs(dense.kl_gauss(np.zeros(2), S, np.zeros(2), S)) < 1e-14
    # scalar closed form
    kl = dense.kl_gauss(np.array([0.0]), np.array([[1.0]]), np.array([1.0]), np.array([[4.0]]))
    assert kl == pytest.approx(math.log(2.0) + (1.0 + 1.0) / 8.0 - 0.5, rel=1e-14)


def test_dense_algorithm1_covariance_lemma():
    # Lemma 4.1 with exact matrices: f - mu is linear in (a, b); its covariance is
    # K M^-1 = Sigma_f of Eq. 3 (pushed through unit vectors)
    rng = np.random.default_rng(3)
    n, tau = 12, 7.0
    x = np.sort(rng.uniform(0, 1, n))
    K = 0.8 * kernels.K1_dense(kernels.SE, 0.3, 1e-6, x)
    y = rng.normal(size=n)
    f0, _, mu = dense.draw_f_dense(K, tau, y, np.zeros(n), np.zeros(n))
    cols = []
    for i in range(2 * n):
        e = np.zeros(2 * n)
        e[i] = 1.0
        fi, _, _ = dense.draw_f_dense(K, tau, y, e[:n], e[n:])
        cols.append(fi - f0)
    A = np.array(cols).T
    mu_ref, S_ref = dense.posterior_f(K, tau, y)
    np.testing.assert_allclose(A @ A.T, S_ref, atol=1e-12)
    np.testing.assert_allclose(mu, mu_ref, atol=1e-12)
