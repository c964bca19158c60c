"""Pins of Algorithm 1, Algorithm 1.h and the Gibbs sweep in oracle/sampler.py."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import hodlr, kernels, sampler, rng


def _setup(n=240, leaf=32, ell=0.1, tol=1e-10, seed=0):
    x = np.sort(np.random.default_rng(seed).uniform(0, 1, n))
    y = np.sin(2 * np.pi * x) + np.random.default_rng(seed + 1).normal(0, 0.2, n)
    H = hodlr.HODLR(x, kernels.SE, ell, 1e-6, leaf, tol)
    return x, y, H


def test_algorithm1_exact_covariance_lemma41():
    """Lemma 4.1: Z** ~ N(mu~, Sigma~) with Sigma~ = K~ M~^-1, mu~ = tau Sigma~ y.  The
    draw is affine in (a, b), so pushing unit vectors through it recovers its exact
    covariance (no sampling error)."""
    x, y, H = _setup()
    n, tau, s2 = x.size, 30.0, 1.7
    W1 = hodlr.Factor(H, 1.0, 0.0)
    WM = hodlr.Factor(H, tau * s2, 1.0)
    f0, r, mu = sampler.draw_f(H, W1, WM, s2, tau, y, np.zeros(n), np.zeros(n))
    A = np.empty((n, 2 * n))
    for i in range(2 * n):
        e = np.zeros(2 * n)
        e[i] = 1.0
        A[:, i] = sampler.draw_f(H, W1, WM, s2, tau, y, e[:n], e[n:])[0] - f0
    Kt = s2 * H.dense()
    M = tau * Kt + np.eye(n)
    Sig = np.linalg.solve(M.T, Kt.T).T
    np.testing.assert_allclose(A @ A.T, Sig, rtol=0, atol=1e-10 * np.abs(Sig).max())
    np.testing.assert_allclose(mu, tau * Sig @ y, rtol=0, atol=1e-9 * np.abs(mu).max())
    np.testing.assert_allclose(f0, mu, atol=1e-12)
    # M~ r = tau y  <=>  K~ r = y - r / tau (HODLR keeps the diagonal exactly)
    np.testing.assert_allclose(mu, y - r / tau, rtol=0, atol=1e-9 * np.abs(y).max())


def test_algorithm1h_exact_covariance():
    """Lemma for Algorithm 1.h: Z*** ~ N(K~ P~^-1 y, K~ P~^-1 D^-1), P~ = K~ + D^-1."""
    x, y, H = _setup(n=200)
    n = x.size
    D = np.random.default_rng(3).uniform(0.5, 40.0, n)
    WK = hodlr.Factor(H, 1.0, 0.0)
    WP = hodlr.Factor(H, 1.0, 0.0, 1.0 / D)
    f0, Rv = sampler.draw_f_hetero(H, WK, WP, D, y, np.zeros(n), np.zeros(n))
    A = np.empty((n, 2 * n))
    for i in range(2 * n):
        e = np.zeros(2 * n)
        e[i] = 1.0
        A[:, i] = sampler.draw_f_hetero(H, WK, WP, D, y, e[:n], e[n:])[0] - f0
    Kt = H.dense()
    P = Kt + np.diag(1.0 / D)
    Sig = np.linalg.solve(P.T, Kt.T).T / D[None, :]
    np.testing.assert_allclose(A @ A.T, Sig, rtol=0, atol=1e-9 * np.abs(Sig).max())
    np.testing.assert_allclose(Rv, Kt @ np.linalg.solve(P, y), rtol=0, atol=1e-9)


def test_chain_deterministic_and_resumable():
    x, y, _ = _setup(n=300, leaf=64)
    kw = dict(kind=kernels.SE, ell0=0.1, nugget=1e-6, leaf=64, tol=1e-10, tau0=25.0,
              sigf2_0=1.0, seed=42)
    c1 = sampler.Chain(x, y, **kw)
    c2 = sampler.Chain(x, y, **kw)
    for _ in range(4):
        r1, r2 = c1.step(), c2.step()
        assert (r1["tau"], r1["sigf2"], r1["k"]) == (r2["tau"], r2["sigf2"], r2["k"])
    np.testing.assert_array_equal(c1.f, c2.f)


@pytest.mark.slow
def test_gibbs_getting_it_right():
    """Geweke's successive-conditional check: alternating one Gibbs sweep with a fresh
    y ~ N(f, 1/tau) leaves the prior invariant, so the chain's marginals of tau and
    sigma_f^-2 (Ga(a/2, b/2), here a = b = 16 so the check mixes quickly) and of the
    grid index (uniform) must match the prior.  A wrong conditional (rate, MH ratio,
    draw of f) breaks this."""
    n = 6
    x = np.linspace(0.0, 1.0, n)
    grid = [0.2, 0.25, 0.3]
    ch = sampler.Chain(x, np.zeros(n), kernels.SE, 0.3, 1e-6, 64, 1e-10, 1.0, 1.0,
                       seed=7, grid=grid, priors=(16.0, 16.0, 16.0, 16.0))
    # start from a prior draw of f
    ch.f = np.linalg.cholesky(kernels.K1_dense(kernels.SE, grid[ch.k], 1e-6, x)) @ \
        rng.normals(n, 99, 9, 0, 0)
    taus, prec, ks = [], [], []
    for it in range(12000):
        e = rng.normals(n, 99, 8, it, 0)
        ch.y = ch.f + e / math.sqrt(ch.tau)
        ch.step()
        if it >= 500 and it % 3 == 0:
            taus.append(ch.tau)
            prec.append(1.0 / ch.sigf2)
            ks.append(ch.k)
    chi = stats.gamma(8.0, scale=1.0 / 8.0)
    # autocorrelated draws: compare coarse quantiles with generous bands
    for v in (np.array(taus), np.array(prec)):
        for q in (0.25, 0.5, 0.75):
            assert abs(np.mean(v < chi.ppf(q)) - q) < 0.04
    freq = np.bincount(ks, minlength=3) / len(ks)
    np.testing.assert_allclose(freq, 1.0 / 3.0, atol=0.03)
