"""Pins of the exact discrete length-scale conditional (oracle/exact_rho.py; Section 4.1,
the fourth conditional) against the dense formula and a library inverse CDF."""
import numpy as np
import pytest

from oracle import exact_rho, kernels, rng


def _chain(n=120, leaf=128, nugget=1e-3, tol=1e-13, seed=0):
    x = np.sort(np.random.default_rng(seed).uniform(0, 1, n))
    y = np.sin(5 * x) + 0.1 * np.random.default_rng(seed + 1).normal(size=n)
    grid = 0.1 * 10.0 ** ((np.arange(9) - 4) / 10.0)
    return x, y, exact_rho.ExactGridChain(x, y, kernels.SE, 0.1, nugget, leaf, tol, 20.0, 1.3,
                                          seed, grid=grid)


@pytest.mark.parametrize("leaf", [128, 16])
def test_probabilities_match_the_dense_conditional(leaf):
    """Pr(rho = s_h | -) proportional to det(K_h)^(-1/2) exp(-f' K_h^-1 f / 2), K_h =
    sigma_f^2 (K_1(s_h) + eta I), from dense slogdet and solve at every grid point."""
    x, y, ch = _chain(leaf=leaf)
    f = np.cos(4 * x)
    sigf2 = 0.8
    p, qs, lp = ch.probs(f, sigf2)
    ref = []
    for ell in ch.grid:
        K = sigf2 * kernels.K1_dense(kernels.SE, ell, 1e-3, x)
        ref.append(-0.5 * np.linalg.slogdet(K)[1] - 0.5 * f @ np.linalg.solve(K, f))
    ref = np.array(ref)
    pr = np.exp(ref - ref.max())
    np.testing.assert_allclose(p, pr / pr.sum(), rtol=1e-7, atol=1e-12)


def test_inverse_cdf_matches_searchsorted():
    g = np.random.default_rng(3)
    for _ in range(200):
        lp = g.normal(size=int(g.integers(1, 30))) * 5
        u = float(g.uniform())
        w = np.exp(lp - lp.max())
        c = np.cumsum(w)
        ref = min(int(np.searchsorted(c, u * c[-1], side="right")), lp.size - 1)
        assert exact_rho.inverse_cdf(lp, u) == ref
    assert exact_rho.inverse_cdf(np.array([0.0, -np.inf, 0.0]), 0.5 - 1e-12) == 0
    assert exact_rho.inverse_cdf(np.array([0.0, -np.inf, 0.0]), 0.5 + 1e-12) == 2
    # a uniform landing exactly on a cumulative boundary goes to the next index
    assert exact_rho.inverse_cdf(np.array([0.0, -np.inf, 0.0]), 0.5) == 2


def test_step_draws_with_its_uniform():
    x, y, ch = _chain(leaf=16)
    for _ in range(4):
        rec = ch.step()
        assert rec["u_rho"] == rng.uniform(0, rng.TAG_RHO, ch.it - 1, 0)
        assert rec["k"] == exact_rho.inverse_cdf(rec["lp"], rec["u_rho"])
        assert ch.logdet1 == ch.lds[rec["k"]]


def test_empirical_frequencies_follow_the_conditional():
    """Drawing many uniforms through the inverse CDF reproduces the probabilities."""
    x, y, ch = _chain()
    p, _, lp = ch.probs(np.cos(3 * x), 1.0)
    u = np.random.default_rng(5).uniform(size=20000)
    counts = np.bincount([exact_rho.inverse_cdf(lp, v) for v in u], minlength=p.size)
    assert np.abs(counts / u.size - p).max() < 4 * np.sqrt(p.max() / u.size) + 1e-3
