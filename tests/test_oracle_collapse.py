"""Pins of the collapsed-data oracle (oracle/collapse.py; Appendix, 'Non-unique input
points'): the collapse against a loop over observations, the residual split, and --
deciding the reading of the printed diagonal -- sufficiency: the collapsed f step has
exactly the mean and covariance of the dense posterior given all n observations."""
import math

import numpy as np
import pytest

from oracle import collapse, hodlr, kernels, rng


def _data(U=24, seed=0):
    g = np.random.default_rng(seed)
    xu = np.sort(g.uniform(0, 1, U))
    reps = g.integers(1, 6, U)                      # |Q_i| from 1 to 5
    x = np.repeat(xu, reps)
    y = np.sin(6 * x) + 0.3 * g.normal(size=x.size)
    perm = g.permutation(x.size)                    # observation order does not matter
    return x[perm], y[perm], xu, reps


def test_collapse_against_a_loop():
    x, y, xu, reps = _data()
    cu, w, ybar, within = collapse.collapse(x, y)
    np.testing.assert_array_equal(cu, xu)
    np.testing.assert_array_equal(w, reps)
    s_w = 0.0
    for i, v in enumerate(xu):
        grp = [y[h] for h in range(x.size) if x[h] == v]
        assert ybar[i] == pytest.approx(sum(grp) / len(grp), rel=1e-14)
        s_w += sum((t - sum(grp) / len(grp)) ** 2 for t in grp)
    assert within == pytest.approx(s_w, rel=1e-12)


def test_residual_split():
    x, y, xu, reps = _data(seed=1)
    cu, w, ybar, within = collapse.collapse(x, y)
    f = np.cos(3 * cu)
    full = sum((y[h] - f[np.searchsorted(cu, x[h])]) ** 2 for h in range(x.size))
    assert np.sum(w * (ybar - f) ** 2) + within == pytest.approx(full, rel=1e-12)


def _chain(x, y, tau, sigf2, leaf=64):
    c = collapse.CollapsedChain(x, y, kernels.SE, 0.15, 1e-3, leaf, 1e-13, tau, sigf2, 4)
    return c


@pytest.mark.parametrize("leaf", [64, 8])
def test_sufficiency_of_the_averages(monkeypatch, leaf):
    """f | y (all n observations, y = A f_u + e, e ~ N(0, I / tau), f_u ~ N(0, sigma_f^2
    K~_1)) has precision (sigma_f^2 K~_1)^-1 + tau A'A and mean Lambda^-1 tau A'y.  The
    collapsed step's f is affine in its normals (a, b); reading it at zero and at unit
    vectors gives its mean and covariance, which must equal these."""
    x, y, xu, reps = _data(seed=2)
    tau, sigf2 = 3.0, 0.7
    U = xu.size
    ch = _chain(x, y, tau, sigf2, leaf)
    K = ch.H.dense()
    A = (x[:, None] == xu[None, :]).astype(float)
    Lam = np.linalg.inv(sigf2 * K) + tau * A.T @ A
    S = np.linalg.inv(Lam)
    m = S @ (tau * A.T @ y)

    def f_for(av, bv):
        vals = {rng.TAG_A: av, rng.TAG_B: bv}
        monkeypatch.setattr(collapse.rng, "normals", lambda n, sd, tag, t, s: vals[tag].copy())
        c = _chain(x, y, tau, sigf2, leaf)
        c._f_and_tau({})
        return c.f

    zero = np.zeros(U)
    mean = f_for(zero, zero)
    np.testing.assert_allclose(mean, m, rtol=1e-8, atol=1e-10)
    La = np.stack([f_for(np.eye(U)[j], zero) - mean for j in range(U)], axis=1)
    Lb = np.stack([f_for(zero, np.eye(U)[j]) - mean for j in range(U)], axis=1)
    np.testing.assert_allclose(La @ La.T + Lb @ Lb.T, S, rtol=1e-7, atol=1e-9 * np.abs(S).max())


def test_tau_step_uses_all_observations():
    x, y, xu, reps = _data(seed=3)
    ch = _chain(x, y, 2.0, 1.0)
    rec = {}
    ch._f_and_tau(rec)
    f_obs = ch.f[np.searchsorted(ch.x, x)]
    assert rec["sse"] == pytest.approx(float(np.sum((y - f_obs) ** 2)), rel=1e-12)
    g, _ = rng.gamma(0.5 * (1.0 + x.size), 4, rng.TAG_G_TAU, 0, 0)
    assert ch.tau == pytest.approx(g / (0.5 * (1.0 + rec["sse"])), rel=1e-14)


def test_loglik_is_that_of_the_averages():
    """ybar ~ N(0, sigma_f^2 K~_1 + diag(1 / (tau |Q_i|))), dense."""
    x, y, xu, reps = _data(seed=5)
    tau, sigf2 = 1.5, 0.9
    ch = _chain(x, y, tau, sigf2)
    rec = {}
    ch._f_and_tau(rec)
    C = sigf2 * ch.H.dense() + np.diag(1.0 / (tau * reps))
    ybar = ch.y
    ref = -0.5 * (xu.size * math.log(2 * math.pi) + np.linalg.slogdet(C)[1]
                  + ybar @ np.linalg.solve(C, ybar))
    assert rec["loglik"] == pytest.approx(ref, rel=1e-10)
    np.testing.assert_allclose(rec["r"], np.linalg.solve(C, ybar), rtol=1e-9)
