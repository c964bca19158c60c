"""Pins of the oracle's function posterior at new inputs (oracle/predict.py; Appendix,
'Function posterior at new inputs') against closed forms and an independent route: the
conditional of one coordinate of a joint Gaussian read off its precision matrix."""
import math

import numpy as np
import pytest

from oracle import hodlr, kernels, predict, rng


def _setup(n, leaf, ell=0.1, nugget=1e-3, tol=1e-12, seed=0):
    x = np.sort(np.random.default_rng(seed).uniform(0, 1, n))
    H = hodlr.HODLR(x, kernels.SE, ell, nugget, leaf, tol)
    W1 = hodlr.Factor(H, 1.0, 0.0)
    f = W1.apply_W(np.random.default_rng(seed + 1).normal(size=n))  # a draw from N(0, K~_1)
    return x, H, W1, f


def test_matches_joint_gaussian_precision():
    """Single leaf (K~_1 = K_1 + eta I exactly).  For the joint Gaussian of (f, f_*) with
    covariance sigma_f^2 [[K~_1, k], [k', 1 + eta]], f_* | f has variance 1 / P_** and mean
    -P_*n f / P_** where P is the inverse of the joint covariance."""
    n, sigf2 = 60, 1.7
    x, H, W1, f = _setup(n, leaf=64)
    xs = np.array([0.013, 0.5, 0.77777, 1.2])
    fs, mu, s2 = predict.predict(H, W1, f, sigf2, xs, np.zeros(xs.size))
    for j, xj in enumerate(xs):
        pts = np.append(x, xj)
        C = sigf2 * (kernels.K1_dense(kernels.SE, 0.1, 1e-3, pts))
        P = np.linalg.inv(C)
        assert mu[j] == pytest.approx(-P[n, :n] @ f / P[n, n], rel=1e-9, abs=1e-11)
        assert s2[j] == pytest.approx(1.0 / P[n, n], rel=1e-8)
        assert fs[j] == mu[j]


def test_at_a_training_input_closed_form():
    """x_* = x_i with K~_1 exact: k_{*n} = K~_1[i] - eta e_i, so mu_* = f_i - eta v_i with
    v = K~_1^-1 f, and sigma_*^2 = sigma_f^2 (2 eta - eta^2 (K~_1^-1)_ii)."""
    n, sigf2, eta = 50, 0.8, 1e-3
    x, H, W1, f = _setup(n, leaf=64)
    A = H.dense()
    v = np.linalg.solve(A, f)
    Ai = np.linalg.inv(A)
    idx = [0, 17, 49]
    _, mu, s2 = predict.predict(H, W1, f, sigf2, x[idx], np.zeros(3))
    for j, i in enumerate(idx):
        assert mu[j] == pytest.approx(f[i] - eta * v[i], rel=1e-9, abs=1e-12)
        assert s2[j] == pytest.approx(sigf2 * (2 * eta - eta * eta * Ai[i, i]), rel=1e-6)


def test_far_from_the_data_is_the_prior():
    n, sigf2 = 500, 2.5
    x, H, W1, f = _setup(n, leaf=64)
    xi = np.array([0.3, -1.1])
    fs, mu, s2 = predict.predict(H, W1, f, sigf2, np.array([-50.0, 80.0]), xi)
    assert np.all(mu == 0.0)
    np.testing.assert_array_equal(s2, sigf2 * (1.0 + 1e-3))
    np.testing.assert_allclose(fs, math.sqrt(sigf2 * 1.001) * xi, rtol=1e-15)


def test_single_observation_closed_form():
    x = np.array([0.4])
    H = hodlr.HODLR(x, kernels.SE, 0.2, 1e-6, 16, 1e-10)
    W1 = hodlr.Factor(H, 1.0, 0.0)
    f, sigf2, xs = np.array([1.3]), 0.9, np.array([0.1, 0.4, 0.55])
    _, mu, s2 = predict.predict(H, W1, f, sigf2, xs, np.zeros(3))
    k = np.exp(-(xs - 0.4) ** 2 / (2 * 0.04))
    np.testing.assert_allclose(mu, k * 1.3 / (1 + 1e-6), rtol=1e-14)
    np.testing.assert_allclose(s2, sigf2 * (1 + 1e-6 - k * k / (1 + 1e-6)), rtol=1e-9, atol=1e-15)


def test_hodlr_levels_match_the_dense_posterior():
    """Several levels with tol 1e-12 and a 1e-3 nugget: the compressed posterior agrees
    with the dense one to the perturbation the max-norm bound allows, kappa(K~_1) tol."""
    n, sigf2 = 1500, 1.0
    x, H, W1, f = _setup(n, leaf=64, ell=0.05)
    xs = np.random.default_rng(9).uniform(-0.1, 1.1, 40)
    _, mu, s2 = predict.predict(H, W1, f, sigf2, xs, np.zeros(40))
    A = kernels.K1_dense(kernels.SE, 0.05, 1e-3, x)
    Kx = kernels.k1(kernels.SE, 0.05, x, xs)
    mu_d = Kx.T @ np.linalg.solve(A, f)
    s2_d = sigf2 * (1.0 + 1e-3 - np.sum(Kx * np.linalg.solve(A, Kx), axis=0))
    kap = np.linalg.cond(A)
    bound = kap * n * 1e-12 / np.linalg.norm(A, 2)
    assert np.abs(mu - mu_d).max() <= bound * np.abs(np.linalg.solve(A, f)).sum()
    assert np.abs(s2 - s2_d).max() <= bound * 2.0 * n
    assert np.abs(mu - mu_d).max() < 1e-6 and np.abs(s2 - s2_d).max() < 1e-6


def test_points_are_independent_of_each_other():
    """Predicting a set at once equals predicting each point alone (marginal draws)."""
    n = 400
    x, H, W1, f = _setup(n, leaf=32)
    xs = np.array([0.2, 0.21, 0.9])
    xi = rng.normals(3, 4, rng.TAG_PRED, 7, 0)
    all3 = predict.predict(H, W1, f, 1.3, xs, xi)
    for j in range(3):
        one = predict.predict(H, W1, f, 1.3, xs[j:j + 1], xi[j:j + 1])
        for a, b in zip(all3, one):
            # sigma_*^2 is the difference 1 + eta - q: compared on the scale sigma_f^2 (1 + eta)
            assert a[j] == pytest.approx(b[0], rel=1e-13, abs=1e-13 * 1.3)
