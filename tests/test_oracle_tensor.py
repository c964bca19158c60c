"""Pins of the tensor-product sampler oracle (Section 4.2 with Algorithm 1.h).

Each pin checks the oracle against something other than itself:
  * the conditional mean and covariance of one factor against the Gaussian
    conditional written densely in observation order (no sorting, no HODLR solve,
    the (I + K D)^-1 K form rather than Algorithm 1.h's K (K + D^-1)^-1);
  * d = 1 against Algorithm 1 with tau' = tau beta^2 on y / beta;
  * the beta conditional against numerical quadrature of prior x likelihood;
  * the residual sum of squares against a loop over observations;
  * the length-scale log ratio against scipy's multivariate normal log-density.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import hodlr, kernels, rng, sampler, tensor
from workloads import tensor_surface


def dense_k(x, ell, nugget=1e-6):
    K = np.exp(-np.subtract.outer(x, x) ** 2 / (2.0 * ell * ell))
    return K + nugget * np.eye(x.size)


def make_chain(d=2, n=200, leaf=32, tol=1e-12, seed=3, positive=False):
    x, y = tensor_surface(d, n, seed=seed, positive=positive)
    c = tensor.TensorChain(x, y, kernels.SE, [0.1 + 0.05 * h for h in range(d)], 1e-6, leaf,
                           tol, 50.0, 1.3, seed)
    r = np.random.default_rng(11)
    c.F = 1.0 + 0.6 * r.standard_normal((d, n))
    return x, y, c


def gvec(c, h):
    g = np.empty(c.n)
    for i in range(c.n):
        v = c.beta
        for k in range(c.d):
            if k != h:
                v *= c.F[k, i]
        g[i] = v
    return g


@pytest.mark.parametrize("h", [0, 1, 2])
def test_factor_conditional_mean_dense(h):
    x, y, c = make_chain(d=3)
    g = gvec(c, h)
    K = dense_k(x[h], c.grids[h][c.k[h]])
    D = c.tau * g * g
    # p(f_h | rest) has precision K^-1 + D and mean (K^-1 + D)^-1 tau g y
    m = np.linalg.solve(np.eye(c.n) + K * D[None, :], K @ (c.tau * g * y))
    z = np.zeros(c.n)
    c.update_factor(h, z, z)
    assert np.linalg.norm(c.F[h] - m) <= 1e-8 * np.linalg.norm(m)


def test_factor_conditional_covariance_dense():
    x, y, c = make_chain(d=2, n=80, leaf=16)
    h = 1
    n = c.n
    z = np.zeros(n)
    f0 = c.update_factor(h, z, z)[0]
    Ma = np.empty((n, n))
    Mb = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        Ma[:, j] = c.update_factor(h, e, z)[0] - f0
        Mb[:, j] = c.update_factor(h, z, e)[0] - f0
    cov = Ma @ Ma.T + Mb @ Mb.T
    p = c.perm[h]
    g = gvec(c, h)[p]
    K = dense_k(x[h][p], c.grids[h][c.k[h]])
    D = c.tau * g * g
    ref = np.linalg.solve(np.eye(n) + K * D[None, :], K)
    assert np.linalg.norm(cov - ref) <= 1e-8 * np.linalg.norm(ref)


def test_one_factor_reduces_to_algorithm1():
    x, y = tensor_surface(1, 300, seed=5, positive=True)
    c = tensor.TensorChain(x, y, kernels.SE, [0.08], 1e-6, 32, 1e-12, 30.0, 0.7, 5)
    z = np.zeros(c.n)
    f = c.update_factor(0, z, z)[0]
    p = c.perm[0]
    H = c.H[0]
    tau1 = c.tau * c.beta ** 2
    W1 = hodlr.Factor(H, 1.0, 0.0)
    WM = hodlr.Factor(H, tau1, 1.0)
    _, _, mu = sampler.draw_f(H, W1, WM, 1.0, tau1, y[p] / c.beta, z, z)
    assert np.linalg.norm(f - mu) <= 1e-9 * np.linalg.norm(mu)


def test_beta_conditional_quadrature():
    r = np.random.default_rng(4)
    G = r.normal(size=300)
    y = 0.8 * G + r.normal(0, 0.3, 300)
    tau = 11.0
    mean, sd = tensor.beta_conditional(G, y, tau)
    b = np.linspace(mean - 12 * sd, mean + 12 * sd, 200001)
    lp = stats.norm.logpdf(b, 0.0, tensor.S_BETA)
    # log-likelihood on the grid, accumulated observation by observation
    ll = np.zeros_like(b)
    for i in range(G.size):
        ll += -0.5 * tau * (y[i] - b * G[i]) ** 2
    w = np.exp(lp + ll - np.max(lp + ll))
    qm = np.trapezoid(b * w, b) / np.trapezoid(w, b)
    qv = np.trapezoid((b - qm) ** 2 * w, b) / np.trapezoid(w, b)
    assert abs(qm - mean) <= 1e-7 * sd
    assert abs(math.sqrt(qv) - sd) <= 1e-6 * sd


def test_step_residual_and_tau_draw():
    x, y, c = make_chain(d=3, n=150)
    rec = c.step()
    sse = 0.0
    for i in range(c.n):
        v = c.beta
        for h in range(c.d):
            v *= c.F[h, i]
        sse += (y[i] - v) ** 2
    assert abs(rec["sse"] - sse) <= 1e-12 * sse
    g, _ = rng.gamma(0.5 * (1.0 + c.n), c.seed, rng.TAG_G_TAU, 0, 0)
    assert c.tau == pytest.approx(g / (0.5 * (1.0 + sse)), rel=1e-14)


def test_step_beta_moments_against_quadrature():
    x, y, c = make_chain(d=2, n=120)
    rec = c.step()
    G = c.product()
    tau0 = 50.0  # beta is drawn before tau changes
    b = np.linspace(rec["beta_mean"] - 12 * rec["beta_sd"], rec["beta_mean"] + 12 * rec["beta_sd"],
                    100001)
    ll = stats.norm.logpdf(b, 0.0, tensor.S_BETA)
    for i in range(c.n):
        ll = ll - 0.5 * tau0 * (y[i] - b * G[i]) ** 2
    w = np.exp(ll - ll.max())
    qm = np.trapezoid(b * w, b) / np.trapezoid(w, b)
    assert abs(qm - rec["beta_mean"]) <= 1e-7 * rec["beta_sd"]
    zb = float(rng.normals(1, c.seed, rng.TAG_BETA, 0, 0)[0])
    assert c.beta == pytest.approx(rec["beta_mean"] + rec["beta_sd"] * zb, rel=1e-14)


def test_lengthscale_log_ratio_scipy():
    x, y, c = make_chain(d=2, n=160, tol=1e-12)
    seen = 0
    for _ in range(4):
        Hs = [c.H[h] for h in range(c.d)]
        rec = c.step()
        for h in range(c.d):
            kp = rec["proposal"][h]
            if not 0 <= kp < len(c.grids[h]):
                continue
            fs = c.F[h][c.perm[h]]
            Hp = hodlr.HODLR(c.xs[h], kernels.SE, c.grids[h][kp], 1e-6, 32, 1e-12)
            lp1 = stats.multivariate_normal(np.zeros(c.n), Hp.dense(), allow_singular=False).logpdf(fs)
            lp0 = stats.multivariate_normal(np.zeros(c.n), Hs[h].dense(), allow_singular=False).logpdf(fs)
            assert rec["mh_log_ratio"][h] == pytest.approx(lp1 - lp0, abs=1e-6 * max(1.0, abs(lp0)))
            seen += 1
    assert seen >= 4


def test_chain_deterministic():
    x, y = tensor_surface(2, 100, seed=9)
    runs = []
    for _ in range(2):
        c = tensor.TensorChain(x, y, kernels.SE, (0.1, 0.2), 1e-6, 16, 1e-10, 50.0, 1.0, 9)
        recs = [c.step() for _ in range(3)]
        runs.append((c.F.copy(), [r["tau"] for r in recs], [r["beta"] for r in recs]))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][1] == runs[1][1] and runs[0][2] == runs[1][2]


def test_clamp_keeps_sign_and_floor():
    g = np.array([0.0, 1e-200, -1e-200, -3.0, 2e-150])
    out = tensor.clamp_g(g)
    assert list(out) == [1e-150, 1e-150, -1e-150, -3.0, 2e-150]


# --- additive tensor products (several components) -------------------------------

def make_additive(d=2, n=150, C=2, leaf=32, seed=4):
    x, y = tensor_surface(d, n, seed=seed)
    c = tensor.TensorChain(x, y, kernels.SE, [0.1 + 0.05 * h for h in range(d)], 1e-6, leaf,
                           1e-12, 30.0, 0.9, seed, ncomp=C)
    r = np.random.default_rng(12)
    c.F = 1.0 + 0.5 * r.standard_normal((C * d, n))
    c.betas = [0.9, -0.4][:C]
    return x, y, c


@pytest.mark.parametrize("m", [0, 3])
def test_additive_factor_conditional_dense(m):
    """Factor m = c d + h of a two-component model: the data are the partial residual
    y - beta_c' G_c' written out observation by observation, with
    g_i = beta_c prod_{k != h} f_{c,k}(x_i); mean and covariance against the dense
    conditional."""
    x, y, c = make_additive()
    cc, h = divmod(m, c.d)
    n = c.n
    other = 1 - cc
    r = np.array([y[i] - c.betas[other] * np.prod([c.F[other * c.d + k, i] for k in range(c.d)])
                  for i in range(n)])
    g = np.array([c.betas[cc] * np.prod([c.F[cc * c.d + k, i] for k in range(c.d) if k != h])
                  for i in range(n)])
    K = dense_k(x[h], c.grids[m][c.k[m]])
    D = c.tau * g * g
    mean = np.linalg.solve(np.eye(n) + K * D[None, :], K @ (c.tau * g * r))
    z = np.zeros(n)
    f0 = c.update_factor(m, z, z)[0]
    assert np.linalg.norm(c.F[m] - mean) <= 1e-8 * np.linalg.norm(mean)
    p = c.perm[h]
    # the draw is affine in its normals (a, b): its covariance from the unit responses
    Mb = np.stack([c.update_factor(m, z, np.eye(n)[j])[0] - f0 for j in range(n)], axis=1)
    Ma = np.stack([c.update_factor(m, np.eye(n)[j], z)[0] - f0 for j in range(n)], axis=1)
    cov = Ma @ Ma.T + Mb @ Mb.T
    Ks = dense_k(x[h][p], c.grids[m][c.k[m]])
    Ds = D[p]
    ref = np.linalg.solve(np.eye(n) + Ks * Ds[None, :], Ks)
    assert np.linalg.norm(cov - ref) <= 1e-8 * np.linalg.norm(ref)


def test_additive_with_a_silent_component_is_the_single_product():
    """beta_1 = 0: component 0 sees y itself, so its factor draws and beta_0 equal those
    of the one-component chain with the same state and seed."""
    x, y, c2 = make_additive()
    c2.betas = [0.9, 0.0]
    c1 = tensor.TensorChain(x, y, kernels.SE, [0.1 + 0.05 * h for h in range(2)], 1e-6, 32,
                            1e-12, 30.0, 0.9, 4)
    c1.F = c2.F[:2].copy()
    c1.betas = [0.9]
    for m in range(2):
        D2, y2 = c2.factor_inputs(m)
        D1, y1 = c1.factor_inputs(m)
        np.testing.assert_array_equal(D2, D1)
        np.testing.assert_array_equal(y2, y1)


def test_additive_tau_uses_the_full_residual():
    x, y, c = make_additive()
    rec = c.step()
    fit = np.array([sum(c.betas[cc] * np.prod([c.F[cc * c.d + k, i] for k in range(c.d)])
                        for cc in range(c.C)) for i in range(c.n)])
    assert rec["sse"] == pytest.approx(float(np.sum((y - fit) ** 2)), rel=1e-12)
    assert len(rec["betas"]) == 2 and rec["betas"][0] == c.beta


def test_additive_beta_on_the_partial_residual_quadrature():
    """beta_c | -: prior N(0, s^2) times prod_i N(r_i; beta G_c,i, 1/tau) with the partial
    residual r_i = y_i - beta_c' G_c',i written out per observation, integrated
    numerically."""
    x, y, c = make_additive()
    n = c.n
    G = np.array([np.prod([c.F[c.d + k, i] for k in range(c.d)]) for i in range(n)])
    r = np.array([y[i] - c.betas[0] * np.prod([c.F[k, i] for k in range(c.d)]) for i in range(n)])
    mean, sd = c.beta_moments(1)
    b = np.linspace(mean - 12 * sd, mean + 12 * sd, 20001)
    logp = -0.5 * b ** 2 / tensor.S_BETA ** 2 - 0.5 * c.tau * np.sum(
        (r[None, :] - b[:, None] * G[None, :]) ** 2, axis=1)
    w = np.exp(logp - logp.max())
    m_q = float(np.sum(w * b) / np.sum(w))
    s_q = math.sqrt(float(np.sum(w * (b - m_q) ** 2) / np.sum(w)))
    assert m_q == pytest.approx(mean, rel=1e-6, abs=1e-9)
    assert s_q == pytest.approx(sd, rel=1e-5)
