"""The HIP path against the exact dense GP (O1) at n = 8000: the large workload's
generator (seed 1, sorted U[0,1] inputs, 5-sinusoid y), squared exponential with
ell = 0.02, nugget 1e-6, leaf 128, tau = 400, sigma_f^2 = 1 -- the dense cross-check
size of the large 1-D workload.

Theorem 4.2 bounds the distance between the exact posterior of f and the one built on
the HODLR approximation by the approximation's error.  With the GPU's K~ made dense
(hodlr_matvec on unit vectors) and dK = K~ - K against the exact kernel matrix:
  * max |dK| <= tol (the bound the construction guarantees);
  * the posterior mean mu~ = K~ r, M~ r = tau y (Algorithm 1's solve and product),
    against Eq. 3's mean: with Sigma = K + I/tau, mu = y - Sigma^-1 y / tau, so exactly
    mu~ - mu = tau^-1 Sigma~^-1 dK Sigma^-1 y
             = tau^-1 Sigma^-1 dK Sigma^-1 y - tau^-1 Sigma~^-1 dK Sigma^-1 dK Sigma^-1 y,
    and as |tau^-1 Sigma~^-1| <= 1 and |Sigma^-1| <= tau the second term is at most
    tau |dK|_2 |dK Sigma^-1 y|: the GPU's mean must equal the exact mean plus the
    first-order term to within that, plus 1e-9 |mu| of rounding;
  * log|Sigma~| - log|Sigma| = log det(I + E), E = Sigma^-1/2 dK Sigma^-1/2, which
    differs from tr(Sigma^-1 dK) by at most |E|_F^2 / (2 (1 - |E|_2)) <=
    (tau |dK|_F)^2 / (2 (1 - tau |dK|_2)), plus 1e-9 |log|Sigma|| of rounding;
  * KL(P || Q) between the exact posterior P and the GPU's Q falls with tol (about as
    tol^2: by more than 100x per factor 100) and at tol = 1e-8 equals, within 10%, the KL
    of the oracle's own HODLR (the same approximation).
"""
import math

import numpy as np
import pytest

from oracle import dense, hodlr as oh, kernels
from workloads import large_1d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N, ELL, NUG, LEAF, TAU = 8000, 0.02, 1e-6, 128, 400.0


@pytest.fixture(scope="module")
def exact():
    x, y = large_1d(N, seed=1)
    K = kernels.K1_dense(kernels.SE, ELL, NUG, x)
    S = K + np.eye(N) / TAU
    Sinv = np.linalg.inv(S)
    Sinv = 0.5 * (Sinv + Sinv.T)
    Siy = Sinv @ y
    mu = y - Siy / TAU
    mu_p, S_p = dense.posterior_f(K, TAU, y)
    return dict(x=x, y=y, K=K, Sinv=Sinv, Siy=Siy, mu=mu, ld=dense.logdet_spd(S), mu_p=mu_p,
                S_p=S_p, kl={})


def _gpu(x, y, tol):
    """K~_1 (made dense), mu~ = K~ r with M~ r = tau y, and log|Sigma~| = log|M~| - n log
    tau, from the HIP path."""
    import paper_2006_06537_amd as fg
    dev = torch.device("cuda:0")
    K1 = fg.Hodlr(torch.tensor(x, device=dev), ELL, nugget=NUG, leaf=LEAF, tol=tol)
    WM = fg.Factor(K1, TAU, 1.0)
    assert WM.status() == 0
    r = WM.solve(TAU * torch.tensor(y, device=dev))
    mu = K1.matvec(r).cpu().numpy()
    ld = float(WM.logdet().cpu()[0]) - N * math.log(TAU)
    Kd = np.empty((N, N))
    for c0 in range(0, N, 4):
        nb = min(4, N - c0)
        E = torch.zeros((nb, N), dtype=torch.float64, device=dev)
        E[torch.arange(nb, device=dev), torch.arange(c0, c0 + nb, device=dev)] = 1.0
        Kd[:, c0:c0 + nb] = K1.matvec(E).cpu().numpy().T
    return Kd, mu, ld


@pytest.mark.parametrize("tol", [1e-8, 1e-10])
def test_posterior_against_exact_gp(exact, tol):
    Kd, mu, ld = _gpu(exact["x"], exact["y"], tol)
    dK = Kd - exact["K"]
    assert np.abs(dK).max() <= tol
    n2, nF = np.linalg.norm(dK, 2), np.linalg.norm(dK)
    # the mean: exact value plus the first-order term, within the second-order remainder
    first = exact["Sinv"] @ (dK @ exact["Siy"]) / TAU
    rem = TAU * n2 * np.linalg.norm(dK @ exact["Siy"]) + 1e-9 * np.linalg.norm(exact["mu"])
    e_mu = np.linalg.norm(mu - exact["mu"] - first)
    # the log-determinant: exact value plus tr(Sigma^-1 dK)
    tr1 = float(np.sum(exact["Sinv"] * dK))
    t2 = TAU * n2
    rem_ld = (TAU * nF) ** 2 / (2.0 * (1.0 - t2)) + 1e-9 * abs(exact["ld"])
    e_ld = abs(ld - exact["ld"] - tr1)
    print(f"tol {tol:g}: |mu~ - mu| {np.linalg.norm(mu - exact['mu']):.2e}, after the "
          f"first-order term {e_mu:.2e} (bound {rem:.2e}); log-det difference "
          f"{abs(ld - exact['ld']):.2e}, after tr(Sigma^-1 dK) {e_ld:.2e} (bound {rem_ld:.2e})")
    assert e_mu <= rem
    assert t2 < 1.0 and e_ld <= rem_ld
    mu_q, S_q = dense.posterior_f(0.5 * (Kd + Kd.T), TAU, exact["y"])
    exact["kl"][tol] = dense.kl_gauss(exact["mu_p"], exact["S_p"], mu_q, S_q)
    print(f"tol {tol:g}: KL(P || Q) {exact['kl'][tol]:.3e}")


def test_kl_falls_with_tol_and_matches_the_oracles_hodlr(exact):
    kl = exact["kl"]
    if set(kl) != {1e-8, 1e-10}:
        pytest.skip("needs test_posterior_against_exact_gp first")
    assert kl[1e-8] > 100.0 * kl[1e-10] > 0.0
    Ko = oh.HODLR(exact["x"], kernels.SE, ELL, NUG, LEAF, 1e-8).dense()
    mu_o, S_o = dense.posterior_f(Ko, TAU, exact["y"])
    kl_o = dense.kl_gauss(exact["mu_p"], exact["S_p"], mu_o, S_o)
    print(f"KL at tol 1e-8: GPU {kl[1e-8]:.4e}, oracle HODLR {kl_o:.4e}")
    assert abs(kl[1e-8] - kl_o) <= 0.1 * kl_o
