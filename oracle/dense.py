"""O1: exact dense FP64 Gaussian-process quantities (test infrastructure only).

Everything here is the plain definition, O(n^3), for n up to a few thousand.

Model (Eq. 1): y_i = f(x_i) + e_i, e_i ~ N(0, 1/tau); f ~ GP(0, k) with
k = sigma_f^2 k_1 and K = sigma_f^2 K_1.
  * log-likelihood (Eq. 2) with the 1/2 on the log-determinant (the printed equation
    drops it; the Gaussian density needs it):
        l_n = -n/2 log 2 pi - 1/2 log det(K + I/tau) - 1/2 y' (K + I/tau)^-1 y
  * posterior of f (Eq. 3): Sigma_f = K (tau K + I)^-1, mu_f = tau Sigma_f y
  * Gibbs conditionals (Section 4.1): tau | - ~ Ga((a1+n)/2, (b1 + |y-f|^2)/2);
    sigma_f^-2 | - ~ Ga((a2+n)/2, (b2 + f' K_1^-1 f)/2) with Ga(shape, rate);
    Pr(rho = s_h | -) proportional to det(K_{sigma_f,s_h})^-1/2 exp(-f' K^-1 f / 2)
  * KL divergence between two Gaussians (the quantity bounded in Theorem 4.2).
"""
from __future__ import annotations

import math
import numpy as np
import scipy.linalg as sla

from . import kernels


def _chol(A):
    return sla.cholesky(A, lower=True)


def logdet_spd(A) -> float:
    L = _chol(A)
    return 2.0 * float(np.sum(np.log(np.diag(L))))


def solve_spd(A, b):
    return sla.cho_solve((_chol(A), True), b)


def posterior_f(K, tau, y):
    """(mu_f, Sigma_f) of Eq. 3 for covariance K = sigma_f^2 K_1 and precision tau."""
    n = K.shape[0]
    M = tau * K + np.eye(n)
    Sigma_f = np.linalg.solve(M.T, K.T).T        # K M^-1 (M and K commute)
    Sigma_f = 0.5 * (Sigma_f + Sigma_f.T)
    mu_f = tau * Sigma_f @ y
    return mu_f, Sigma_f


def loglik(K, tau, y) -> float:
    """Eq. 2 with the 1/2 on log det."""
    n = K.shape[0]
    S = K + np.eye(n) / tau
    return (-0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet_spd(S)
            - 0.5 * float(y @ solve_spd(S, y)))


def tau_conditional(a1, b1, y, f):
    """(shape, rate) of tau | - (Section 4.1)."""
    r = y - f
    return 0.5 * (a1 + y.size), 0.5 * (b1 + float(r @ r))


def sigf_conditional(a2, b2, K1, f):
    """(shape, rate) of sigma_f^-2 | -; sigma_f^2 f' K^-1 f = f' K_1^-1 f."""
    return 0.5 * (a2 + f.size), 0.5 * (b2 + float(f @ solve_spd(K1, f)))


def rho_conditional(kind, ells, nugget, x, sigf2, f):
    """Normalised Pr(ell = ells[h] | f, sigma_f^2) over a uniform discrete prior."""
    logw = np.empty(len(ells))
    for h, ell in enumerate(ells):
        K = sigf2 * kernels.K1_dense(kind, ell, nugget, x)
        logw[h] = -0.5 * logdet_spd(K) - 0.5 * float(f @ solve_spd(K, f))
    logw -= logw.max()
    w = np.exp(logw)
    return w / w.sum()


def kl_gauss(mu_p, S_p, mu_q, S_q) -> float:
    """KL(P || Q) for P = N(mu_p, S_p), Q = N(mu_q, S_q) (the three terms of the proof
    of Theorem 4.2: log-det ratio, trace, and the mean term)."""
    n = mu_p.size
    Lq = _chol(S_q)
    d = mu_q - mu_p
    t_logdet = logdet_spd(S_q) - logdet_spd(S_p)
    X = sla.cho_solve((Lq, True), S_p)
    t_trace = float(np.trace(X)) - n
    t_mean = float(d @ sla.cho_solve((Lq, True), d))
    return 0.5 * (t_logdet + t_trace + t_mean)


def draw_f_dense(K, tau, y, a, b):
    """Algorithm 1 with exact dense matrices (W = chol K, M = tau K + I):
    Z = sqrt(tau) K a + W b; w = M^-1 Z; r = M^-1 tau y; returns (w + K r, r, K r)."""
    n = K.shape[0]
    W = _chol(K)
    M = tau * K + np.eye(n)
    Z = math.sqrt(tau) * (K @ a) + W @ b
    w = np.linalg.solve(M, Z)
    r = np.linalg.solve(M, tau * y)
    mu = K @ r
    return w + mu, r, mu
