"""Function posterior at new inputs (Appendix, 'Function posterior at new inputs', the
equation giving mu_* and sigma_*^2).  TEST INFRASTRUCTURE ONLY: imported by tests/,
the smoke check and the benchmark's CPU baseline, never by the product path.

Given the chain's f, sigma_f^2 and the length-scale's compressed K~_1 = K_1 + eta I, the
prior covariance of f is K = sigma_f^2 K~_1, and a new input x_* has

    mu_*      = k_{*n} K^-1 f            = k1(x_*, X) K~_1^-1 f
    sigma_*^2 = k_** - k_{*n} K^-1 k_{n*} = sigma_f^2 (k1(x_*, x_*) + eta - k1(x_*, X) K~_1^-1 k1(X, x_*)).

The nugget is read as part of the process (jitter), so it enters k_** as it enters the
diagonal of K~_1.  k1(x_*, X) is the exact kernel; K~_1^-1 is the oracle's HODLR solve.
Each new point is drawn from its own marginal N(mu_*, sigma_*^2), as the paper states the
predictive distribution point by point.
"""
import numpy as np

from . import kernels


def predict(H, W1, f, sigf2, xstar, xi):
    """(f_*, mu_*, sigma_*^2) for the new inputs xstar; W1 is the oracle factor of K~_1
    (alpha = 1, beta = 0) on H, xi the standard normals of the draw."""
    xstar = np.asarray(xstar, dtype=np.float64)
    Kx = kernels.k1(H.kind, H.ell, H.x, xstar)          # k1(X, x_*), n x N
    mu = Kx.T @ W1.solve(np.asarray(f, dtype=np.float64))
    quad = np.sum(Kx * W1.solve(Kx), axis=0)             # k_{*n} K~_1^-1 k_{n*}
    s2 = sigf2 * (1.0 + H.nugget - quad)
    fstar = mu + np.sqrt(np.maximum(s2, 0.0)) * np.asarray(xi, dtype=np.float64)
    return fstar, mu, s2
