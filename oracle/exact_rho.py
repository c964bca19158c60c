"""The exact discrete conditional of the length-scale (Section 4.1, the fourth conditional:
Pr(rho = s_h | -) proportional to det(K_h)^(-1/2) exp(-f' K_h^-1 f / 2), uniform prior over
the grid).  TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU baseline, never by the product path.

With K_h = sigma_f^2 K~_1(s_h) = sigma_f^2 W_h W_h' the log-weights are
    lp_h = -1/2 log det K~_1(s_h) - q_h / (2 sigma_f^2),   q_h = |W_h^-1 f|^2
(the -n/2 log sigma_f^2 term is common to every h and dropped).  Every grid point's
HODLR, factor and log-determinant are computed once, before the chain runs, as the
paper suggests.  The draw takes one uniform u and returns the first h whose cumulative
weight sum_{l <= h} exp(lp_l - max lp) exceeds u times the total.
"""
import math

import numpy as np

from . import hodlr, rng, sampler


def log_weights(logdets, qs, sigf2):
    return -0.5 * np.asarray(logdets) - np.asarray(qs) / (2.0 * sigf2)


def inverse_cdf(lp, u):
    """Index drawn from probabilities proportional to exp(lp) with the uniform u."""
    w = np.exp(lp - np.max(lp))
    c = np.cumsum(w)
    t = u * c[-1]
    for h in range(len(c)):
        if c[h] > t:
            return h
    return len(c) - 1


class ExactGridChain(sampler.Chain):
    """The 1-D chain with the length-scale drawn from its exact discrete conditional."""

    def __init__(self, *args, **kw):
        super().__init__(*args, **kw)
        self.Hs = [self._build(h) for h in range(len(self.grid))]
        self.Ws = [hodlr.Factor(H, 1.0, 0.0) for H in self.Hs]
        self.lds = np.array([W.logdet() for W in self.Ws])
        self.H, self.W1, self.logdet1 = self.Hs[self.k], self.Ws[self.k], self.lds[self.k]

    def probs(self, f, sigf2):
        qs = np.array([float(np.sum(W.apply_Winv(f) ** 2)) for W in self.Ws])
        lp = log_weights(self.lds, qs, sigf2)
        p = np.exp(lp - lp.max())
        return p / p.sum(), qs, lp

    def _sigf_and_rho(self, rec):
        t, s, sd = self.it, self.stream, self.seed
        n, f = self.y.size, self.f
        # sigma_f^-2 | -  (as the plain chain)
        u1 = self.W1.apply_Winv(f)
        q = float(u1 @ u1)
        rec["q"] = q
        g, _ = rng.gamma(0.5 * (self.a2 + n), sd, rng.TAG_G_SIGF, t, s)
        self.sigf2 = 1.0 / (g / (0.5 * (self.b2 + q)))
        # rho | -  (exact, over the whole grid)
        _, qs, lp = self.probs(f, self.sigf2)
        u = rng.uniform(sd, rng.TAG_RHO, t, s)
        h = inverse_cdf(lp, u)
        old = self.k
        self.k, self.H, self.W1, self.logdet1 = h, self.Hs[h], self.Ws[h], self.lds[h]
        rec["proposal"], rec["accept"] = h, h != old
        rec["q_all"], rec["lp"], rec["u_rho"] = qs, lp, u
        rec["mh_log_ratio"] = float(lp[h] - (lp.max() + math.log(np.sum(np.exp(lp - lp.max())))))
        rec["tau"], rec["sigf2"], rec["k"] = self.tau, self.sigf2, self.k
