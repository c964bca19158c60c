"""Non-unique inputs (Appendix, 'Non-unique input points').  TEST INFRASTRUCTURE ONLY:
imported by tests/, the smoke check and the benchmark's CPU baseline, never by the
product path.

n observations y_h at inputs x_h with only U < n distinct values x^u_i.  With
Q_i = {h : x_h = x^u_i}, the GP runs on the U unique inputs with the averages
ybar_i = (1/|Q_i|) sum_{h in Q_i} y_h.  Each average of |Q_i| independent observations of
precision tau has precision |Q_i| tau; the paper prints |Q_i|^2 tau for the diagonal, which
is read here as |Q_i| tau (the sufficiency pin in the tests decides between the two).

Given f on the unique inputs, the full-data residual sum of squares splits into
    sum_h (y_h - f_u(h))^2 = sum_i |Q_i| (ybar_i - f_i)^2 + S_w,
    S_w = sum_i sum_{h in Q_i} (y_h - ybar_i)^2 (constant),
so tau | - keeps its full-data conditional Ga((a1 + n)/2, (b1 + that sum)/2).
f | - is the heteroskedastic draw (Algorithm 1.h) with noise precisions |Q_i| tau; with
g = f / sigma_f it has the unit-variance prior K~_1 and precisions sigma_f^2 |Q_i| tau on
ybar / sigma_f, so Algorithm 1.h applies as written and f = sigma_f g.
"""
import math

import numpy as np

from . import hodlr, rng, sampler


def collapse(x, y):
    """(unique inputs ascending, counts |Q_i|, averages ybar_i, within-group S_w)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xu, inv, cnt = np.unique(x, return_inverse=True, return_counts=True)
    ybar = np.bincount(inv, weights=y) / cnt
    within = float(np.sum((y - ybar[inv]) ** 2))
    return xu, cnt.astype(np.float64), ybar, within


class CollapsedChain(sampler.Chain):
    """The 1-D chain on the collapsed data; sigma_f^-2 and the length-scale steps are the
    plain chain's on the U unique inputs."""

    def __init__(self, x, y, kind, ell0, nugget, leaf, tol, tau0, sigf2_0, seed, stream=0,
                 grid=None, priors=(sampler.A1, sampler.B1, sampler.A2, sampler.B2)):
        xu, w, ybar, within = collapse(x, y)
        super().__init__(xu, ybar, kind, ell0, nugget, leaf, tol, tau0, sigf2_0, seed, stream,
                         grid, priors)
        self.w, self.within, self.n_obs = w, within, int(np.asarray(y).size)

    def _f_and_tau(self, rec):
        U, t, s, sd = self.y.size, self.it, self.stream, self.seed
        sigf = math.sqrt(self.sigf2)
        # f | -  (Algorithm 1.h on g = f / sigma_f)
        D = self.tau * self.sigf2 * self.w                  # precisions of ybar / sigma_f
        WP = hodlr.Factor(self.H, 1.0, 0.0, 1.0 / D)        # K~_1 + D^-1
        a = rng.normals(U, sd, rng.TAG_A, t, s)
        b = rng.normals(U, sd, rng.TAG_B, t, s)
        ys = self.y / sigf
        g, R = sampler.draw_f_hetero(self.H, self.W1, WP, D, ys, a, b)
        self.f = sigf * g
        # log-likelihood of the averages: ybar ~ N(0, sigma_f^2 (K~_1 + D^-1))
        rs = WP.solve(ys)
        rec["logdet_sigma"] = WP.logdet() + U * math.log(self.sigf2)
        rec["yr"] = float(ys @ rs)
        rec["loglik"] = (-0.5 * U * math.log(2.0 * math.pi) - 0.5 * rec["logdet_sigma"]
                         - 0.5 * rec["yr"])
        rec["r"], rec["mu"] = rs / sigf, sigf * R
        # tau | -  (full-data residual sum of squares)
        e = self.y - self.f
        rec["sse"] = float(np.sum(self.w * e * e)) + self.within
        gt, _ = rng.gamma(0.5 * (self.a1 + self.n_obs), sd, rng.TAG_G_TAU, t, s)
        self.tau = gt / (0.5 * (self.b1 + rec["sse"]))
