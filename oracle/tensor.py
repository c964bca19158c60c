"""Tensor-product surface sampler on the CPU (test infrastructure only).

Model (Section 4.2): y_i = beta prod_h f_h(x[h, i]) + e_i, e_i ~ N(0, 1/tau), f_h a
unit-variance GP with a squared-exponential kernel of length-scale ell_h (mean zero).

Given every other factor, y_i / g_i with g_i = beta prod_{k != h} f_k(x[k, i]) is a
noisy observation of f_h(x[h, i]) with precision D_i = tau g_i^2 (Section 4.2), so f_h
is drawn by Algorithm 1.h (Appendix, heteroskedastic noise) on the inputs of dimension
h sorted ascending.

One sweep, in this order:
  f_1, ..., f_d  by Algorithm 1.h, one after the other (each sees the new values of
                 the factors drawn before it);
  beta | -       Gaussian: prior N(0, s_beta^2), precision tau G'G + s_beta^-2,
                 mean tau G'y / precision, G_i = prod_h f_h(x[h, i]);
  tau  | -       Ga((a1 + n)/2, (b1 + |y - beta G|^2)/2)  (shape, rate);
  ell_h | -      for h = 1..d, the grid Metropolis step of the 1-D sampler with the
                 unit-variance prior: D = -1/2 (log|K~_h'| - log|K~_h|) - (q' - q)/2,
                 q = f_h' K~_h^-1 f_h.
Readings where the paper is silent: zero prior mean; beta ~ N(0, 10^2); a systematic
scan h = 1..d; start values f_h = 1, beta = beta0; g^2 is floored at 1e-300 (g is
replaced by +-1e-150, sign kept, zero counted as positive) so that D^-1 stays finite.
Random numbers: factor h draws a, b, its proposal and its acceptance uniform on the
1-D sampler's tags plus 16 (h + 1); beta uses its own tag.

Additive tensor products (Sections 4.2 and 5.2: y_i = sum_c beta_c prod_h f_{c,h}(x[h, i])
+ e_i).  Component c sees the partial residual r_c = y - sum_{c' != c} beta_c' G_c' in place
of y; its factors f_{c,1..d} are drawn as above from r_c, then beta_c from r_c; tau follows
the full residual; then every factor's length-scale.  Factor m = c d + h; its draws use
the tags of factor m, and beta_c uses tag 7 for c = 0 and 7 + 16 (9 + c) otherwise.  With
one component this is the sweep above, unchanged.
"""
from __future__ import annotations

import math
import numpy as np

from . import hodlr, rng
from .sampler import draw_f_hetero, ell_grid, GRID_CENTER

A1 = B1 = 1.0
S_BETA = 10.0
G_FLOOR = 1e-150


def factor_tag(tag, h):
    return tag + rng.TAG_FACTOR_STRIDE * (h + 1)


def beta_tag(c):
    return rng.TAG_BETA if c == 0 else rng.TAG_BETA + rng.TAG_FACTOR_STRIDE * (9 + c)


def clamp_g(g):
    """g with |g| floored at 1e-150 (sign kept, zero treated as positive)."""
    g = np.asarray(g, dtype=np.float64)
    small = np.abs(g) < G_FLOOR
    return np.where(small, np.where(g < 0.0, -G_FLOOR, G_FLOOR), g)


def beta_conditional(G, y, tau, s_beta=S_BETA):
    """Mean and standard deviation of beta | - (Gaussian prior, Gaussian likelihood)."""
    prec = tau * float(G @ G) + 1.0 / (s_beta * s_beta)
    return tau * float(G @ y) / prec, 1.0 / math.sqrt(prec)


class TensorChain:
    """State of one tensor-product chain: factors F[h] in observation order, and per
    dimension the sorting permutation, the cached (K~_h, W_h, log|K~_h|) and the grid
    index."""

    def __init__(self, x, y, kind, ell0, nugget, leaf, tol, tau0, beta0, seed, stream=0,
                 grids=None, priors=(A1, B1), s_beta=S_BETA, ncomp=1):
        self.x = np.asarray(x, dtype=np.float64)
        self.y = np.asarray(y, dtype=np.float64)
        self.d, self.n = self.x.shape
        self.C = int(ncomp)
        self.nf = self.C * self.d                       # factor m = c d + h
        self.kind, self.nugget, self.leaf, self.tol = kind, nugget, leaf, tol
        self.tau = float(tau0)
        self.betas = [float(beta0)] * self.C
        self.seed, self.stream, self.it = seed, stream, 0
        self.a1, self.b1 = priors
        self.s_beta = s_beta
        self.perm = [np.argsort(self.x[h], kind="stable") for h in range(self.d)]
        self.xs = [self.x[h][self.perm[h]] for h in range(self.d)]
        ell0 = list(ell0)
        if len(ell0) == self.d:
            ell0 = ell0 * self.C
        if grids is None:
            self.grids = [ell_grid(e) for e in ell0]
            self.k = [GRID_CENTER] * self.nf
        else:
            grids = list(grids)
            if len(grids) == self.d:
                grids = grids * self.C
            self.grids = [np.asarray(g, dtype=np.float64) for g in grids]
            self.k = [len(g) // 2 for g in self.grids]
        self.F = np.ones((self.nf, self.n))
        self.H, self.W, self.logdet = [], [], []
        for h in range(self.nf):
            H = self._build(h, self.k[h])
            W = hodlr.Factor(H, 1.0, 0.0)
            self.H.append(H)
            self.W.append(W)
            self.logdet.append(W.logdet())
        self.last = {}

    @property
    def beta(self):
        return self.betas[0]

    def _build(self, m, k):
        return hodlr.HODLR(self.xs[m % self.d], self.kind, self.grids[m][k], self.nugget,
                           self.leaf, self.tol)

    def partial_residual(self, c):
        """y - sum_{c' != c} beta_c' G_c' (observation order)."""
        r = self.y.copy()
        for cc in range(self.C):
            if cc != c:
                r = r - self.betas[cc] * self.product(cc)
        return r

    def factor_inputs(self, m):
        """(D, y~) of factor m = c d + h in the sorted order of dimension h."""
        c, h = divmod(m, self.d)
        g = np.full(self.n, self.betas[c])
        for k in range(self.d):
            if k != h:
                g = g * self.F[c * self.d + k]
        gs = clamp_g(g[self.perm[h]])
        D = self.tau * gs * gs
        return D, self.partial_residual(c)[self.perm[h]] / gs

    def update_factor(self, m, a_std, b):
        """Draw f_m by Algorithm 1.h from the given standard normals (sorted order)."""
        h = m % self.d
        D, yt = self.factor_inputs(m)
        WP = hodlr.Factor(self.H[m], 1.0, 0.0, 1.0 / D)
        f, R = draw_f_hetero(self.H[m], self.W[m], WP, D, yt, a_std, b)
        self.F[m][self.perm[h]] = f
        return f, R, WP

    def product(self, c=0):
        G = np.ones(self.n)
        for h in range(self.d):
            G = G * self.F[c * self.d + h]
        return G

    def beta_moments(self, c):
        """Mean and standard deviation of beta_c | - (data: the partial residual r_c)."""
        return beta_conditional(self.product(c), self.partial_residual(c), self.tau, self.s_beta)

    def fitted(self):
        return sum(self.betas[c] * self.product(c) for c in range(self.C))

    def step(self):
        n, t, s, sd = self.n, self.it, self.stream, self.seed
        rec = {"beta_means": [], "beta_sds": []}
        for c in range(self.C):
            for h in range(self.d):
                m = c * self.d + h
                a = rng.normals(n, sd, factor_tag(rng.TAG_A, m), t, s)
                b = rng.normals(n, sd, factor_tag(rng.TAG_B, m), t, s)
                self.update_factor(m, a, b)
            # beta_c | -  (on the partial residual)
            mean, sdv = self.beta_moments(c)
            z = float(rng.normals(1, sd, beta_tag(c), t, s)[0])
            self.betas[c] = mean + sdv * z
            rec["beta_means"].append(mean)
            rec["beta_sds"].append(sdv)
        rec["beta_mean"], rec["beta_sd"] = rec["beta_means"][0], rec["beta_sds"][0]
        # tau | -
        e = self.y - self.fitted()
        rec["sse"] = float(e @ e)
        g, _ = rng.gamma(0.5 * (self.a1 + n), sd, rng.TAG_G_TAU, t, s)
        self.tau = g / (0.5 * (self.b1 + rec["sse"]))
        # ell_h | -  (grid Metropolis per dimension)
        rec["q"], rec["proposal"], rec["accept"], rec["mh_log_ratio"] = [], [], [], []
        rec["logdet_prop"], rec["q_prop"] = [], []
        for h in range(self.nf):
            fs = self.F[h][self.perm[h % self.d]]
            u = self.W[h].apply_Winv(fs)
            q = float(u @ u)
            up = rng.uniform(sd, factor_tag(rng.TAG_PROP, h), t, s)
            kp = self.k[h] + (1 if up < 0.5 else -1)
            acc, D, ldp, qp = False, 0.0, 0.0, 0.0
            if 0 <= kp < len(self.grids[h]):
                Hp = self._build(h, kp)
                Wp = hodlr.Factor(Hp, 1.0, 0.0)
                ldp = Wp.logdet()
                up1 = Wp.apply_Winv(fs)
                qp = float(up1 @ up1)
                D = -0.5 * (ldp - self.logdet[h]) - 0.5 * (qp - q)
                ua = rng.uniform(sd, factor_tag(rng.TAG_ACC, h), t, s)
                if math.log(ua) < D:
                    self.k[h], self.H[h], self.W[h], self.logdet[h] = kp, Hp, Wp, ldp
                    acc = True
            rec["q"].append(q)
            rec["proposal"].append(kp)
            rec["accept"].append(acc)
            rec["mh_log_ratio"].append(D)
            rec["logdet_prop"].append(ldp)
            rec["q_prop"].append(qp)
        rec["tau"], rec["beta"], rec["k"] = self.tau, self.betas[0], list(self.k)
        rec["betas"] = list(self.betas)
        rec["logdet"] = list(self.logdet)
        self.it += 1
        self.last = rec
        return rec
