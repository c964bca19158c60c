"""Algorithm 1, Algorithm 1.h and the FIFA-GP Gibbs sweep on the CPU (test
infrastructure only).

Algorithm 1 (Section 4.1.1), with K~ = sigma_f^2 K~_1, W = sigma_f W_1 (K~_1 = W_1 W_1')
and M~ = tau K~ + I built from K~ (the Appendix proof notes this satisfies both
tolerance bounds):
    a, b ~ N(0, I);  Z = sqrt(tau) K~ a + W b;  solve M~ w = Z;  solve M~ r = tau y;
    return f = w + K~ r.
r is also Sigma~^-1 y with Sigma~ = K~ + I/tau, and mu~ = K~ r is the approximate
posterior mean (Lemma 4.1).

Gibbs sweep (Section 4.1, Eqs. for f, tau, sigma_f^-2, rho in that order):
  f     | -  by Algorithm 1 on the current (tau, sigma_f^2, ell);
  tau   | -  ~ Ga((a1+n)/2, (b1 + |y-f|^2)/2)           (shape, rate);
  sf^-2 | -  ~ Ga((a2+n)/2, (b2 + f' K~_1^-1 f)/2);
  rho   | -  the discrete conditional over the length-scale grid, sampled with the
             Metropolis step the paper suggests in its place: propose the grid
             neighbour k+-1 with probability 1/2 each, off-grid proposals rejected,
             accept with probability min(1, exp(D)),
             D = -1/2 (log|K~_1'| - log|K~_1|) - (q' - q) / (2 sigma_f^2),
             q = f' K~_1^-1 f = |W_1^-1 f|^2.
Readings where the paper is silent: priors a1 = b1 = a2 = b2 = 1; grid
ell_k = ell_0 10^((k-50)/50), k = 0..99 (a 100-point grid as in Section 5.2), start
at k = 50; the tolerance is an absolute max-norm bound on the unit-amplitude K_1,
fixed per grid point (K~ is rebuilt per length-scale, as the paper precomputes it).
"""
from __future__ import annotations

import math
import numpy as np

from . import hodlr, rng

A1 = B1 = A2 = B2 = 1.0
GRID_SIZE = 100
GRID_CENTER = 50


def ell_grid(ell0, size=GRID_SIZE, center=GRID_CENTER):
    """The length-scale grid ell0 10^((g - center) / 50), g = 0 .. size - 1 (Section 4.1's
    discrete grid).  Each point is evaluated by the C library's pow, one point at a time,
    as the HIP library evaluates it: numpy's vectorised power can round a point
    differently by one unit, and both sides must run at the same length-scales."""
    return np.array([ell0 * math.pow(10.0, (g - center) / 50.0) for g in range(size)])


def draw_f(H: hodlr.HODLR, W1: hodlr.Factor, WM: hodlr.Factor, sigf2, tau, y, a, b):
    """Algorithm 1.  W1: factor of K~_1; WM: factor of tau sigma_f^2 K~_1 + I.
    Returns (f, r, mu) with r = M~^-1 tau y = Sigma~^-1 y and mu = K~ r."""
    Z = math.sqrt(tau) * sigf2 * H.matvec(a) + math.sqrt(sigf2) * W1.apply_W(b)
    w = WM.solve(Z)
    r = WM.solve(tau * y)
    mu = sigf2 * H.matvec(r)
    return w + mu, r, mu


def draw_f_hetero(H: hodlr.HODLR, WK: hodlr.Factor, WP: hodlr.Factor, D, y, a_std, b):
    """Algorithm 1.h (Appendix, heteroskedastic noise) for unit-variance K~ = K~_1,
    precisions D (diagonal), P~ = K~ + D^-1 with factor WP:
      a ~ N(0, D) (a = sqrt(D) a_std), b ~ N(0, I); Z = K~ a + W b; Z* = P~^-1 Z;
      Z** = D^-1 Z*; R = K~ P~^-1 y; return R + Z**."""
    a = np.sqrt(D) * a_std
    Z = H.matvec(a) + WK.apply_W(b)
    Zs = WP.solve(Z)
    Zss = Zs / D
    Rv = H.matvec(WP.solve(y))
    return Rv + Zss, Rv


class Chain:
    """State of one 1-D chain plus its cached (K~_1, W_1, log|K~_1|) for the current
    grid point."""

    def __init__(self, x, y, kind, ell0, nugget, leaf, tol, tau0, sigf2_0, seed,
                 stream=0, grid=None, priors=(A1, B1, A2, B2)):
        self.x, self.y = np.asarray(x, float), np.asarray(y, float)
        self.kind, self.nugget, self.leaf, self.tol = kind, nugget, leaf, tol
        self.grid = ell_grid(ell0) if grid is None else np.asarray(grid, float)
        self.k = GRID_CENTER if grid is None else len(self.grid) // 2
        self.tau, self.sigf2 = float(tau0), float(sigf2_0)
        self.seed, self.stream, self.it = seed, stream, 0
        self.a1, self.b1, self.a2, self.b2 = priors
        self.f = np.zeros_like(self.y)
        self.H = self._build(self.k)
        self.W1 = hodlr.Factor(self.H, 1.0, 0.0)
        self.logdet1 = self.W1.logdet()
        self.last = {}

    def _build(self, k):
        return hodlr.HODLR(self.x, self.kind, self.grid[k], self.nugget, self.leaf, self.tol)

    def step(self):
        rec = {}
        self._f_and_tau(rec)
        self._sigf_and_rho(rec)
        self.it += 1
        self.last = rec
        return rec

    def _f_and_tau(self, rec):
        n, y, t, s, sd = self.y.size, self.y, self.it, self.stream, self.seed
        # f | -
        WM = hodlr.Factor(self.H, self.tau * self.sigf2, 1.0)
        a = rng.normals(n, sd, rng.TAG_A, t, s)
        b = rng.normals(n, sd, rng.TAG_B, t, s)
        f, r, mu = draw_f(self.H, self.W1, WM, self.sigf2, self.tau, y, a, b)
        logdet_M = WM.logdet()
        rec["logdet_sigma"] = logdet_M - n * math.log(self.tau)
        rec["yr"] = float(y @ r)
        rec["loglik"] = (-0.5 * n * math.log(2.0 * math.pi) - 0.5 * rec["logdet_sigma"]
                         - 0.5 * rec["yr"])
        rec["r"], rec["mu"] = r, mu
        self.f = f
        # tau | -
        e = y - f
        rec["sse"] = float(e @ e)
        g, _ = rng.gamma(0.5 * (self.a1 + n), sd, rng.TAG_G_TAU, t, s)
        self.tau = g / (0.5 * (self.b1 + rec["sse"]))

    def _sigf_and_rho(self, rec):
        n, t, s, sd = self.y.size, self.it, self.stream, self.seed
        f = self.f
        # sigma_f^-2 | -
        u1 = self.W1.apply_Winv(f)
        q = float(u1 @ u1)
        rec["q"] = q
        g, _ = rng.gamma(0.5 * (self.a2 + n), sd, rng.TAG_G_SIGF, t, s)
        self.sigf2 = 1.0 / (g / (0.5 * (self.b2 + q)))
        # rho | -  (Metropolis on the grid)
        up = rng.uniform(sd, rng.TAG_PROP, t, s)
        kp = self.k + (1 if up < 0.5 else -1)
        rec["proposal"], rec["accept"] = kp, False
        if 0 <= kp < len(self.grid):
            Hp = self._build(kp)
            Wp = hodlr.Factor(Hp, 1.0, 0.0)
            ldp = Wp.logdet()
            up1 = Wp.apply_Winv(f)
            qp = float(up1 @ up1)
            D = -0.5 * (ldp - self.logdet1) - (qp - q) / (2.0 * self.sigf2)
            ua = rng.uniform(sd, rng.TAG_ACC, t, s)
            rec["logdet1_prop"], rec["q_prop"], rec["mh_log_ratio"] = ldp, qp, D
            if math.log(ua) < D:
                self.k, self.H, self.W1, self.logdet1 = kp, Hp, Wp, ldp
                rec["accept"] = True
        rec["tau"], rec["sigf2"], rec["k"] = self.tau, self.sigf2, self.k
