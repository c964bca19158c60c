"""Pins of the oracle's covariance kernels (oracle/kernels.py) and window radii
(oracle/hodlr.py) against independent definitions.

Section 2.1 names the Matern family.  Its general form, for smoothness nu, is
    k_nu(d) = 2^(1-nu) / Gamma(nu) * (sqrt(2 nu) d / ell)^nu * K_nu(sqrt(2 nu) d / ell),
with K_nu the modified Bessel function of the second kind and k_nu(0) = 1.  The oracle
writes nu = 1/2, 3/2, 5/2 in their closed forms; here they are checked against this
Bessel form evaluated by scipy.special.kv, which shares nothing with the closed forms.
The squared exponential is checked against the normal density of scipy.stats (the
kernel is that density rescaled to 1 at d = 0), and every window radius against a
bracketing root solve of k_1(R) = tol/3 on the Bessel / density form.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
from scipy import optimize, special, stats

from oracle import hodlr, kernels

NU = {kernels.EXP: 0.5, kernels.MATERN32: 1.5, kernels.MATERN52: 2.5}


def matern_bessel(nu: float, ell: float, d: np.ndarray) -> np.ndarray:
    """The general Matern correlation at distances d >= 0 (Bessel form)."""
    d = np.abs(np.asarray(d, dtype=np.float64))
    z = math.sqrt(2.0 * nu) * d / ell
    out = np.ones_like(z)
    pos = z > 0
    zp = z[pos]
    # log form keeps z^nu K_nu(z) finite where K_nu underflows separately
    lg = ((1.0 - nu) * math.log(2.0) - special.gammaln(nu) + nu * np.log(zp)
          + np.log(special.kve(nu, zp)) - zp)
    out[pos] = np.exp(lg)
    return out


def se_density(ell: float, d: np.ndarray) -> np.ndarray:
    """exp(-d^2 / (2 ell^2)) as the N(0, ell^2) density divided by its peak."""
    d = np.asarray(d, dtype=np.float64)
    return stats.norm.pdf(d, scale=ell) / stats.norm.pdf(0.0, scale=ell)


def reference(kind: int, ell: float, d: np.ndarray) -> np.ndarray:
    if kind == kernels.SE:
        return se_density(ell, d)
    return matern_bessel(NU[kind], ell, d)


DISTS = np.concatenate([[0.0], np.logspace(-8, 1.2, 400)])


def _max_rel(a, b):
    m = np.abs(b) > 1e-280
    return float(np.max(np.abs(a[m] - b[m]) / np.abs(b[m])))


@pytest.mark.parametrize("kind", [kernels.SE, kernels.EXP, kernels.MATERN32, kernels.MATERN52])
@pytest.mark.parametrize("ell", [0.003, 0.02, 0.1, 0.3, 2.0])
def test_kernel_matches_independent_definition(kind, ell):
    """k_1 on both sides of zero equals the Bessel-form Matern (nu = 1/2, 3/2, 5/2) or the
    normal density (SE) to a few ulps relative, wherever the value is representable."""
    got = kernels.k1(kind, ell, DISTS, [0.0])[:, 0]
    got_neg = kernels.k1(kind, ell, [0.0], DISTS)[0, :]
    ref = reference(kind, ell, DISTS)
    assert got[0] == 1.0
    assert _max_rel(got, ref) < 2e-13
    assert np.array_equal(got, got_neg)  # symmetric in (x, x')


@pytest.mark.parametrize("kind,mutant", [
    (kernels.MATERN32, lambda d, ell: (1 + 3 * d / ell) * np.exp(-3 * d / ell)),
    (kernels.MATERN32, lambda d, ell: (1 + math.sqrt(3) * d / ell) * np.exp(-d / ell)),
    (kernels.MATERN52, lambda d, ell: (1 + math.sqrt(5) * d / ell) * np.exp(-math.sqrt(5) * d / ell)),
    (kernels.MATERN52, lambda d, ell: (1 + math.sqrt(5) * d / ell + 5 * d * d / ell ** 2)
     * np.exp(-math.sqrt(5) * d / ell)),
    (kernels.SE, lambda d, ell: np.exp(-d * d / (ell * ell))),
])
def test_pin_rejects_plausible_slips(kind, mutant):
    """The comparison above is sharp enough to reject a slipped constant or a dropped
    term (each mutant misses the independent form by far more than the 2e-13 bar)."""
    ell = 0.1
    ref = reference(kind, ell, DISTS)
    assert _max_rel(mutant(DISTS, ell), ref) > 1e-3


@pytest.mark.parametrize("kind", [kernels.SE, kernels.EXP, kernels.MATERN32, kernels.MATERN52])
@pytest.mark.parametrize("ell,tol", [(0.1, 1e-10), (0.02, 1e-12), (0.3, 1e-6), (1e-3, 1e-14)])
def test_window_radius_is_the_tol_over_three_crossing(kind, ell, tol):
    """The window radius is the distance where the independent form of k_1 falls to
    tol/3 (Brent's method on a bracket), to 1e-10 relative."""
    target = tol / 3.0

    def g(r):
        return math.log(reference(kind, ell, np.array([r]))[0]) - math.log(target)

    hi = ell
    while g(hi) > 0:
        hi *= 2.0
    R_ref = optimize.brentq(g, 0.0 if g(1e-300) > 0 else 1e-300, hi, xtol=1e-300, rtol=1e-14)
    assert hodlr.window_radius(kind, ell, tol) == pytest.approx(R_ref, rel=1e-10)


@pytest.mark.parametrize("kind,nu_poly", [
    (kernels.MATERN32, lambda u, p: 1 + u - p),
    (kernels.MATERN52, lambda u, p: 1 + u + u * u / 3 - p * (1 + 2 * u / 3) + p * (p - 1) / 3),
])
def test_matern_derivative_formula(kind, nu_poly):
    """The p-th derivative in u that interp_bound relies on, (-1)^p e^-u times the
    stated polynomial, against finite differences of the Bessel form (p = 1..4)."""
    nu = NU[kind]
    h = 1e-2
    for u0 in [0.7, 2.0, 5.0]:
        f = lambda u: matern_bessel(nu, math.sqrt(2 * nu), np.array([u]))[0]  # ell = sqrt(2 nu): z = u
        for p in range(1, 5):
            # p-th central difference (truncation O(h^2), rounding ~ 2^p u / h^p)
            fd = sum((-1) ** k * math.comb(p, k) * f(u0 + (p / 2 - k) * h) for k in range(p + 1)) / h ** p
            exact = (-1) ** p * math.exp(-u0) * nu_poly(u0, p)
            assert fd == pytest.approx(exact, rel=2e-3, abs=1e-3 * math.exp(-u0) * (1 + u0) ** 2)
