"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws data.  It holds none of the sampler's arithmetic, so both the
CPU oracle and the HIP path can consume its arrays without sharing any computation.

Workloads (all x sorted ascending, numpy.random.default_rng(seed), draws in the
order written below):

* ``small_1d``   -- n=1000, x ~ U[0,1], y = sin(2 pi x) + 0.5 x^2 + N(0, 0.1^2), seed 0.
  Shaped like the paper's small-n simulation (Section 5.1): a smooth function and
  Gaussian noise at n = 1000.
* ``large_1d``   -- n=2^20, x ~ U[0,1], y = sum_{k=1..5} a_k sin(2 pi f_k x + phi_k)
  + N(0, 0.05^2) with f_k ~ U[1,20], a_k ~ N(0,1), phi_k ~ U[0, 2 pi), seed 1.
  Shaped like the large-n simulation (Section 5.2) but at n = 2^20.
* ``sinusoid_1d(n, seed, noise)`` -- the large_1d generator at any n (parity cases,
  batched chains, served jobs).
"""
from __future__ import annotations

import math
import numpy as np


def small_1d(n: int = 1000, seed: int = 0, noise: float = 0.1):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0.0, 1.0, n))
    y = np.sin(2.0 * math.pi * x) + 0.5 * x * x + rng.normal(0.0, noise, n)
    return x, y


def sinusoid_1d(n: int, seed: int = 1, noise: float = 0.05, ncomp: int = 5):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0.0, 1.0, n))
    freq = rng.uniform(1.0, 20.0, ncomp)
    amp = rng.normal(0.0, 1.0, ncomp)
    phase = rng.uniform(0.0, 2.0 * math.pi, ncomp)
    f = np.zeros(n)
    for k in range(ncomp):
        f += amp[k] * np.sin(2.0 * math.pi * freq[k] * x + phase[k])
    y = f + rng.normal(0.0, noise, n)
    return x, y


def large_1d(n: int = 1 << 20, seed: int = 1):
    return sinusoid_1d(n, seed=seed, noise=0.05)


# Sampler settings of the two single-chain workloads.  Every constant the paper leaves
# open is spelled out here (nugget, priors, grid, start values).
SMALL_1D = dict(n=1000, leaf=64, tol=1e-12, ell0=0.1, tau0=100.0, sigf2_0=1.0,
                nugget=1e-6, iters=50, seed=0)
LARGE_1D = dict(n=1 << 20, leaf=128, tol=1e-10, ell0=0.02, tau0=400.0, sigf2_0=1.0,
                nugget=1e-6, iters=200, seed=1)


def tensor_surface(d: int = 4, n: int = 65536, seed: int = 3, noise: float = 0.1,
                   positive: bool = False):
    """Tensor-product surface (Section 4.2 model, shaped like the d = 2 simulation of
    Section 5.3 with its separable function sin(u) sqrt(u) per coordinate, u = 4 x on
    [0, 4]): x[h, i] ~ U[0,1] in observation order (not sorted),
    y_i = prod_h s(x[h, i]) + N(0, noise^2) with s(x) = sin(4x) sqrt(4x), or
    s(x) = 1.5 + sin(2 pi x) when ``positive`` (a surface without zero crossings)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, (d, n))
    if positive:
        s = 1.5 + np.sin(2.0 * math.pi * x)
    else:
        s = np.sin(4.0 * x) * np.sqrt(4.0 * x)
    y = np.prod(s, axis=0) + rng.normal(0.0, noise, n)
    return x, y


# Tensor-product workload: d = 4 factors, n = 65,536 observations.  Start values:
# every f_h = 1, beta = 1, tau = tau0; grid centre ell0[h] per factor.
TENSOR_4D = dict(d=4, n=65536, leaf=128, tol=1e-10, ell0=(0.05, 0.1333, 0.2167, 0.3),
                 tau0=100.0, beta0=1.0, nugget=1e-6, iters=200, seed=3)


def served_jobs(count: int = 512, seed: int = 5):
    """GP-regression jobs for the serving workload, in arrival order: n log-uniform on
    [1e3, 2e5], sorted x ~ U[0,1], y = 5-sinusoid mixture (the large_1d generator's
    recipe) + N(0, s^2) with s ~ U[0.02, 0.2], grid centre ell0 log-uniform on
    [0.01, 0.3].  Returns a list of dicts (x, y, ell0, noise, tau0 = 1 / noise^2 -- the
    chain's starting noise precision --, seed, n)."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        noise = float(rng.uniform(0.02, 0.2))
        ell0 = float(math.exp(rng.uniform(math.log(0.01), math.log(0.3))))
        jseed = int(rng.integers(1, 2 ** 31))
        x, y = sinusoid_1d(n, seed=jseed, noise=noise)
        jobs.append(dict(x=x, y=y, ell0=ell0, noise=noise, tau0=1.0 / noise ** 2, seed=jseed,
                         n=n))
    return jobs


def new_inputs(count: int = 1024, seed: int = 7):
    """New inputs for predictive draws: uniform on [-0.02, 1.02] (the data's range on
    [0, 1] and a little past both ends), in no particular order."""
    return np.random.default_rng(seed).uniform(-0.02, 1.02, count)


def gridded_1d(n_unique: int = 1 << 14, reps: int = 64, seed: int = 11, noise: float = 0.2):
    """Repeated measurements on a grid: n_unique evenly spaced inputs on (0, 1), each
    observed `reps` times (n = n_unique * reps observations, in shuffled order), y = a
    5-sinusoid signal as in sinusoid_1d plus N(0, noise^2)."""
    g = np.random.default_rng(seed)
    xu = (np.arange(n_unique) + 0.5) / n_unique
    x = np.repeat(xu, reps)
    freq = g.uniform(1.0, 20.0, 5)
    amp = g.normal(0.0, 1.0, 5)
    phase = g.uniform(0.0, 2.0 * math.pi, 5)
    y = sum(amp[k] * np.sin(2.0 * math.pi * freq[k] * x + phase[k]) for k in range(5))
    y = y + noise * g.normal(size=x.size)
    p = g.permutation(x.size)
    return x[p], y[p]
