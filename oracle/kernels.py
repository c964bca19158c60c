"""Unit-amplitude covariance kernels k_1 (test infrastructure only).

Squared exponential (Section 2.1 and Section 4.1): the paper writes it both as
sigma_f^2 exp(-(x-x')^2 / (2 rho^2)) and as sigma_f^2 exp(-rho |x-x'|^2).  The oracle
uses the length-scale form, k_1(x,x') = exp(-(x-x')^2 / (2 ell^2)); the second
form's rho equals 1/(2 ell^2).

Exponential (Matern-1/2), k_1(x,x') = exp(-|x-x'|/ell): Section 2.1 admits Matern
kernels.  It is kept as a test kernel: on sorted inputs its off-diagonal blocks have
rank one exactly, and an O(n) state-space recursion (kalman.py) gives its log
determinant and solves exactly at any n.

Matern-3/2 and Matern-5/2 (Section 2.1 names the Matern family), in the usual
length-scale form with u = sqrt(3) |x-x'| / ell, resp. u = sqrt(5) |x-x'| / ell:
    k_1 = (1 + u) exp(-u),   k_1 = (1 + u + u^2 / 3) exp(-u).
"""
from __future__ import annotations

import numpy as np

SE = 0
EXP = 1
MATERN32 = 2
MATERN52 = 3


def k1(kind: int, ell: float, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Kernel values k_1(a_i, b_j) as an |a| x |b| array (no nugget)."""
    d = np.asarray(a, dtype=np.float64)[:, None] - np.asarray(b, dtype=np.float64)[None, :]
    if kind == SE:
        return np.exp(-(d * d) / (2.0 * ell * ell))
    if kind == EXP:
        return np.exp(-np.abs(d) / ell)
    if kind == MATERN32:
        u = np.sqrt(3.0) * np.abs(d) / ell
        return (1.0 + u) * np.exp(-u)
    if kind == MATERN52:
        u = np.sqrt(5.0) * np.abs(d) / ell
        return (1.0 + u + u * u / 3.0) * np.exp(-u)
    raise ValueError(f"unknown kernel kind {kind}")


def K1_dense(kind: int, ell: float, nugget: float, x: np.ndarray) -> np.ndarray:
    """K_1 = [k_1(x_i, x_j)] + nugget * I (the nugget is added before the H-matrix
    construction, Section 4.1 'Additional considerations')."""
    K = k1(kind, ell, x, x)
    K[np.diag_indices_from(K)] += nugget
    return K
