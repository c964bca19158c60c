"""Exact O(n) log-determinant and solve for the exponential kernel (test
infrastructure only).

For k_1(x, x') = exp(-|x - x'| / ell) on sorted inputs, f is an Ornstein-Uhlenbeck
process: f_1 ~ N(0, a), f_i = phi_i f_{i-1} + w_i with phi_i = exp(-(x_i - x_{i-1})/ell)
and w_i ~ N(0, a (1 - phi_i^2)).  With b = f + e, e ~ N(0, s I), Cov(b) = a K_1 + s I.
The Kalman filter's innovation variances S_i give log det(a K_1 + s I) = sum log S_i
(prediction-error decomposition), and the Rauch-Tung-Striebel smoother's mean f^ gives
(a K_1 + s I)^-1 b = (b - f^) / s.  This is an exact route (up to rounding) that shares
nothing with the hierarchical factorization, at any n.
"""
from __future__ import annotations

import math
import numpy as np


def exp_kernel_logdet_solve(x, ell, a, s, b):
    x = np.asarray(x, float)
    b = np.asarray(b, float)
    n = x.size
    phi = np.empty(n)
    phi[0] = 0.0
    phi[1:] = np.exp(-np.diff(x) / ell)
    mp = np.empty(n)
    Pp = np.empty(n)
    mf = np.empty(n)
    Pf = np.empty(n)
    logdet = 0.0
    m, P = 0.0, 0.0
    for i in range(n):
        if i == 0:
            mpi, Ppi = 0.0, a
        else:
            ph = phi[i]
            mpi = ph * m
            Ppi = ph * ph * P + a * (1.0 - ph * ph)
        S = Ppi + s
        logdet += math.log(S)
        K = Ppi / S
        m = mpi + K * (b[i] - mpi)
        P = Ppi * s / S
        mp[i], Pp[i], mf[i], Pf[i] = mpi, Ppi, m, P
    ms = np.empty(n)
    ms[-1] = mf[-1]
    for i in range(n - 2, -1, -1):
        G = Pf[i] * phi[i + 1] / Pp[i + 1]
        ms[i] = mf[i] + G * (ms[i + 1] - mp[i + 1])
    return logdet, (b - ms) / s
