"""Pins of the oracle's counter-based generator (oracle/rng.py).

Philox4x64-10 is checked bit for bit against numpy's own implementation of the same
published generator (numpy.random.Philox); the transforms against their
distributions."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import rng


@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)),
                                     ((5, 7, 11, 13), (12345, 678)),
                                     ((2**64 - 3, 2**63, 1, 2**40), (2**64 - 1, 2**62 + 17))])
def test_philox_matches_numpy(ctr, key):
    # numpy increments the counter before generating its first block
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    ref = bg.random_raw(12)
    got = []
    c0 = ctr[0]
    for blk in range(1, 4):
        cc = c0 + blk
        carry = cc >> 64
        w = rng.philox4x64_10(
            (np.array([cc & (2**64 - 1)], dtype=np.uint64), np.uint64((ctr[1] + carry) % 2**64),
             np.uint64(ctr[2]), np.uint64(ctr[3])), key)
        got += [int(v[0]) for v in w]
    assert got == [int(v) for v in ref]


def test_uniform_open_interval():
    w = np.array([0, 2**64 - 1, 2**12 - 1, 2**12], dtype=np.uint64)
    u = rng.to_uniform(w)
    assert u[0] == 0.5 * 2.0 ** -52 and 0.0 < u[0]
    assert u[1] < 1.0 and u[1] == 1.0 - 0.5 * 2.0 ** -52
    assert u[2] == u[0] and u[3] == 1.5 * 2.0 ** -52


def test_normals_distribution_and_layout():
    z = rng.normals(200001, 3, rng.TAG_A, 4, 5)
    assert z.shape == (200001,)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # layout: block j -> entries 4j..4j+3; Box-Muller pairs (cos, sin)
    u0, u1, u2, u3 = rng.block_uniforms(3, rng.TAG_A, 4, 5, [7])
    r = math.sqrt(-2.0 * math.log(u0[0]))
    assert z[28] == pytest.approx(r * math.cos(2 * math.pi * u1[0]), rel=0, abs=1e-15)
    assert z[29] == pytest.approx(r * math.sin(2 * math.pi * u1[0]), rel=0, abs=1e-15)
    # distinct streams differ
    assert not np.allclose(z[:8], rng.normals(8, 3, rng.TAG_B, 4, 5))
    assert not np.allclose(z[:8], rng.normals(8, 3, rng.TAG_A, 4, 6))


@pytest.mark.parametrize("shape", [0.3, 1.0, 2.5, 500.5])
def test_gamma_distribution(shape):
    g = np.array([rng.gamma(shape, 11, rng.TAG_G_TAU, it, 0)[0] for it in range(4000)])
    assert stats.kstest(g, stats.gamma(shape).cdf).pvalue > 1e-4
