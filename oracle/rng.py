"""Counter-based random numbers for the oracle (test infrastructure only).

Philox4x64-10 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11).  One block maps a 256-bit
counter and a 128-bit key to four 64-bit words through ten rounds of two 64x64->128
multiplies; the key is bumped by two Weyl constants between rounds.

Stream layout used by the sampler (the HIP path implements the same definition on
its own):
  key     = (seed, 0)
  counter = (block, tag, iteration, stream)      stream = chain / job id
  uniform = ((w >> 12) + 0.5) * 2^-52            in (0, 1), never 0 or 1
            (52 bits so that the half-step offset is exact in FP64)
  normals: block j yields words w0..w3 -> uniforms u0..u3; Box-Muller on (u0,u1)
           gives z[4j] = r cos(2 pi u1), z[4j+1] = r sin(2 pi u1) with
           r = sqrt(-2 log u0); (u2, u3) gives z[4j+2], z[4j+3] the same way.
  Gamma(a, 1), a >= 1: Marsaglia & Tsang (ACM TOMS 26(3), 2000).  Try t uses block t:
           z from (u0, u1) (cosine branch), acceptance uniform u2; at most 64 tries.
           a < 1 uses Gamma(a+1) * u^(1/a) with u = u3 of the accepted block.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1
MASK32 = np.uint64(0xFFFFFFFF)

# tags of the Gibbs sweep's draws
TAG_A, TAG_B, TAG_G_TAU, TAG_G_SIGF, TAG_PROP, TAG_ACC = 1, 2, 3, 4, 5, 6
TAG_BETA = 7          # tensor-product model: normal draw of beta
TAG_PRED = 8          # function draws at new inputs
TAG_RHO = 9           # exact discrete length-scale conditional (inverse-CDF uniform)
TAG_FACTOR_STRIDE = 16  # tensor-product model: factor h uses tag + 16*(h+1)


def _mulhilo(a: np.ndarray, b: int):
    """Full 64x64 -> 128-bit product of uint64 array ``a`` and constant ``b``."""
    a = a.astype(np.uint64)
    b_lo = np.uint64(b & 0xFFFFFFFF)
    b_hi = np.uint64(b >> 32)
    a_lo = a & MASK32
    a_hi = a >> np.uint64(32)
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> np.uint64(32)) + (lh & MASK32) + (hl & MASK32)
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    lo = (mid << np.uint64(32)) | (ll & MASK32)
    return hi, lo


def philox4x64_10(counter, key):
    """Ten Philox-4x64 rounds.  ``counter``: 4 uint64 arrays (broadcastable),
    ``key``: 2 python ints.  Returns 4 uint64 arrays."""
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = [np.asarray(c, dtype=np.uint64) for c in counter]
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
        for r in range(10):
            hi0, lo0 = _mulhilo(c0, M0)
            hi1, lo1 = _mulhilo(c2, M1)
            c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                              hi0 ^ c3 ^ np.uint64(k1), lo0)
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        return c0, c1, c2, c3


def to_uniform(w: np.ndarray) -> np.ndarray:
    """52-bit uniform strictly inside (0, 1); every step is exact in FP64."""
    return ((w >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def block_uniforms(seed, tag, iteration, stream, blocks):
    """Uniforms u0..u3 of the given block indices (array)."""
    blocks = np.asarray(blocks, dtype=np.uint64)
    w = philox4x64_10((blocks, np.uint64(tag), np.uint64(iteration), np.uint64(stream)),
                      (seed, 0))
    return [to_uniform(wi) for wi in w]


def normals(n, seed, tag, iteration, stream):
    """n standard normals of stream (seed, tag, iteration, stream)."""
    nb = (n + 3) // 4
    u0, u1, u2, u3 = block_uniforms(seed, tag, iteration, stream, np.arange(nb))
    out = np.empty(4 * nb)
    r01 = np.sqrt(-2.0 * np.log(u0))
    r23 = np.sqrt(-2.0 * np.log(u2))
    out[0::4] = r01 * np.cos(2.0 * np.pi * u1)
    out[1::4] = r01 * np.sin(2.0 * np.pi * u1)
    out[2::4] = r23 * np.cos(2.0 * np.pi * u3)
    out[3::4] = r23 * np.sin(2.0 * np.pi * u3)
    return out[:n]


def uniform(seed, tag, iteration, stream):
    """One uniform (word 0 of block 0)."""
    return float(block_uniforms(seed, tag, iteration, stream, [0])[0][0])


def gamma(shape, seed, tag, iteration, stream, max_tries=64):
    """Gamma(shape, 1) by Marsaglia & Tsang; returns (value, tries_used)."""
    boost = shape < 1.0
    a = shape + 1.0 if boost else shape
    d = a - 1.0 / 3.0
    c = 1.0 / np.sqrt(9.0 * d)
    for t in range(max_tries):
        u0, u1, u2, u3 = [float(v[0]) for v in block_uniforms(seed, tag, iteration, stream, [t])]
        z = np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)
        v = 1.0 + c * z
        if v <= 0.0:
            continue
        v = v * v * v
        if np.log(u2) < 0.5 * z * z + d - d * v + d * np.log(v):
            g = d * v
            if boost:
                g *= u3 ** (1.0 / shape)
            return g, t + 1
    return d, max_tries
