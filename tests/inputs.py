"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module draws random numbers and builds arrays of given shapes; it holds
none of the method's arithmetic.  Prior draws are N(0, I_K), as the prior of
the KL coefficients; uniforms are exact multiples of 2^-53 in [0, 1).
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def theta_batch(seed, N, K, scale=1.0):
    return scale * rng(seed).standard_normal((N, K))


def uniforms53(seed, N):
    """iid uniforms in [0,1), each an exact multiple of 2^-53."""
    bits = rng(seed).integers(0, 2 ** 53, size=N, dtype=np.int64)
    return bits.astype(np.float64) * 2.0 ** -53


def weights(seed, N, spread=3.0, zero_frac=0.0):
    g = rng(seed)
    w = np.exp(spread * g.standard_normal(N))
    if zero_frac > 0:
        w[g.random(N) < zero_frac] = 0.0
    return w


def kappa_batch(seed, N, n_elem, spread=1.0):
    """piecewise-constant positive coefficients, log-normal per element"""
    return np.exp(spread * rng(seed).standard_normal((N, n_elem)))


def potentials(seed, N, scale=10.0):
    return scale * rng(seed).gamma(2.0, size=N)
