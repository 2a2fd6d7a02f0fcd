"""Seeded dense vectors."""
import numpy as np


def uniform_vector(n, seed, low=-1.0, high=1.0):
    """x ~ U[low, high)^n from numpy's PCG64 generator seeded with ``seed``."""
    return np.random.default_rng(seed).uniform(low, high, int(n))


def integer_vector(n, seed, bound=1 << 20):
    """Integer-valued FP64 vector, entries uniform in [-bound, bound].

    With stencil matrices (integer entries, max row sum of |a_ij| <= 12) and a
    handful of powers every partial sum stays an integer below 2^53, so the
    matrix powers of such a vector are exact in FP64 for any summation order.
    """
    rng = np.random.default_rng(seed)
    return rng.integers(-bound, bound, int(n), endpoint=True).astype(np.float64)
