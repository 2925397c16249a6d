"""Seeded random arrays for adjoint and gradient tests."""
import numpy as np


def random_array(shape, seed, dist="normal", low=0.0, high=1.0):
    """float64 array from ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    if dist == "normal":
        return rng.standard_normal(size=shape)
    if dist == "uniform":
        return rng.uniform(low, high, size=shape)
    raise ValueError(f"unknown dist {dist!r}")
