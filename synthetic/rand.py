"""Seeded random complex vectors (probe and timing inputs)."""

import numpy as np


def complex_normal(shape, seed):
    """complex128 array whose real and imaginary parts are independent N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
