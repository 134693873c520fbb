"""Seeded uniform draws used by the optimiser's cold start."""
import numpy as np


def box_uniform(seed, shape, lo, hi):
    return np.random.default_rng(seed).uniform(lo, hi, shape)
