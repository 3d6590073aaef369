"""Seeded synthetic inputs shared by the oracle side and the HIP side of the tests.

This module holds none of the method's arithmetic (no stencil tables, no
equilibria): only seeded random numbers with the structure the tests need.
Values are FP32 so both sides start from bit-identical numbers.
"""
import numpy as np


def uniform_deviations(q, n, amplitude, seed):
    """(q, n, n, n) FP32 values uniform in [-amplitude, amplitude]: population deviations."""
    rng = np.random.default_rng(seed)
    return (amplitude * rng.uniform(-1.0, 1.0, (q, n, n, n))).astype(np.float32)


def sample_nodes(n, count, seed):
    """`count` distinct node coordinates (z, y, x) of an n^3 box, including the corners of the box."""
    rng = np.random.default_rng(seed)
    corners = [(z, y, x) for z in (0, n - 1) for y in (0, n - 1) for x in (0, n - 1)]
    pts = set(corners)
    while len(pts) < count:
        pts.add(tuple(int(v) for v in rng.integers(0, n, 3)))
    return sorted(pts)
