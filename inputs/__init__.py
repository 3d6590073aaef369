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


def index_pattern(i, z, y, x):
    """A deterministic population-deviation pattern over (direction i, node z, y, x):
    ((37 i + 11 x + 5 y + 3 z) mod 251 - 125) / 4096.  Every value is a multiple of 2^-12
    of magnitude at most 125 * 2^-12, so FP32, FP16 and BF16 all hold it exactly; it lets a
    large box be checked at sampled nodes without the whole state on the host.  Works on
    NumPy arrays and on torch tensors (of any device) alike."""
    k = (37 * i + 11 * x + 5 * y + 3 * z) % 251
    return (k - 125) * (1.0 / 4096.0)


def index_pattern_state(q, n, device):
    """(q, n, n, n) FP32 torch tensor of index_pattern, built on `device` one direction at
    a time (int32 intermediates of one n^3 slice)."""
    import torch
    out = torch.empty((q, n, n, n), dtype=torch.float32, device=device)
    z = torch.arange(n, device=device, dtype=torch.int32).view(n, 1, 1)
    y = torch.arange(n, device=device, dtype=torch.int32).view(1, n, 1)
    x = torch.arange(n, device=device, dtype=torch.int32).view(1, 1, n)
    for i in range(q):
        out[i] = index_pattern(i, z, y, x).to(torch.float32)
    return out
