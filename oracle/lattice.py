"""Discrete velocity sets D3Q7, D3Q15, D3Q19 and D3Q27 (paper, Section 2.3, Table 1).

Test infrastructure only: this module belongs to the FP64 CPU oracle, which
exists to check the HIP path.  Nothing in the product library imports it.

Table 1 lists, per stencil, the lattice speed of sound c_s and, per group of
velocities (rest, faces, edges, corners), the weight w_i.  The paper gives
index *ranges* per group but not the order inside a group, so the order below
is a convention of this project: directions come in opposite pairs
(i, i+1) for odd i, and the smaller sets are prefixes or sub-selections of the
D3Q27 list (D3Q7 = 0..6, D3Q19 = 0..18, D3Q15 = 0..6 plus the 8 corners).
Weights are kept as exact rationals so the isotropy identities can be checked
without rounding.
"""
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

REST = [(0, 0, 0)]
FACES = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
EDGES = [
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
]
CORNERS = [
    (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
    (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1),
]

# Table 1: c_s^2 and the weight of each group, per stencil.
_TABLE1 = {
    7: (Fraction(1, 4), [(REST, Fraction(1, 4)), (FACES, Fraction(1, 8))]),
    15: (Fraction(1, 3), [(REST, Fraction(2, 9)), (FACES, Fraction(1, 9)),
                          (CORNERS, Fraction(1, 72))]),
    19: (Fraction(1, 3), [(REST, Fraction(1, 3)), (FACES, Fraction(1, 18)),
                          (EDGES, Fraction(1, 36))]),
    27: (Fraction(1, 3), [(REST, Fraction(8, 27)), (FACES, Fraction(2, 27)),
                          (EDGES, Fraction(1, 54)), (CORNERS, Fraction(1, 216))]),
}


@dataclass(frozen=True)
class Lattice:
    q: int
    e: np.ndarray          # (q, 3) int64, columns are (x, y, z)
    w: np.ndarray          # (q,) float64
    w_exact: tuple         # (q,) Fraction
    cs2: float
    cs2_exact: Fraction
    opp: np.ndarray        # (q,) index of -e_i


def make(q):
    """Build the D3Q<q> set of Table 1."""
    if q not in _TABLE1:
        raise ValueError(f"no D3Q{q} stencil in Table 1")
    cs2, groups = _TABLE1[q]
    vel, wts = [], []
    for members, weight in groups:
        vel.extend(members)
        wts.extend([weight] * len(members))
    e = np.array(vel, dtype=np.int64)
    opp = np.array([vel.index(tuple(-c for c in v)) for v in vel], dtype=np.int64)
    return Lattice(q=q, e=e, w=np.array([float(x) for x in wts]), w_exact=tuple(wts),
                   cs2=float(cs2), cs2_exact=cs2, opp=opp)


D3Q7 = make(7)
D3Q15 = make(15)
D3Q19 = make(19)
D3Q27 = make(27)
BY_Q = {7: D3Q7, 15: D3Q15, 19: D3Q19, 27: D3Q27}
