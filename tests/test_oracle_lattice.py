"""Pins of the oracle's velocity sets: Table 1 as printed, and exact isotropy identities."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import lattice as lat

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_stencils.json")
GROUP_OF_NORM = {0: "rest", 1: "face", 2: "edge", 3: "corner"}


def _frac(s):
    return Fraction(s)


@pytest.mark.parametrize("q", [7, 15, 19, 27])
def test_matches_table1_as_printed(q):
    table = json.load(open(GOLDEN))[f"D3Q{q}"]
    L = lat.BY_Q[q]
    cs = table["cs"]
    expect_cs2 = Fraction(1, 4) if cs == "1/2" else Fraction(1, 3)
    assert L.cs2_exact == expect_cs2
    # group sizes and weights
    seen = {}
    for i in range(q):
        norm = int(np.abs(L.e[i]).sum())
        seen.setdefault(GROUP_OF_NORM[norm], []).append(L.w_exact[i])
    assert sorted(seen) == sorted(g[0] for g in table["groups"])
    for name, count, weight in table["groups"]:
        assert len(seen[name]) == count
        assert all(w == _frac(weight) for w in seen[name])
    # every velocity distinct, components in {-1, 0, 1}
    assert len({tuple(v) for v in L.e}) == q
    assert np.all(np.abs(L.e) <= 1)


@pytest.mark.parametrize("q", [7, 15, 19, 27])
def test_opposite_map(q):
    L = lat.BY_Q[q]
    for i in range(q):
        assert np.array_equal(L.e[L.opp[i]], -L.e[i])
    # directions come in pairs (i, i + 1) for odd i
    for i in range(1, q, 2):
        assert L.opp[i] == i + 1


def _moment(L, idx):
    tot = Fraction(0)
    for i in range(L.q):
        term = L.w_exact[i]
        for a in idx:
            term *= int(L.e[i][a])
        tot += term
    return tot


@pytest.mark.parametrize("q", [7, 15, 19, 27])
def test_isotropy_to_third_order(q):
    L = lat.BY_Q[q]
    c2 = L.cs2_exact
    assert _moment(L, ()) == 1
    for a in range(3):
        assert _moment(L, (a,)) == 0
    for a, b in itertools.product(range(3), repeat=2):
        assert _moment(L, (a, b)) == (c2 if a == b else 0)
    for idx in itertools.product(range(3), repeat=3):
        assert _moment(L, idx) == 0


@pytest.mark.parametrize("q", [15, 19, 27])
def test_fourth_order_isotropy(q):
    L = lat.BY_Q[q]
    c4 = L.cs2_exact ** 2
    for a, b, c, d in itertools.product(range(3), repeat=4):
        delta = lambda i, j: 1 if i == j else 0
        expect = c4 * (delta(a, b) * delta(c, d) + delta(a, c) * delta(b, d)
                       + delta(a, d) * delta(b, c))
        assert _moment(L, (a, b, c, d)) == expect


def test_d3q7_is_not_fourth_order_isotropic():
    # sum w e_x^4 = 1/4, while 3 c_s^4 = 3/16: the compact scalar stencil is only
    # second-order isotropic, which is why its equilibrium keeps exact zeroth and
    # first moments only.
    L = lat.D3Q7
    assert _moment(L, (0, 0, 0, 0)) == Fraction(1, 4)
    assert 3 * L.cs2_exact ** 2 == Fraction(3, 16)


def test_subsets_share_the_d3q27_order():
    full = [tuple(v) for v in lat.D3Q27.e]
    assert [tuple(v) for v in lat.D3Q19.e] == full[:19]
    assert [tuple(v) for v in lat.D3Q7.e] == full[:7]
    assert [tuple(v) for v in lat.D3Q15.e] == full[:7] + full[19:]
