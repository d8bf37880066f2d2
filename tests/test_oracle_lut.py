"""Pins of the oracle's simple-point table (Sec. 2: T, T-bar and the local
characterisation of simple points) against independent definitions."""
import numpy as np
import pytest

import oracle
import topo_checks as tc


def test_count_116_of_256():
    # closed-form count for (8,4) and (4,8) on the 3x3 ring, re-derived by the
    # global check below
    assert int(oracle.simple_lut(8).sum()) == 116
    assert int(oracle.simple_lut(4).sum()) == 116


def test_matches_yokoi_crossing_number():
    lut = oracle.simple_lut(8)
    for m in range(256):
        assert bool(lut[m]) == tc.yokoi_simple(m), m


def test_matches_global_definition_by_component_labelling():
    lut = oracle.simple_lut(8)
    for m in range(256):
        assert bool(lut[m]) == tc.global_simple(m), m


def test_spot_values():
    lut = oracle.simple_lut(8)
    E, NE, N, NW, W, SW, S, SE = (1 << k for k in range(8))
    assert lut[0] == 0          # isolated point
    assert lut[255] == 0        # interior point
    assert lut[E] == 1          # end point
    assert lut[NE] == 1         # diagonal end point
    assert lut[N | S] == 0      # bridge
    assert lut[E | W] == 0
    assert lut[NE | SW] == 0    # diagonal bridge
    assert lut[N | NE | E] == 1  # corner


def _rot90(m):
    # rotating the ring by 90 degrees moves neighbour k to k + 2
    return ((m << 2) | (m >> 6)) & 0xFF


def _mirror(m):
    # reflection about the horizontal axis maps direction k to (8 - k) mod 8
    out = 0
    for k in range(8):
        if (m >> k) & 1:
            out |= 1 << ((8 - k) % 8)
    return out


@pytest.mark.parametrize("n", [8, 4])
def test_dihedral_invariance(n):
    lut = oracle.simple_lut(n)
    for m in range(256):
        assert lut[m] == lut[_rot90(m)] == lut[_mirror(m)]


def test_duality_84_48():
    l84, l48 = oracle.simple_lut(8), oracle.simple_lut(4)
    for m in range(256):
        assert l84[m] == l48[m ^ 0xFF]


def test_topological_numbers_of_known_configurations():
    E, NE, N, NW, W, SW, S, SE = (1 << k for k in range(8))
    assert oracle.topo_numbers(8, 0) == (0, 1)
    assert oracle.topo_numbers(8, 255) == (1, 0)
    assert oracle.topo_numbers(8, N | S) == (2, 2)
    assert oracle.topo_numbers(8, NE | SW | NW | SE) == (4, 4)
    assert oracle.topo_numbers(8, N | NE | E) == (1, 1)
