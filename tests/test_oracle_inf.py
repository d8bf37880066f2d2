"""Pins of the oracle's "r = infinity" (Tab. 1 reports r = infinity; the paper
does not define it): radii 1, 2, ... until the first radius whose cutting and
filling leave the set unchanged, at most up to the saturation radius (from
there on every radius applies the same operator).

The oracle is compared, result and stopping radius, with an independent
composition (tests/topo_checks.py: ball stamping, scipy's exact transform, a
numpy subfield schedule), and with its own finite-radius filter at the
stopping radius and one below it (the last radius changed nothing)."""
import numpy as np
import pytest

import oracle
import topo_checks as tc
from paper_1603_09337_amd import synth


def _case(k):
    rng = np.random.default_rng(4400 + k)
    H = int(rng.integers(12, 34))
    W = int(rng.integers(12, 34))
    if k % 3 == 2:
        X = synth.random_binary(H, W, 0.5, 4500 + k)
    else:
        X = synth.draw(H, W, synth._rng(4500 + k), 3, 3, 10, 0.3, n_holes=1, p_flip=0.25, sp_frac=0.03)
    C = ((rng.random((H, W)) < 0.04) & (X != 0)).astype(np.uint8)
    D = ((rng.random((H, W)) < 0.04) & (X == 0)).astype(np.uint8)
    return X, C, D


COMBOS = [(n, order, useC, useD) for n in (8, 4) for order in (0, 1) for useC in (0, 1) for useD in (0, 1)]


@pytest.mark.parametrize("k", range(16))
def test_inf_equals_independent_composition(k):
    n, order, useC, useD = COMBOS[k]
    X, C, D = _case(k)
    C = C if useC else None
    D = D if useD else None
    got, used = oracle.hasf_inf(X, C, D, n=n, order=order)
    ref, ref_used = tc.hasf_inf_composed(X, C, D, n=n, order=order)
    assert used == ref_used
    assert np.array_equal(got, ref)
    # the finite filter at the stopping radius, and one below it, agree
    assert np.array_equal(oracle.hasf(X, C, used, D=D, n=n, order=order), got)
    if used > 1:
        assert np.array_equal(oracle.hasf(X, C, used - 1, D=D, n=n, order=order), got)


def test_inf_past_the_fixed_radii_of_the_kernels():
    # a square's corners are rounded at every radius up to about half its side
    X = np.zeros((48, 52), np.uint8)
    X[6:42, 8:44] = 1
    got, used = oracle.hasf_inf(X)
    ref, ref_used = tc.hasf_inf_composed(X, None, None)
    assert used == ref_used and used > 15
    assert np.array_equal(got, ref)
    assert tc.topology(got) == tc.topology(X)


def test_inf_keeps_topology_and_constraints():
    for k in range(6):
        X, C, D = _case(20 + k)
        got, used = oracle.hasf_inf(X, C, D)
        assert tc.topology(got) == tc.topology(X)
        assert ((C != 0) <= (got != 0)).all()
        assert not ((D != 0) & (got != 0)).any()
        # one more application of the stopping radius changes nothing
        again = tc.hf_composed(tc.hc_composed(got, C & got, used, tc.simple_table(8))[1], D, used,
                               tc.simple_table(8))[1]
        assert np.array_equal(again.astype(np.uint8), got)


def test_inf_caps():
    X = np.zeros((48, 52), np.uint8)
    X[6:42, 8:44] = 1
    got, used = oracle.hasf_inf(X, r_max=4)
    assert used == 4 and np.array_equal(got, oracle.hasf(X, None, 4))
    # saturation radius of a 3 x 3 window: 3 (3^2 >= 2^2 + 2^2)
    F = np.ones((3, 3), np.uint8)
    got, used = oracle.hasf_inf(F)
    assert used <= 3 and np.array_equal(got, tc.hasf_inf_composed(F, None, None)[0])
    Z = np.zeros((9, 7), np.uint8)
    got, used = oracle.hasf_inf(Z)
    assert used == 1 and not got.any()
