"""Pins of the oracle's dual filter order (order = 1): at every radius the
homotopic filling first, then the cutting (HC_i o HF_i), beside the formula
of Sec. 2 (HF_i o HC_i). The stage bounds come from brute-force ball stamping
and the topology from component counting, both independent of the oracle."""
import numpy as np
import pytest

import oracle
import topo_checks as tc
from paper_1603_09337_amd import synth


def _img(k):
    if k == 0:
        return synth.workload_disks(H=64, W=72)[0]
    return synth.random_binary(40 + 3 * k, 37 + 5 * k, 0.55, 700 + k)


@pytest.mark.parametrize("k", range(3))
@pytest.mark.parametrize("r", [1, 3])
def test_dual_order_stage_bounds_and_topology(k, r):
    X = _img(k)
    rng = np.random.default_rng(40 + k)
    C = ((rng.random(X.shape) < 0.02) & (X != 0)).astype(np.uint8)
    out, st = oracle.hasf(X, C, r, stages=True, order=1)
    prev = X != 0
    for i in range(1, r + 1):
        z, f, y, c = (st[i - 1, s] != 0 for s in range(4))
        # HF_i: the thickening Z and the filling stay between prev and its dilation
        for s in (z, f):
            assert (prev <= s).all() and (s <= tc.dilate_stamp(prev, i)).all()
        # HC_i of the filled set: between its erosion (with C) and itself
        low = tc.erode_stamp(f, i) | (C != 0)
        for s in (y, c):
            assert (s <= f).all() and (low <= s).all()
        for s in (z, f, y, c):
            assert tc.topology(s) == tc.topology(X)
        prev = c
    assert np.array_equal(out != 0, prev)


def test_dual_order_composes_single_steps():
    X, r = synth.workload_disks(H=80, W=64)[0], 3
    C = ((np.random.default_rng(5).random(X.shape) < 0.03) & (X != 0)).astype(np.uint8)
    out = oracle.hasf(X, C, r, order=1)
    x = X.copy()
    for i in range(1, r + 1):
        x = oracle.hf(x, i)
        x = oracle.hc(x, C, i)
    assert np.array_equal(out, x)


# disks left unchanged by the classical opening and closing for every i <= r:
# both orders must leave them unchanged
@pytest.mark.parametrize("R,r", [(5, 1), (9, 2), (14, 3), (23, 5)])
def test_dual_order_smooth_disk_is_a_fixed_point(R, r):
    X = tc.disk_image(R)
    for i in range(1, r + 1):
        assert np.array_equal(tc.opening(X, i), X != 0)
        assert np.array_equal(tc.closing(X, i), X != 0)
    assert np.array_equal(oracle.hasf(X, None, r, order=1), X)


def test_the_order_matters():
    # filling first closes notches the cutting would otherwise widen; on
    # noisy shapes the two orders give different (both valid) smoothings
    diff = 0
    for k in range(3):
        X = _img(k)
        a, b = oracle.hasf(X, None, 2), oracle.hasf(X, None, 2, order=1)
        assert tc.topology(a) == tc.topology(b) == tc.topology(X)
        diff += int((a != b).sum())
    assert diff > 0


def test_dual_order_identity_empty_and_constraints():
    X = _img(1)
    assert np.array_equal(oracle.hasf(X, None, 0, order=1), (X != 0).astype(np.uint8))
    assert not oracle.hasf(np.zeros((30, 20), np.uint8), None, 4, order=1).any()
    rng = np.random.default_rng(9)
    C = ((rng.random(X.shape) < 0.05) & (X != 0)).astype(np.uint8)
    D = ((rng.random(X.shape) < 0.05) & (X == 0)).astype(np.uint8)
    for n, topo in ((8, tc.topology), (4, tc.topology48)):
        Y = oracle.hasf(X, C, 3, D=D, n=n, order=1)
        assert topo(Y) == topo(X)
        assert ((C != 0) <= (Y != 0)).all()
        assert not (Y[D != 0]).any()


def test_bad_order_is_refused():
    with pytest.raises(Exception):
        oracle.hasf(_img(1), None, 2, order=2)
