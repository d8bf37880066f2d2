"""Pins of the ball dilation / erosion by thresholding the oracle's distance map
(Sec. 2: B_r, delta_r, epsilon_r = dual of delta_r)."""
import numpy as np
import pytest

import oracle
import topo_checks as tc

# number of lattice points a^2 + b^2 <= r^2, r = 0..10 (Gauss circle problem)
GAUSS = [1, 5, 13, 29, 49, 81, 113, 149, 197, 253, 317]


def dilate(X, r):
    return oracle.edt_sq(X) <= r * r


def erode(X, r):
    return (oracle.edt_sq((X == 0).astype(np.uint8), frame=True) > r * r) & (X != 0)


@pytest.mark.parametrize("r", range(11))
def test_ball_size_is_gauss_count(r):
    X = np.zeros((31, 31), np.uint8)
    X[15, 15] = 1
    assert int(dilate(X, r).sum()) == GAUSS[r]


@pytest.mark.parametrize("r", [1, 2, 3, 5])
def test_threshold_equals_ball_stamping(r):
    rng = np.random.default_rng(r)
    for d in (0.02, 0.2, 0.6):
        X = (rng.random((40, 33)) < d).astype(np.uint8)
        assert np.array_equal(dilate(X, r), tc.dilate_stamp(X, r))
        assert np.array_equal(erode(X, r), tc.erode_stamp(X, r))


@pytest.mark.parametrize("r", [1, 4])
def test_duality(r):
    rng = np.random.default_rng(100 + r)
    X = (rng.random((37, 41)) < 0.5).astype(np.uint8)
    # erosion of X = complement of the dilation of the complement, where the
    # complement includes the outside of the window
    comp_outside = np.ones((37 + 2 * r + 2, 41 + 2 * r + 2), np.uint8)
    comp_outside[r + 1:-r - 1, r + 1:-r - 1] = X == 0
    dil = tc.dilate_stamp(comp_outside, r)[r + 1:-r - 1, r + 1:-r - 1]
    assert np.array_equal(erode(X, r), ~dil)
