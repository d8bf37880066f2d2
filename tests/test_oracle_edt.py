"""Pins of the oracle's squared Euclidean distance transform (Sec. 4.1)."""
import numpy as np
import pytest

import oracle
import topo_checks as tc
from paper_1603_09337_amd import synth

U32MAX = np.iinfo(np.uint32).max


def _cases():
    rng = np.random.default_rng(20160330)
    out = []
    for k in range(120):
        H, W = (int(v) for v in rng.integers(1, 25, 2))
        d = [0.0, 0.01, 0.3, 0.9, 1.0][k % 5]
        out.append(((rng.random((H, W)) < d).astype(np.uint8), bool(k % 2)))
    return out


@pytest.mark.parametrize("direct", [True, False])
def test_against_brute_force(direct):
    for F, frame in _cases():
        assert np.array_equal(oracle.edt_sq(F, frame, direct=direct), tc.edt_brute(F, frame))


@pytest.mark.parametrize("shape", [(1, 1), (1, 17), (17, 1), (2, 2), (31, 5)])
@pytest.mark.parametrize("frame", [False, True])
def test_degenerate_shapes(shape, frame):
    rng = np.random.default_rng(7)
    for d in (0.0, 0.2, 1.0):
        F = (rng.random(shape) < d).astype(np.uint8)
        exp = tc.edt_brute(F, frame)
        assert np.array_equal(oracle.edt_sq(F, frame), exp)
        assert np.array_equal(oracle.edt_sq(F, frame, direct=True), exp)


def test_closed_forms():
    H, W = 23, 37
    # empty, no frame: "infinite" distance
    assert (oracle.edt_sq(np.zeros((H, W), np.uint8)) == U32MAX).all()
    # all features: zero
    assert (oracle.edt_sq(np.ones((H, W), np.uint8)) == 0).all()
    # frame only: squared distance to the nearest side outside the window
    ii, jj = np.mgrid[0:H, 0:W]
    d = np.minimum(np.minimum(ii + 1, H - ii), np.minimum(jj + 1, W - jj))
    assert np.array_equal(oracle.edt_sq(np.zeros((H, W), np.uint8), frame=True), d * d)
    # one feature pixel: (di)^2 + (dj)^2
    F = np.zeros((H, W), np.uint8)
    F[5, 30] = 1
    assert np.array_equal(oracle.edt_sq(F), (ii - 5) ** 2 + (jj - 30) ** 2)


def test_values_are_sums_of_two_squares_and_zero_on_features():
    X, _, _ = synth.workload_disks()
    D = oracle.edt_sq(X)
    sums = set(a * a + b * b for a in range(0, 400) for b in range(0, 400))
    assert set(np.unique(D).tolist()) <= sums
    assert (D[X != 0] == 0).all() and (D[X == 0] > 0).all()


def test_meijster_equals_direct_on_a_generated_image():
    X, _, _ = synth.workload_disks(H=96, W=80)
    for frame in (False, True):
        F = (X == 0).astype(np.uint8) if frame else X
        assert np.array_equal(oracle.edt_sq(F, frame), oracle.edt_sq(F, frame, direct=True))
