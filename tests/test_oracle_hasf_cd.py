"""Pins of the oracle's HASF^{C,D} with a background constraint set D and the
(4,8) connectivity pair (Sec. 2: (n, n-bar) is (8,4) or (4,8); D is a subset
of the complement of X that the filling never adds to)."""
import numpy as np
import pytest

import oracle
import topo_checks as tc
from paper_1603_09337_amd import synth


def _img(k, H=44, W=52):
    if k == 0:
        return synth.workload_disks(H=64, W=72)[0]
    return synth.random_binary(H + 3 * k, W + 5 * k, 0.55, 700 + k)


def test_euler48_on_textbook_cases():
    # a 4-connected ring has Euler number 0; two diagonal pixels are two
    # 4-components (Euler 2) but one 8-component (Euler 1)
    ring = np.zeros((5, 5), np.uint8)
    ring[1:4, 1:4] = 1
    ring[2, 2] = 0
    assert tc.euler48_quads(ring) == 0 and tc.components4(ring) == 1
    diag = np.array([[1, 0], [0, 1]], np.uint8)
    assert tc.euler48_quads(diag) == 2 and tc.euler84_quads(diag) == 1
    for k in range(1, 6):
        X = synth.random_binary(20, 23, 0.5, 800 + k)
        # Euler = components - holes under the same pair
        assert tc.euler48_quads(X) == tc.components4(X) - (tc.components8_complement(X) - 1)


@pytest.mark.parametrize("k", range(4))
@pytest.mark.parametrize("r", [1, 2, 3])
def test_48_filter_keeps_48_topology_at_every_stage(k, r):
    X = _img(k)
    rng = np.random.default_rng(k + 10 * r)
    C = ((rng.random(X.shape) < 0.03) & (X != 0)).astype(np.uint8)
    out, st = oracle.hasf(X, C, r, stages=True, n=4)
    t = tc.topology48(X)
    for i in range(r):
        for s in range(4):
            assert tc.topology48(st[i, s]) == t, (i, s)
    assert ((C != 0) <= (out != 0)).all()


@pytest.mark.parametrize("k", range(3))
@pytest.mark.parametrize("i", [1, 2])
def test_48_cutting_and_filling_bounds(k, i):
    X = _img(k)
    out, st = oracle.hasf(X, None, i, stages=True, n=4)
    # radius i: before it, the state after radius i - 1
    prev = X if i == 1 else oracle.hasf(X, None, i - 1, n=4)
    cut, filled = st[i - 1, 1], st[i - 1, 3]
    assert ((cut != 0) <= (prev != 0)).all()
    assert (tc.erode_stamp(prev, i) <= (cut != 0)).all()
    assert ((cut != 0) <= (filled != 0)).all()
    assert ((filled != 0) <= tc.dilate_stamp(cut, i)).all()


def test_the_pair_matters():
    # the (8,4) filter changes the (4,8) topology of some image (so a filter
    # that used the wrong table would fail the check above), and the two
    # filters give different results
    broke, differ = False, False
    for k in range(1, 8):
        X = synth.random_binary(40, 45, 0.5, 900 + k)
        y8 = oracle.hasf(X, None, 2, n=8)
        y4 = oracle.hasf(X, None, 2, n=4)
        broke |= tc.topology48(y8) != tc.topology48(X)
        differ |= not np.array_equal(y8, y4)
    assert broke and differ


@pytest.mark.parametrize("R,r", [(5, 1), (10, 1), (9, 2), (12, 2), (14, 3)])
def test_48_smooth_disk_is_a_fixed_point(R, r):
    X = tc.disk_image(R)
    assert np.array_equal(oracle.hasf(X, None, r, n=4), X)


@pytest.mark.parametrize("n", [8, 4])
def test_background_constraint_stays_background(n):
    for k in range(4):
        X = _img(k)
        rng = np.random.default_rng(k)
        D = ((rng.random(X.shape) < 0.2) & (X == 0)).astype(np.uint8)
        out, st = oracle.hasf(X, None, 3, stages=True, D=D, n=n)
        assert not (st[:, :, D != 0]).any()
        t = tc.topology(X) if n == 8 else tc.topology48(X)
        assert (tc.topology(out) if n == 8 else tc.topology48(out)) == t


@pytest.mark.parametrize("n", [8, 4])
def test_background_constraint_special_cases(n):
    X = _img(2)
    ref = oracle.hasf(X, None, 3, n=n)
    # empty D is the plain filter; D n X is ignored
    assert np.array_equal(oracle.hasf(X, None, 3, D=np.zeros_like(X), n=n), ref)
    ones = np.ones_like(X)
    comp = (X == 0).astype(np.uint8)
    full = oracle.hasf(X, None, 3, D=ones, n=n)
    assert np.array_equal(full, oracle.hasf(X, None, 3, D=comp, n=n))
    # D = complement of the input: a filling may only give back points of the
    # input that a cutting removed, so every stage stays inside the input
    _, st = oracle.hasf(X, None, 3, stages=True, D=comp, n=n)
    assert ((st != 0) <= (X != 0)).all()
    assert ((full != 0) <= (X != 0)).all()


def test_background_constraint_keeps_a_notch_open():
    # a notch one pixel wide in a block: the filling closes all but its mouth
    # (left as a rounded dent), unless D covers it
    X = np.zeros((24, 24), np.uint8)
    X[4:20, 4:20] = 1
    X[4:12, 11] = 0
    plain = oracle.hasf(X, None, 1)
    assert plain[6:12, 11].all() and not plain[4:6, 11].any()
    D = np.zeros_like(X)
    D[4:12, 11] = 1
    kept = oracle.hasf(X, None, 1, D=D)
    assert not kept[4:12, 11].any()
    assert tc.topology(kept) == tc.topology(X)
