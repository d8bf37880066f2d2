"""Pins of the oracle's homotopic cutting HC, filling HF and the alternating
sequential filter HASF (Sec. 2, eq. (i), eq. (ii) and the composition)."""
import numpy as np
import pytest

import oracle
import topo_checks as tc
from paper_1603_09337_amd import synth


def _img(k):
    if k == 0:
        return synth.workload_disks(H=64, W=72)[0]
    return synth.random_binary(40 + 3 * k, 37 + 5 * k, 0.55, 300 + k)


@pytest.mark.parametrize("k", range(3))
@pytest.mark.parametrize("i", [1, 2, 3])
def test_cutting_bounds(k, i):
    X = _img(k)
    rng = np.random.default_rng(k * 10 + i)
    C = ((rng.random(X.shape) < 0.02) & (X != 0)).astype(np.uint8)
    Y = oracle.hc(X, C, i)
    assert tc.topology(Y) == tc.topology(X)
    assert ((Y != 0) <= (X != 0)).all()
    assert ((tc.erode_stamp(X, i) | (C != 0)) <= (Y != 0)).all()


@pytest.mark.parametrize("k", range(3))
@pytest.mark.parametrize("i", [1, 2, 3])
def test_filling_bounds(k, i):
    X = _img(k)
    Z = oracle.hf(X, i)
    assert tc.topology(Z) == tc.topology(X)
    assert ((X != 0) <= (Z != 0)).all()
    assert ((Z != 0) <= tc.dilate_stamp(X, i)).all()


def test_stages_compose():
    X, C, r = synth.workload_disks(H=80, W=64)[0], None, 3
    out, st = oracle.hasf(X, C, r, stages=True)
    assert st.shape == (3, 4, 80, 64)
    x = X.copy()
    for i in range(1, r + 1):
        x = oracle.hc(x, C, i)
        assert np.array_equal(x, st[i - 1, 1])
        x = oracle.hf(x, i)
        assert np.array_equal(x, st[i - 1, 3])
    assert np.array_equal(out, x)
    for i in range(r):
        for s in range(4):
            assert tc.topology(st[i, s]) == tc.topology(X)


def test_identity_and_empty():
    X = _img(1)
    assert np.array_equal(oracle.hasf(X, None, 0), (X != 0).astype(np.uint8))
    E = np.zeros((30, 20), np.uint8)
    assert not oracle.hasf(E, None, 4).any()
    # the full window is a rectangle (the outside is background): the filter
    # only rounds its corners
    F = np.ones((30, 20), np.uint8)
    G = oracle.hasf(F, None, 3)
    assert tc.topology(G) == tc.topology(F)
    assert (tc.erode_stamp(F, 3) <= (G != 0)).all()
    assert G[10:20, :].all() and G[:, 5:15].all() and not G[0, 0]


def test_constraint_kept_and_topology_on_generated_workloads():
    X, C, r = synth.workload_shapes(H=160, W=144)
    Y = oracle.hasf(X, C, 3)
    assert tc.topology(Y) == tc.topology(X)
    assert ((C != 0) <= (Y != 0)).all()


def test_constraint_outside_object_is_ignored():
    X = _img(2)
    C = np.ones_like(X)
    assert np.array_equal(oracle.hasf(X, C, 2), oracle.hasf(X, (X != 0).astype(np.uint8), 2))


# (R, r): disks B_R left unchanged by the classical opening and closing by B_i
# for every i <= r (checked below by ball stamping); then the topology is
# trivial and the homotopic filter must leave the disk unchanged too.
DISKS = [(4, 1), (5, 1), (10, 1), (6, 2), (9, 2), (12, 2), (10, 3), (14, 3), (23, 5)]


@pytest.mark.parametrize("R,r", DISKS)
def test_smooth_disk_is_a_fixed_point(R, r):
    X = tc.disk_image(R)
    for i in range(1, r + 1):
        assert np.array_equal(tc.opening(X, i), X != 0)
        assert np.array_equal(tc.closing(X, i), X != 0)
    assert np.array_equal(oracle.hasf(X, None, r), X)


def test_disk_the_opening_cuts_is_smoothed_but_keeps_topology():
    # (R, r) = (8, 2): the classical opening by B_2 removes pixels of B_8
    X = tc.disk_image(8)
    assert not np.array_equal(tc.opening(X, 2), X != 0)
    Y = oracle.hasf(X, None, 2)
    assert tc.topology(Y) == tc.topology(X)


def test_queue_ordered_filter_invariants():
    X, C, r = synth.workload_disks(H=72, W=64)[0], None, 3
    Yq = oracle.hasf(X, C, r, queue=True)
    Ys = oracle.hasf(X, C, r)
    assert tc.topology(Yq) == tc.topology(X) == tc.topology(Ys)
    # both are correct smoothings; they may differ in a few pixels only
    assert (Yq != Ys).mean() < 0.05
