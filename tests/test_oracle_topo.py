"""Pins of the oracle's constrained thinning H and thickening *H (Sec. 2):
topology preserved, constraints kept, result ultimate, and agreement with a
second, in-place implementation of the same schedule."""
import numpy as np
import pytest

import oracle
import topo_checks as tc
from paper_1603_09337_amd import synth


def _images():
    out = []
    for k, (H, W, d) in enumerate([(24, 31, 0.5), (33, 20, 0.7), (40, 40, 0.35), (17, 45, 0.6)]):
        out.append(synth.random_binary(H, W, d, 900 + k))
    out.append(synth.workload_disks(H=48, W=56)[0])
    return out


def _thin_priority(S):
    return oracle.edt_sq((S == 0).astype(np.uint8), frame=True)


@pytest.mark.parametrize("idx", range(5))
def test_thin_preserves_topology_and_is_ultimate(idx):
    S = _images()[idx]
    rng = np.random.default_rng(idx)
    K = ((rng.random(S.shape) < 0.05) & (S != 0)).astype(np.uint8)
    P = _thin_priority(S)
    T, rounds = oracle.thin_p(S, K, P)
    assert tc.topology(T) == tc.topology(S)
    assert ((T != 0) <= (S != 0)).all()                 # anti-extensive
    assert ((K != 0) <= (T != 0)).all()                 # constraint kept
    # ultimate: no unconstrained object point is still simple
    assert not (tc.simple_mask(T) & (T != 0) & (K == 0)).any()
    assert rounds >= 1


@pytest.mark.parametrize("idx", range(5))
def test_thicken_preserves_topology_and_is_ultimate(idx):
    S = _images()[idx]
    rng = np.random.default_rng(50 + idx)
    V = (rng.random(S.shape) < 0.7).astype(np.uint8)
    P = oracle.edt_sq(S)
    T, _ = oracle.thicken_p(S, V, P)
    assert tc.topology(T) == tc.topology(S)
    assert ((S != 0) <= (T != 0)).all()                  # extensive
    assert ((T != 0) <= ((S != 0) | (V != 0))).all()     # stays within S u V
    assert not (tc.simple_mask(T) & (T == 0) & (V != 0)).any()


@pytest.mark.parametrize("idx", range(4))
def test_schedule_matches_in_place_raster_implementation(idx):
    S = _images()[idx]
    rng = np.random.default_rng(77 + idx)
    K = ((rng.random(S.shape) < 0.03) & (S != 0)).astype(np.uint8)
    P = _thin_priority(S)
    assert np.array_equal(oracle.thin_p(S, K, P)[0], tc.sequential_schedule(0, S, K, P))
    V = (rng.random(S.shape) < 0.6).astype(np.uint8)
    P2 = oracle.edt_sq(S)
    assert np.array_equal(oracle.thicken_p(S, V, P2)[0], tc.sequential_schedule(1, S, V, P2))


def test_distinct_levels_equal_all_integer_levels():
    # empty levels are no-ops: collapsing P onto a coarser set of keys that keeps
    # the order of distinct values gives the same result
    S = _images()[2]
    P = _thin_priority(S)
    vals = np.unique(P)
    rank = np.searchsorted(vals, P).astype(np.uint32)
    assert np.array_equal(oracle.thin_p(S, None, P)[0], oracle.thin_p(S, None, rank)[0])


def test_constant_priority_is_plain_ultimate_thinning():
    S = _images()[0]
    T, _ = oracle.thin_p(S, None, np.zeros(S.shape, np.uint32))
    assert tc.topology(T) == tc.topology(S)
    assert not (tc.simple_mask(T) & (T != 0)).any()


def test_queue_variant_invariants():
    for idx, S in enumerate(_images()):
        P = _thin_priority(S)
        T, _ = oracle.thin_p(S, None, P, queue=True)
        assert tc.topology(T) == tc.topology(S)
        assert not (tc.simple_mask(T) & (T != 0)).any()
        V = np.ones(S.shape, np.uint8)
        U, _ = oracle.thicken_p(S, V, oracle.edt_sq(S), queue=True)
        assert tc.topology(U) == tc.topology(S)
        assert not (tc.simple_mask(U) & (U == 0)).any()


def test_homotopic_thin_and_thicken_entry_points():
    S = _images()[4]
    T = oracle.homotopic_thin(S)
    assert np.array_equal(T, oracle.thin_p(S, None, _thin_priority(S))[0])
    V = tc.dilate_stamp(S, 3).astype(np.uint8)
    U = oracle.homotopic_thicken(S, V)
    assert np.array_equal(U, oracle.thicken_p(S, V, oracle.edt_sq(S))[0])


def test_planted_table_mistake_is_caught():
    """Mark the bridge configuration N+S as simple: thinning a vertical bar of
    width one with that table breaks it, and the invariant check notices."""
    lut = oracle.simple_lut(8).copy()
    N, S_ = 1 << 2, 1 << 6
    lut[N | S_] = 1
    X = np.zeros((9, 9), np.uint8)
    X[1:8, 4] = 1
    X[1, 3] = X[7, 5] = 1
    P = _thin_priority(X)
    good, _ = oracle.thin_p(X, None, P)
    bad, _ = oracle.thin_p_lut(X, None, P, lut)
    assert tc.topology(good) == tc.topology(X)
    assert tc.topology(bad) != tc.topology(X)
