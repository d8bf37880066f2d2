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


# The (4,8) pair in the standalone entry points: pinned to a raster-order
# implementation with a table from the global definition (scipy labelling),
# to the (4,8) topology, and to ultimacy under that table.
_T48 = None


def _table48():
    global _T48
    if _T48 is None:
        _T48 = np.array([tc.global_simple48(m) for m in range(256)], dtype=bool)
    return _T48


@pytest.mark.parametrize("idx", range(4))
def test_homotopic_thin_48(idx):
    S = _images()[idx]
    rng = np.random.default_rng(50 + idx)
    K = ((rng.random(S.shape) < 0.05) & (S != 0)).astype(np.uint8)
    T = oracle.homotopic_thin(S, K, n=4)
    P = tc.edt_brute((S == 0).astype(np.uint8), True)
    assert np.array_equal(T, tc.sequential_schedule(0, S, K, P, table=list(_table48())))
    assert tc.topology48(T) == tc.topology48(S)
    assert ((K != 0) <= (T != 0)).all() and ((T != 0) <= (S != 0)).all()
    assert not (_table48()[tc.neighbourhood_codes(T)] & (T != 0) & (K == 0)).any()


def test_the_pair_matters_for_standalone_thinning():
    diff = sum(int((oracle.homotopic_thin(S, None, n=4) != oracle.homotopic_thin(S)).sum()) for S in _images())
    assert diff > 0


@pytest.mark.parametrize("idx", range(4))
def test_homotopic_thicken_48(idx):
    S = _images()[idx]
    V = tc.dilate_stamp(S, 4).astype(np.uint8)
    U = oracle.homotopic_thicken(S, V, n=4)
    P = tc.edt_brute(S, False)
    assert np.array_equal(U, tc.sequential_schedule(1, S, V, P, table=list(_table48())))
    assert tc.topology48(U) == tc.topology48(S)
    assert ((S != 0) <= (U != 0)).all() and ((U != 0) <= (V != 0) | (S != 0)).all()
    # ultimate: no point of V outside U can be added (simple for U plus it)
    assert not (_table48()[tc.neighbourhood_codes(U)] & (U == 0) & (V != 0)).any()
