"""Pin of the oracle's wiring of the cutting and the filling (Sec. 2: H deletes
simple points in increasing order of their distance to the background, *H
adds them in increasing order of their distance to the set; eq. (i), eq. (ii)).

The oracle's filter is compared stage by stage, bit for bit, with an
independent composition (tests/topo_checks.py: ball stamping, scipy's exact
distance transform, a numpy subfield schedule). A wrong priority map in any
of the four thinnings and thickenings of a radius, a swapped or constant one,
a wrong threshold or a wrong order of the operators changes some stage of
some of these images."""
import numpy as np
import pytest

import oracle
import topo_checks as tc
from paper_1603_09337_amd import synth


def _case(k):
    """Image k: noisy disks or Bernoulli noise, at most 48 x 48, with a
    constraint set C and a background constraint set D drawn for it."""
    rng = np.random.default_rng(9100 + k)
    H = int(rng.integers(20, 49))
    W = int(rng.integers(20, 49))
    if k % 3 == 2:
        X = synth.random_binary(H, W, 0.5 + 0.02 * (k % 5), 7700 + k)
    else:
        X = synth.draw(H, W, synth._rng(7700 + k), 4, 4, 12, 0.3, n_holes=1, p_flip=0.25, sp_frac=0.03)
    C = ((rng.random((H, W)) < 0.04) & (X != 0)).astype(np.uint8)
    D = ((rng.random((H, W)) < 0.04) & (X == 0)).astype(np.uint8)
    return X, C, D


# every combination of pair, order, C and D, on two images each
COMBOS = [(n, order, useC, useD) for n in (8, 4) for order in (0, 1) for useC in (0, 1) for useD in (0, 1)]


@pytest.mark.parametrize("k", range(32))
def test_stages_equal_independent_composition(k):
    n, order, useC, useD = COMBOS[k % 16]
    X, C, D = _case(k)
    r = 1 + k % 3
    C = C if useC else None
    D = D if useD else None
    out, st = oracle.hasf(X, C, r, stages=True, D=D, n=n, order=order)
    ref = tc.hasf_composed(X, C, D, r, n=n, order=order)
    for i in range(r):
        for s in range(4):
            bad = int((st[i, s] != ref[i, s]).sum())
            assert bad == 0, "radius %d stage %d: %d pixels differ" % (i + 1, s, bad)
    assert np.array_equal(out, ref[-1, 3])


def test_composition_sees_the_order():
    """The composition itself depends on the priority maps: ordering the
    cutting's thinning by a constant instead of the distance to the background
    gives another set on these images (so the stage test above can tell)."""
    table = tc.simple_table(8)
    differs = 0
    for k in range(12):
        X, _, _ = _case(k)
        for i in (1, 2, 3):
            K = tc.erode_stamp(X, i)
            good = tc.schedule_np(0, X, K, tc.edt_sq_lib(X == 0, True), table)
            flat = tc.schedule_np(0, X, K, np.zeros(X.shape, np.uint32), table)
            differs += not np.array_equal(good, flat)
    assert differs >= 6


def test_edt_sq_lib_matches_brute_force():
    for k in range(12):
        F = synth.random_binary(7 + k, 11 + 2 * k, 0.1 + 0.05 * (k % 4), 500 + k)
        for frame in (False, True):
            assert np.array_equal(tc.edt_sq_lib(F, frame), tc.edt_brute(F, frame))
    Z = np.zeros((5, 9), np.uint8)
    assert np.array_equal(tc.edt_sq_lib(Z, False), tc.edt_brute(Z, False))
    assert np.array_equal(tc.edt_sq_lib(Z, True), tc.edt_brute(Z, True))


@pytest.mark.parametrize("mode", [0, 1])
def test_schedule_np_matches_raster_schedule(mode):
    for k in range(6):
        X = synth.random_binary(12 + k, 15 + k, 0.55, 600 + k)
        rng = np.random.default_rng(k)
        B = (rng.random(X.shape) < 0.5).astype(np.uint8)
        P = rng.integers(0, 6, X.shape).astype(np.uint32)
        for n in (8, 4):
            t = tc.simple_table(n)
            assert np.array_equal(tc.schedule_np(mode, X, B, P, t), tc.sequential_schedule(mode, X, B, P, t))


# Inputs on which the order inside a phase decides pixels. On most images the
# cutting's thickening and the filling's thinning reach the same set in any
# order (their limit sets rarely have another topology than the set being
# grown or shrunk); these were found by searching seeded noise for images where
# a constant or reversed priority gives another result.
def _bern_case(k):
    """k-th image of a search over Bernoulli noise (sides U[24, 96))."""
    rng = np.random.default_rng(k)
    H, W = int(rng.integers(24, 96)), int(rng.integers(24, 96))
    return synth.random_binary(H, W, 0.45 + 0.01 * k % 0.2, 100 + k)


def _constrained_case(k):
    """k-th image of a search over noise and noisy shapes (sides U[16, 64))
    with 5 % of the object pixels constrained."""
    rng = np.random.default_rng(k)
    H, W = int(rng.integers(16, 64)), int(rng.integers(16, 64))
    if k % 2:
        X = synth.random_binary(H, W, rng.uniform(0.3, 0.7), 1000 + k)
    else:
        X = synth.draw(H, W, synth._rng(k), 8, 2, 12, 0.5, n_holes=3, p_flip=0.4, sp_frac=0.08)
    C = ((rng.random((H, W)) < 0.05) & (X != 0)).astype(np.uint8)
    return X, C


@pytest.mark.parametrize("k,r", [(4, 3), (24, 5), (28, 3)])
def test_filling_thinning_order_decides(k, r):
    """The filling's thinning (priority: distance to the background of the
    filled set) decides pixels of these images."""
    X = _bern_case(k)
    out, st = oracle.hasf(X, None, r, stages=True)
    ref = tc.hasf_composed(X, None, None, r)
    for i in range(r):
        for s in range(4):
            assert np.array_equal(st[i, s], ref[i, s]), "radius %d stage %d" % (i + 1, s)
    assert np.array_equal(out, ref[-1, 3])


@pytest.mark.parametrize("k,i", [(97, 3), (100, 3), (283, 3), (556, 4)])
def test_cutting_thickening_order_decides(k, i):
    """The cutting's thickening (priority: distance to the thinned set)
    decides pixels of these images: one cutting at radius i, compared with
    the composition, and the same thickening with a constant priority gives
    another set."""
    X, C = _constrained_case(k)
    Y, ref = tc.hc_composed(X, C, i, tc.simple_table(8))
    assert np.array_equal(oracle.hc(X, C, i), ref)
    V = tc.dilate_stamp(Y, i) & (X != 0)
    flat = tc.schedule_np(1, Y, V, np.zeros(X.shape, np.uint32), tc.simple_table(8))
    rev = tc.schedule_np(1, Y, V, (10 ** 6 - np.minimum(tc.edt_sq_lib(Y, False), 10 ** 6)).astype(np.uint32),
                         tc.simple_table(8))
    assert not (np.array_equal(flat, ref) and np.array_equal(rev, ref))
