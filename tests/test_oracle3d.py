"""Pins of the 3D oracle ((26,6) connectivity; Sec. 1 and Sec. 4.1 extend the
method to 3D images, Sec. 2 gives the operators):
- the simple-voxel test against the global definition (removing the voxel
  leaves the numbers of object and background components and the Euler
  characteristic unchanged), on random and special neighbourhoods;
- the 3D squared EDT against brute force;
- thinning and thickening against a raster-order schedule that uses the global
  definition, and topology kept;
- the filter: topology at every stage, the bounds of each cutting and filling
  by ball stamping, smooth balls fixed, r = 0 and empty volumes."""
import numpy as np
import pytest

import oracle
import topo3_checks as t3
from paper_1603_09337_amd import synth


def test_simple_test_matches_the_global_definition():
    rng = np.random.default_rng(33)
    codes = [0, (1 << 26) - 1, 1 << 12, (1 << 12) | (1 << 13), 1 << 0]
    for dens in (0.1, 0.3, 0.5, 0.7, 0.9):
        codes += [int(sum(1 << b for b in range(26) if rng.random() < dens)) for _ in range(250)]
    n_simple = 0
    for c in codes:
        s = t3.simple_by_topology(c)
        n_simple += s
        assert oracle.simple3(c) == s, hex(c)
    assert 0.1 * len(codes) < n_simple < 0.9 * len(codes)


def test_topological_numbers_special_cases():
    assert oracle.topo_numbers3(0) == (0, 1)              # isolated voxel
    assert oracle.topo_numbers3((1 << 26) - 1) == (1, 0)  # interior voxel
    # two opposite face neighbours only: two object components
    up, down = t3.OFF26.index((-1, 0, 0)), t3.OFF26.index((1, 0, 0))
    assert oracle.topo_numbers3((1 << up) | (1 << down))[0] == 2
    # a single neighbour: an end voxel, simple
    assert oracle.simple3(1 << up)


@pytest.mark.parametrize("frame", [False, True])
def test_edt3_matches_brute_force(frame):
    rng = np.random.default_rng(5 + frame)
    for k in range(12):
        shape = tuple(int(v) for v in rng.integers(1, 9, 3))
        F = (rng.random(shape) < (0.02, 0.1, 0.4)[k % 3]).astype(np.uint8)
        assert np.array_equal(oracle.edt_sq3(F, frame), t3.edt3_brute(F, frame)), (shape, k)
    Z = np.zeros((3, 4, 5), np.uint8)
    assert np.array_equal(oracle.edt_sq3(Z, False), np.full(Z.shape, 2**32 - 1, np.uint32))


@pytest.mark.parametrize("mode", [0, 1])
def test_schedule3_matches_raster_order_with_the_global_definition(mode):
    rng = np.random.default_rng(40 + mode)
    for k in range(5):
        shape = tuple(int(v) for v in rng.integers(3, 7, 3))
        S = (rng.random(shape) < 0.55).astype(np.uint8)
        B = (rng.random(shape) < 0.5).astype(np.uint8)
        P = rng.integers(0, 5, shape).astype(np.uint32)
        got = oracle.schedule3(mode, S, B, P)
        ref = t3.schedule3_raster(mode, S, B, P, t3.simple_by_topology)
        assert np.array_equal(got, ref), (mode, k)
        assert t3.topology3(got) == t3.topology3(S)


def _volume(D, H, W, seed, n=5):
    """Noisy balls with a few cavities: the 3D analogue of the disks recipe."""
    rng = np.random.default_rng(seed)
    zz, yy, xx = np.mgrid[0:D, 0:H, 0:W]
    V = np.zeros((D, H, W), bool)
    for k in range(n):
        c = rng.uniform(0, (D, H, W))
        R = rng.uniform(1.5, max(2.5, 0.35 * min(D, H, W)))
        ball = (zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2 <= R * R
        if k % 3 == 2:
            ball &= (zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2 > (0.45 * R) ** 2
        V |= ball
    flip = rng.random(V.shape) < 0.03
    return (V ^ flip).astype(np.uint8)


def test_hasf3_keeps_topology_and_bounds_at_every_stage():
    for seed in range(3):
        X = _volume(14, 15, 16, 70 + seed)
        C = ((np.random.default_rng(seed).random(X.shape) < 0.03) & (X != 0)).astype(np.uint8)
        r = 2
        out, st = oracle.hasf3(X, C, r, stages=True)
        topo = t3.topology3(X)
        prev = X != 0
        for i in range(r):
            thinned, cut, filled_t, filled = (st[i, s] != 0 for s in range(4))
            for s in range(4):
                assert t3.topology3(st[i, s]) == topo, (seed, i, s)
            # HC_i(X) between eps_i(X) u C and X; HF_i between X and delta_i(X)
            assert (cut <= prev).all()
            assert ((t3.erode3(prev, i + 1) | (C != 0)) <= cut).all()
            assert (cut <= filled).all()
            assert (filled <= t3.dilate3(cut, i + 1)).all()
            prev = filled
        assert ((C != 0) <= (out != 0)).all()


def test_hasf3_fixes_smooth_balls_and_r0_and_empty():
    D = 23
    zz, yy, xx = np.mgrid[0:D, 0:D, 0:D]
    checked = 0
    for R in (4, 5, 6, 8):
        B = ((zz - 11) ** 2 + (yy - 11) ** 2 + (xx - 11) ** 2 <= R * R)
        for r in (1, 2):
            # only balls that the classical opening and closing by B_i leave
            # unchanged for every i <= r are asserted fixed (4, 5 and 8 at r = 1)
            fixed = all(np.array_equal(t3.dilate3(t3.erode3(B, i), i), B) and
                        np.array_equal(t3.erode3(t3.dilate3(B, i), i), B) for i in range(1, r + 1))
            if fixed:
                checked += 1
                assert np.array_equal(oracle.hasf3(B.astype(np.uint8), None, r), B.astype(np.uint8)), (R, r)
    assert checked == 3
    X = _volume(8, 9, 10, 3)
    assert np.array_equal(oracle.hasf3(X, None, 0), (X != 0).astype(np.uint8))
    Z = np.zeros((6, 7, 8), np.uint8)
    assert np.array_equal(oracle.hasf3(Z, None, 2), Z)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_hasf3_stages_equal_an_independent_composition(seed):
    # which distance map orders each of the four thinnings and thickenings
    X = _volume(7, 8, 9, 300 + seed, n=3)
    C = ((np.random.default_rng(seed).random(X.shape) < 0.05) & (X != 0)).astype(np.uint8)
    out, st = oracle.hasf3(X, C, 2, stages=True)
    ref = t3.hasf3_composed(X, C, 2)
    for i in range(2):
        for s in range(4):
            assert np.array_equal(st[i, s], ref[i, s]), (seed, i, s)
