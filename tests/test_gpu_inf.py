"""Parity of "r = infinity" (hasf_filter_inf: radii until the first that
leaves the set unchanged, at most the saturation radius) with the oracle, bit
exact, result and stopping radius: the fused per-radius path (radii up to
HASF_R_MAX), the composed path (exact distance maps, ball thresholds and the
standalone thinning and thickening; beyond HASF_R_MAX, or forced), both
connectivity pairs, both orders, with C and D, on one workgroup, on row tiles
and on the grid kernel."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu

# The device radius loop is switched off: its first GPU run (test_inf_random,
# the 33 x 22 image, the fused filter one radius per launch) ended in a device
# memory fault whose cause was not found by reading the code. hasf_filter_inf
# returns HASF_EINTERNAL without device work until it is.
OFF = pytest.mark.skip(reason="device r = infinity switched off: its first GPU run faulted, cause not found")

_CTX = {}


def _c(kind):
    if kind not in _CTX:
        _CTX[kind] = {"tile": lambda: hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1, tile_rows=8),
                      "grid": lambda: hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1,
                                                   tile_rows=-1)}[kind]()
    return _CTX[kind]


def _run(c, X, C=None, D=None, n=8, order=0, r_max=0, composed=False):
    x = dev(X)
    cd = dev(C) if C is not None else None
    dd = dev(D) if D is not None else None
    used = c.filter_inf(x, cd, dd, conn=n, order=order, r_max=r_max, composed=composed)
    return host(x), used


def _case(k):
    rng = np.random.default_rng(6600 + k)
    H, W = int(rng.integers(20, 70)), int(rng.integers(20, 70))
    if k % 3 == 2:
        X = synth.random_binary(H, W, 0.5, 6700 + k)
    else:
        X = synth.draw(H, W, synth._rng(6700 + k), 4, 3, 16, 0.3, n_holes=1, p_flip=0.25, sp_frac=0.03)
    C = ((rng.random((H, W)) < 0.03) & (X != 0)).astype(np.uint8)
    D = ((rng.random((H, W)) < 0.03) & (X == 0)).astype(np.uint8)
    return X, C, D


COMBOS = [(n, order, useC, useD) for n in (8, 4) for order in (0, 1) for useC in (0, 1) for useD in (0, 1)]


@OFF
@pytest.mark.parametrize("composed", [False, True])
@pytest.mark.parametrize("k", range(8))
def test_inf_random(k, composed):
    n, order, useC, useD = COMBOS[2 * k + (1 if composed else 0)]
    X, C, D = _case(k)
    C = C if useC else None
    D = D if useD else None
    exp, eu = oracle.hasf_inf(X, C, D, n=n, order=order)
    say("r = inf", X.shape, (n, order, useC, useD), "composed" if composed else "fused", "stops at", eu)
    got, used = _run(ctx(), X, C, D, n, order, composed=composed)
    assert used == eu
    assert np.array_equal(got, exp)


@OFF
@pytest.mark.parametrize("kind", ["wg", "tile", "grid"])
def test_inf_beyond_the_fused_radii(kind):
    # a square's corners are rounded at every radius up to about half its side
    X = np.zeros((80, 84), np.uint8)
    X[8:72, 10:74] = 1
    X[30:34, 20:60] = 0
    exp, eu = oracle.hasf_inf(X)
    assert eu > hasf.HASF_R_MAX
    say("r = inf on a square with a slot, stops at", eu, kind)
    got, used = _run(ctx() if kind == "wg" else _c(kind), X)
    assert used == eu
    assert np.array_equal(got, exp)


@OFF
def test_inf_workloads():
    X, C, _ = synth.workload_disks()
    exp, eu = oracle.hasf_inf(X, C)
    say("r = inf, 256x256 disks, stops at", eu)
    got, used = _run(ctx(), X, C)
    assert used == eu and np.array_equal(got, exp)
    X, C, _ = synth.workload_shapes()
    exp, eu = oracle.hasf_inf(X, C)
    say("r = inf, 512x512 shapes, stops at", eu)
    got, used = _run(ctx(), X, C)
    assert used == eu and np.array_equal(got, exp)
    say("r = inf, 512x512 shapes on row tiles")
    got, used = _run(_c("tile"), X, C)
    assert used == eu and np.array_equal(got, exp)


@OFF
def test_inf_cap_and_arguments():
    X = np.zeros((60, 64), np.uint8)
    X[5:55, 6:58] = 1
    got, used = _run(ctx(), X, r_max=3)
    assert used == 3 and np.array_equal(got, oracle.hasf(X, None, 3))
    got, used = _run(ctx(), np.zeros((9, 7), np.uint8))
    assert used == 1 and not got.any()
    lib = hasf.lib()
    p = ctypes.c_void_p(0x1000)
    u = ctypes.c_int(0)
    h = ctx()._h
    assert lib.hasf_filter_inf(h, p, None, None, 8, 8, 8, 8, 0, 0, 0, None) == hasf.HASF_EINVAL
    assert lib.hasf_filter_inf(h, p, None, None, 8, 8, 8, 8, 0, -1, 0, ctypes.byref(u)) == hasf.HASF_EINVAL
    assert lib.hasf_filter_inf(h, p, None, None, 8, 8, 8, 8, 0, 0, 2, ctypes.byref(u)) == hasf.HASF_EINVAL
    assert lib.hasf_filter_inf(h, p, None, None, 8, 8, 8, 6, 0, 0, 0, ctypes.byref(u)) == hasf.HASF_EINVAL
    assert lib.hasf_filter_inf(h, p, None, None, 8, 8, 8, 8, 2, 0, 0, ctypes.byref(u)) == hasf.HASF_EINVAL


def test_switched_off_entry_point_does_no_device_work():
    X = np.zeros((30, 40), np.uint8)
    X[5:25, 5:35] = 1
    x = dev(X)
    with pytest.raises(hasf.HasfError) as ei:
        ctx().filter_inf(x)
    assert ei.value.status == hasf.HASF_EINTERNAL
    assert np.array_equal(host(x), X)
