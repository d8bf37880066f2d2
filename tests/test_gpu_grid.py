"""Parity of the grid path (one image filtered by a grid of workgroups, state
in global memory, grid-wide barriers) with the oracle, bit-exact. A context
with grid_min_pixels = 1 sends every image down the grid path, so small,
ragged and degenerate images check it at sizes the oracle finishes quickly;
a context with grid_min_pixels = SIZE_MAX keeps large images on one
workgroup, so both paths stay covered at the same sizes."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu

_CTX = {}


def grid_ctx():
    if "grid" not in _CTX:
        _CTX["grid"] = hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1, tile_rows=-1)
    return _CTX["grid"]


def wg_ctx():
    if "wg" not in _CTX:
        _CTX["wg"] = hasf.Context(0, grid_min_pixels=2**64 - 1, batch_grid_min_pixels=2**64 - 1)
    return _CTX["wg"]


def _filter(c, X, C, r, pitch=None):
    d = dev(X, pitch)
    cd = dev(C, pitch) if C is not None else None
    c.filter(d, cd, r)
    c.sync()
    return host(d)


GRID_CASES = [
    # (H, W, r, density, with C, seed)
    (1, 90, 2, 0.6, False, 1),
    (77, 1, 2, 0.6, False, 2),
    (2, 2, 1, 1.0, False, 3),
    (37, 130, 3, 0.55, True, 4),
    (64, 64, 5, 0.5, False, 5),
    (100, 300, 4, 0.45, True, 6),
    (257, 65, 6, 0.5, False, 7),
    (129, 191, 8, 0.5, True, 8),
]


@pytest.mark.parametrize("case", GRID_CASES)
def test_grid_random(case):
    H, W, r, dens, withC, seed = case
    X = synth.random_binary(H, W, dens, 900 + seed)
    C = synth.random_binary(H, W, 0.05, 950 + seed) if withC else None
    say("grid random", case)
    assert np.array_equal(_filter(grid_ctx(), X, C, r), oracle.hasf(X, C, r))


def test_grid_disks_and_shapes_workloads():
    X, C, r = synth.workload_disks()
    say("grid 256x256 r=2")
    assert np.array_equal(_filter(grid_ctx(), X, C, r), oracle.hasf(X, C, r))
    X, C, r = synth.workload_shapes()
    say("grid 512x512 r=5")
    assert np.array_equal(_filter(grid_ctx(), X, C, r), oracle.hasf(X, C, r))


def test_grid_pitch_and_r0_and_empty_and_full():
    X = synth.disks_image(90, 140, np.random.default_rng(3))
    say("grid pitch")
    assert np.array_equal(_filter(grid_ctx(), X, None, 3, pitch=201), oracle.hasf(X, None, 3))
    assert np.array_equal(_filter(grid_ctx(), X, None, 0), (X != 0).astype(np.uint8))
    Z = np.zeros((70, 80), np.uint8)
    assert np.array_equal(_filter(grid_ctx(), Z, None, 4), Z)
    F = np.ones((70, 80), np.uint8)
    assert np.array_equal(_filter(grid_ctx(), F, None, 4), oracle.hasf(F, None, 4))


def test_grid_and_single_workgroup_agree_on_a_large_image():
    X, _, _ = synth.workload_disks(H=700, W=1000)
    say("700x1000 r=3 grid and one workgroup")
    exp = oracle.hasf(X, None, 3)
    assert np.array_equal(_filter(grid_ctx(), X, None, 3), exp)
    assert np.array_equal(_filter(wg_ctx(), X, None, 3), exp)


def test_batch_with_grid_and_workgroup_images():
    c = hasf.Context(0, batch_grid_min_pixels=60000)
    items = [synth.batch_item(k, lo=60, hi=420) for k in range(10)]
    dX = [dev(X) for X, _, _ in items]
    say("batch, grid and workgroup images:", sum(X.size >= 60000 for X, _, _ in items), "on the grid")
    c.filter_batch([(d, None, r) for d, (_, _, r) in zip(dX, items)])
    c.sync()
    for k, ((X, C, r), d) in enumerate(zip(items, dX)):
        assert np.array_equal(host(d), oracle.hasf(X, C, r)), "image %d" % k
