"""The radius limit: r = HASF_R_MAX is filtered bit-exactly on the
single-workgroup and the grid path and in a batch; r outside [0, HASF_R_MAX]
is refused before any device work and leaves the image untouched."""
import numpy as np
import pytest

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu

_GRID = {}


def grid_ctx(kind="grid"):
    if kind not in _GRID:
        _GRID[kind] = hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1,
                                   tile_rows=-1 if kind == "grid" else 8)
    return _GRID[kind]


def _img(H, W, seed):
    return synth.disks_image(H, W, np.random.default_rng(seed))


@pytest.mark.parametrize("path", ["wg", "grid", "tile"])
def test_max_radius(path):
    X = _img(120, 150, 31)
    C = synth.random_binary(120, 150, 0.02, 32)
    c = grid_ctx(path) if path != "wg" else ctx()
    say("r = HASF_R_MAX", path)
    d = dev(X)
    c.filter(d, dev(C), hasf.HASF_R_MAX)
    c.sync()
    assert np.array_equal(host(d), oracle.hasf(X, C, hasf.HASF_R_MAX))


def test_max_radius_in_a_batch():
    items = [(_img(90, 70, 41), None, 0), (_img(100, 130, 42), None, hasf.HASF_R_MAX),
             (_img(64, 200, 43), None, 7)]
    say("batch with r = 0, HASF_R_MAX, 7")
    ds = [dev(X) for X, _, _ in items]
    ctx().filter_batch([(d, None, r) for d, (_, _, r) in zip(ds, items)])
    ctx().sync()
    for d, (X, C, r) in zip(ds, items):
        assert np.array_equal(host(d), oracle.hasf(X, C, r))


@pytest.mark.parametrize("r", [-1, hasf.HASF_R_MAX + 1, 1000])
def test_radius_out_of_range_is_refused(r):
    X = _img(50, 60, 51)
    d = dev(X)
    say("refused r =", r)
    with pytest.raises(hasf.HasfError) as e:
        ctx().filter(d, None, r)
    assert e.value.status == hasf.HASF_EINVAL
    with pytest.raises(hasf.HasfError) as e:
        ctx().filter_batch([(dev(X), None, 2), (d, None, r)])
    assert e.value.status == hasf.HASF_EINVAL
    ctx().sync()
    assert np.array_equal(host(d), X)


def test_batch_larger_than_the_device_uses_smaller_workgroups():
    # more images than CUs: 512-thread workgroups, two per CU; fewer: 1024
    # threads per image. Both must give the oracle's result.
    rng = np.random.default_rng(61)
    items = []
    for k in range(300):
        H, W = int(rng.integers(20, 70)), int(rng.integers(20, 70))
        items.append((synth.random_binary(H, W, 0.5, 6100 + k), None, int(rng.integers(0, 4))))
    say("batch of 300 small images")
    ds = [dev(X) for X, _, _ in items]
    ctx().filter_batch([(d, None, r) for d, (_, _, r) in zip(ds, items)])
    ctx().sync()
    for k, (d, (X, C, r)) in enumerate(zip(ds, items)):
        assert np.array_equal(host(d), oracle.hasf(X, C, r)), "image %d" % k
    say("the first 40 of them as their own batch")
    ds = [dev(X) for X, _, _ in items[:40]]
    ctx().filter_batch([(d, None, r) for d, (_, _, r) in zip(ds, items[:40])])
    ctx().sync()
    for k, (d, (X, C, r)) in enumerate(zip(ds, items[:40])):
        assert np.array_equal(host(d), oracle.hasf(X, C, r)), "image %d" % k
