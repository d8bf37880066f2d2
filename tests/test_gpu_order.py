"""Parity of the dual filter order (hasf_image.order = 1: at every radius the
filling first, then the cutting) with the oracle, bit-exact, on every path:
one workgroup (state in LDS and in global memory), the grid, row tiles,
batches mixing both orders, and the served stream."""
import numpy as np
import pytest

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu

_CTX = {}


def _grid(kind="grid"):
    if kind not in _CTX:
        _CTX[kind] = hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1,
                                  tile_rows=-1 if kind == "grid" else 8)
    return _CTX[kind]


def _background(X, p, seed):
    rng = np.random.default_rng(seed)
    return ((rng.random(X.shape) < p) & (X == 0)).astype(np.uint8)


def _run(c, X, C, D, r, n, pitch=None):
    x = dev(X, pitch)
    cd = dev(C, pitch) if C is not None else None
    dd = dev(D, pitch) if D is not None else None
    c.filter(x, cd, r, D=dd, conn=n, order=1)
    c.sync()
    return host(x)


CASES = [
    # (H, W, density, r, with C, with D, n)
    (1, 90, 0.6, 2, True, False, 8), (77, 1, 0.6, 2, False, True, 4), (37, 130, 0.55, 3, True, False, 8),
    (64, 64, 0.5, 5, False, False, 8), (100, 300, 0.45, 4, True, True, 8), (129, 191, 0.5, 6, True, True, 4),
    (60, 66, 0.5, 12, True, False, 8), (64, 130, 1.0, 3, False, False, 8), (64, 130, 0.0, 3, False, True, 4),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("path", ["default", "grid", "tile"])
def test_dual_order_random(case, path):
    H, W, dens, r, wc, wd, n = case
    X = synth.random_binary(H, W, dens, 2000 + H + W + r)
    C = synth.random_binary(H, W, 0.03, 2100 + H) if wc else None
    D = _background(X, 0.3, 2200 + W) if wd else None
    c = ctx() if path == "default" else _grid(path)
    say("dual order", case, path)
    got = _run(c, X, C, D, r, n)
    assert np.array_equal(got, oracle.hasf(X, C, r, D=D, n=n, order=1))


def test_dual_order_workloads_and_pitch():
    X, C, r = synth.workload_shapes()
    say("dual order 512x512 r=5")
    assert np.array_equal(_run(ctx(), X, C, None, r, 8), oracle.hasf(X, C, r, order=1))
    X, C, r = synth.workload_disks()
    say("dual order 256x256 r=2, pitch 300")
    assert np.array_equal(_run(ctx(), X, C, None, r, 8, pitch=300), oracle.hasf(X, C, r, order=1))


def test_dual_order_global_state():
    # too large for the workgroup's LDS: the state lives in global memory
    X = synth.disks_image(700, 1000, np.random.default_rng(77))
    big = 2**64 - 1
    c = hasf.Context(0, grid_min_pixels=big, batch_grid_min_pixels=big)
    say("dual order 700x1000 r=3, one workgroup, global state")
    assert np.array_equal(_run(c, X, None, None, 3, 8), oracle.hasf(X, None, 3, order=1))


def test_batch_mixes_orders():
    items = []
    for k in range(8):
        X, C, r = synth.batch_item(k, lo=60, hi=300)
        items.append((X, C, r, k % 2))
    say("batch of 8, orders alternating")
    ds = [dev(X) for X, _, _, _ in items]
    cs = [dev(C) if C is not None else None for _, C, _, _ in items]
    ctx().filter_batch([(d, c, r, None, 0, o) for d, c, (_, _, r, o) in zip(ds, cs, items)])
    ctx().sync()
    for k, (d, (X, C, r, o)) in enumerate(zip(ds, items)):
        assert np.array_equal(host(d), oracle.hasf(X, C, r, order=o)), "image %d" % k


def test_served_frames_in_both_orders():
    srv = hasf.Server(ctx(), lanes=2)
    try:
        frames = []
        for k in range(6):
            X = synth.random_binary(90 + 7 * k, 110, 0.5, 2300 + k)
            frames.append((X, 2 + k % 3, k % 2))
        say("served frames, both orders")
        ds = [dev(X) for X, _, _ in frames]
        ts = [srv.submit(d, None, r, order=o) for d, (_, r, o) in zip(ds, frames)]
        for t in ts:
            srv.wait(t)
        for d, (X, r, o) in zip(ds, frames):
            assert np.array_equal(host(d), oracle.hasf(X, None, r, order=o))
    finally:
        srv.stop()


def test_bad_order_is_refused():
    X = synth.random_binary(40, 50, 0.5, 2400)
    d = dev(X)
    for o in (-1, 2):
        with pytest.raises(hasf.HasfError) as e:
            ctx().filter_batch([(d, None, 2, None, 0, o)])
        assert e.value.status == hasf.HASF_EINVAL
    ctx().sync()
    assert np.array_equal(host(d), X)
