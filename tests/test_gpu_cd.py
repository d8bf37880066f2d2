"""Parity of HASF^{C,D} and the (4,8) connectivity pair (hasf_filter_cd and
the D / conn fields of hasf_image) with the oracle, bit-exact, on every path:
one workgroup (state in LDS and in global memory), the grid, row tiles,
batches and the served stream."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu

_CTX = {}


def _c(kind):
    if kind not in _CTX:
        big = 2**64 - 1
        _CTX[kind] = {"grid": lambda: hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1, tile_rows=-1),
                      "tile": lambda: hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1, tile_rows=8),
                      "wg": lambda: hasf.Context(0, grid_min_pixels=big, batch_grid_min_pixels=big)}[kind]()
    return _CTX[kind]


def _background(X, p, seed):
    rng = np.random.default_rng(seed)
    return ((rng.random(X.shape) < p) & (X == 0)).astype(np.uint8)


def _run(c, X, C, D, r, n, pitch=None):
    x = dev(X, pitch)
    cd = dev(C, pitch) if C is not None else None
    dd = dev(D, pitch) if D is not None else None
    c.filter(x, cd, r, D=dd, conn=n)
    c.sync()
    return host(x)


CASES = [
    # (H, W, density, r, with C, with D, n)
    (1, 90, 0.6, 2, False, True, 4), (90, 1, 0.6, 2, True, True, 4), (40, 63, 0.55, 2, True, False, 4),
    (65, 65, 0.45, 4, True, True, 4), (100, 127, 0.5, 5, False, True, 4), (128, 200, 0.5, 6, True, True, 4),
    (47, 64, 0.5, 3, False, True, 8), (100, 127, 0.5, 5, True, True, 8), (60, 66, 0.5, 12, True, True, 4),
    (64, 130, 1.0, 3, False, True, 4), (64, 130, 0.0, 3, False, True, 4),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("path", ["default", "grid", "tile"])
def test_cd_random(case, path):
    H, W, dens, r, wc, wd, n = case
    X = synth.random_binary(H, W, dens, 1000 + H + W + r)
    C = synth.random_binary(H, W, 0.03, 1100 + H) if wc else None
    D = _background(X, 0.3, 1200 + W) if wd else None
    c = ctx() if path == "default" else _c(path)
    say("cd", case, path)
    assert np.array_equal(_run(c, X, C, D, r, n), oracle.hasf(X, C, r, D=D, n=n))


def test_cd_shapes_workload_and_global_state():
    X, C, r = synth.workload_shapes()
    D = _background(X, 0.1, 5)
    say("cd 512x512 r=5, (4,8) and D")
    exp = oracle.hasf(X, C, r, D=D, n=4)
    assert np.array_equal(_run(ctx(), X, C, D, r, 4, pitch=530), exp)
    Xg, _, _ = synth.workload_disks(H=700, W=1000)
    Dg = _background(Xg, 0.05, 6)
    say("cd 700x1000 r=3, one workgroup (global state) and grid")
    expg = oracle.hasf(Xg, None, 3, D=Dg, n=4)
    assert np.array_equal(_run(_c("wg"), Xg, None, Dg, 3, 4), expg)
    assert np.array_equal(_run(_c("grid"), Xg, None, Dg, 3, 4), expg)
    assert np.array_equal(_run(_c("tile"), Xg, None, Dg, 3, 4), expg)


def test_cd_batch_and_stream_mix_pairs_and_constraints():
    items = []
    for k in range(12):
        X, _, r = synth.batch_item(k, lo=40, hi=260)
        D = _background(X, 0.2, 1300 + k) if k % 2 else None
        items.append((X, None, r, D, 4 if k % 3 else 8))
    dX = [dev(X) for X, _, _, _, _ in items]
    dD = [dev(D) if D is not None else None for _, _, _, D, _ in items]
    say("cd batch of 12")
    ctx().filter_batch([(x, None, r, d, n) for x, d, (_, _, r, _, n) in zip(dX, dD, items)])
    ctx().sync()
    exp = [oracle.hasf(X, None, r, D=D, n=n) for X, _, r, D, n in items]
    for k, (x, e) in enumerate(zip(dX, exp)):
        assert np.array_equal(host(x), e), "batch image %d" % k
    sX = [dev(X) for X, _, _, _, _ in items]
    torch.cuda.synchronize()
    srv = hasf.Server(ctx(), pool_bytes=128 << 20)
    say("cd stream of 12")
    tickets = [srv.submit(x, None, r, D=d, conn=n) for x, d, (_, _, r, _, n) in zip(sX, dD, items)]
    assert all(srv.wait(t, 60000) is not None for t in tickets)
    srv.stop()
    for k, (x, e) in enumerate(zip(sX, exp)):
        assert np.array_equal(host(x), e), "stream frame %d" % k


def test_cd_rejects_bad_connectivity():
    x = dev(np.zeros((8, 8), np.uint8))
    with pytest.raises(hasf.HasfError) as e:
        ctx().filter(x, None, 1, conn=6)
    assert e.value.status == hasf.HASF_EINVAL
