"""Parity of the 3D filter ((26,6) connectivity, hasf_filter3 and
hasf_filter3_batch) with the 3D oracle, bit-exact: random and degenerate
volumes, noisy balls with cavities, constraint sets, every radius up to 4,
batches of uneven volumes in one launch, r = 0, empty and full boxes, and
argument errors before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import topo3_checks as t3
from gpu_util import ctx, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu


def _vol(V):
    return torch.from_numpy(np.ascontiguousarray(V, dtype=np.uint8)).to("cuda:0")


def _run(V, C, r):
    x = _vol(V)
    ctx().filter3(x, _vol(C) if C is not None else None, r)
    ctx().sync()
    return x.cpu().numpy()


def balls(D, H, W, seed, n=5):
    return synth.balls_volume(D, H, W, seed, n=n, noise=0.03)


CASES = [
    # (D, H, W, r, density or None for balls, with C, seed)
    (1, 1, 40, 2, 0.6, False, 1),
    (30, 1, 1, 2, 0.6, False, 2),
    (1, 20, 25, 2, 0.5, True, 3),
    (5, 6, 7, 1, 0.5, False, 4),
    (9, 8, 11, 2, 0.55, True, 5),
    (12, 13, 14, 3, None, True, 6),
    (16, 16, 16, 4, None, False, 7),
    (10, 21, 17, 3, 0.45, False, 8),
    (32, 28, 36, 4, None, True, 10),
]


@pytest.mark.parametrize("case", CASES)
def test_vol_random_and_balls(case):
    D, H, W, r, dens, withC, seed = case
    rng = np.random.default_rng(seed)
    V = (rng.random((D, H, W)) < dens).astype(np.uint8) if dens is not None else balls(D, H, W, seed)
    C = ((rng.random(V.shape) < 0.05) & (V != 0)).astype(np.uint8) if withC else None
    say("3D", case)
    got = _run(V, C, r)
    assert np.array_equal(got, oracle.hasf3(V, C, r))
    assert t3.topology3(got) == t3.topology3(V)


def test_vol_batch_of_uneven_volumes_in_one_launch():
    rng = np.random.default_rng(9)
    items, vols = [], []
    for k in range(12):
        D, H, W = (int(v) for v in rng.integers(4, 15, 3))
        V = balls(D, H, W, 100 + k, n=3)
        C = ((rng.random(V.shape) < 0.04) & (V != 0)).astype(np.uint8) if k % 2 else None
        r = int(rng.integers(0, 4))
        vols.append((V, C, r))
        items.append((_vol(V), _vol(C) if C is not None else None, r))
    say("3D batch of 12 volumes")
    ctx().filter3_batch(items)
    ctx().sync()
    for k, ((V, C, r), (x, _, _)) in enumerate(zip(vols, items)):
        assert np.array_equal(x.cpu().numpy(), oracle.hasf3(V, C, r)), k


def test_vol_r0_empty_full():
    V = balls(8, 9, 10, 4)
    assert np.array_equal(_run(V, None, 0), (V != 0).astype(np.uint8))
    Z = np.zeros((6, 7, 8), np.uint8)
    assert np.array_equal(_run(Z, None, 3), Z)
    F = np.ones((6, 7, 8), np.uint8)
    assert np.array_equal(_run(F, None, 2), oracle.hasf3(F, None, 2))


def test_vol_arguments():
    lib = hasf.lib()
    h = ctx()._h
    p = ctypes.c_void_p(0x1000)
    assert lib.hasf_filter3(h, p, None, 0, 4, 4, 1) == hasf.HASF_EINVAL
    assert lib.hasf_filter3(h, p, None, 4, 4, 4, hasf.HASF_R_MAX + 1) == hasf.HASF_EINVAL
    assert lib.hasf_filter3(h, None, None, 4, 4, 4, 1) == hasf.HASF_EINVAL
    assert lib.hasf_filter3(h, p, None, 2048, 2048, 1024, 1) == hasf.HASF_EINVAL
    assert lib.hasf_filter3(None, p, None, 4, 4, 4, 1) == hasf.HASF_EINVAL
