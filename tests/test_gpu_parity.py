"""Parity of the HIP path with the oracle, through the C ABI (bit-exact: all
arithmetic is integer and the schedule is deterministic)."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import topo_checks as tc
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = pytest.mark.gpu

U32MAX = np.iinfo(np.uint32).max


def _edt_gpu(F, frame, pitch=None):
    import torch
    out = ctx().edt_sq(dev(F, pitch), frame)
    ctx().sync()
    return host(out).view(np.uint32)


EDT_SHAPES = [(1, 1), (1, 70), (70, 1), (2, 3), (33, 65), (64, 64), (100, 129), (257, 190), (31, 513)]


@pytest.mark.parametrize("shape", EDT_SHAPES)
@pytest.mark.parametrize("frame", [False, True])
def test_edt_random(shape, frame):
    for k, d in enumerate((0.0, 0.003, 0.05, 0.5, 1.0)):
        F = synth.random_binary(shape[0], shape[1], d, 11 + k)
        say("edt", shape, frame, d)
        assert np.array_equal(_edt_gpu(F, frame), oracle.edt_sq(F, frame))


def test_edt_pitch_and_generated_image():
    X, _, _ = synth.workload_shapes()
    for frame in (False, True):
        F = (X == 0).astype(np.uint8) if frame else X
        assert np.array_equal(_edt_gpu(F, frame, pitch=515), oracle.edt_sq(F, frame))


def test_edt_large_workload():
    X, _, _ = synth.workload_large()
    say("edt 4096x4096")
    assert np.array_equal(_edt_gpu(X, False), oracle.edt_sq(X, False))
    B = (X == 0).astype(np.uint8)
    assert np.array_equal(_edt_gpu(B, True), oracle.edt_sq(B, True))


def _filter_gpu(X, C, r, pitch=None):
    Xd = dev(X, pitch)
    Cd = dev(C, pitch) if C is not None else None
    ctx().filter(Xd, Cd, r)
    ctx().sync()
    return host(Xd)


FILTER_CASES = [
    # (H, W, density, r, with C)
    (1, 1, 1.0, 2, False), (1, 90, 0.6, 3, False), (90, 1, 0.6, 3, False), (5, 5, 0.5, 1, True),
    (40, 63, 0.55, 2, True), (47, 64, 0.5, 3, False), (65, 65, 0.45, 4, True), (100, 127, 0.5, 5, False),
    (128, 200, 0.5, 6, True), (33, 300, 0.6, 8, False), (120, 77, 0.5, 0, True), (64, 130, 0.0, 3, False),
    (64, 130, 1.0, 3, False), (70, 90, 0.5, 10, False), (60, 66, 0.5, 15, True),
]


@pytest.mark.parametrize("case", FILTER_CASES)
def test_filter_random(case):
    H, W, d, r, withC = case
    X = synth.random_binary(H, W, d, 1000 + H * 7 + W)
    C = synth.random_binary(H, W, 0.03, 77) if withC else None
    say("filter", case)
    assert np.array_equal(_filter_gpu(X, C, r), oracle.hasf(X, C, r))


@pytest.mark.parametrize("pitch", [None, 301, 320])
def test_filter_pitch(pitch):
    X, _, _ = synth.workload_disks(H=180, W=300)
    C = synth.random_binary(180, 300, 0.02, 5)
    say("filter pitch", pitch)
    assert np.array_equal(_filter_gpu(X, C, 4, pitch), oracle.hasf(X, C, 4))


def test_filter_disks_workload():
    X, C, r = synth.workload_disks()
    say("filter 256x256 r=2")
    assert np.array_equal(_filter_gpu(X, C, r), oracle.hasf(X, C, r))


def test_filter_shapes_workload_and_each_radius():
    X, C, r = synth.workload_shapes()
    exp, stages = oracle.hasf(X, C, r, stages=True)
    for i in range(1, r + 1):
        say("filter 512x512 r=%d" % i)
        assert np.array_equal(_filter_gpu(X, C, i), stages[i - 1, 3]), "radius %d" % i
    got = _filter_gpu(X, C, r)
    assert np.array_equal(got, exp)
    assert tc.topology(got) == tc.topology(X)


def test_filter_large_image_global_planes():
    # does not fit in LDS: the planes live in global memory (one workgroup;
    # by default an image this large goes to row tiles)
    from paper_1603_09337_amd import hasf
    X, _, _ = synth.workload_disks(H=700, W=1000)
    say("filter 700x1000 r=3, one workgroup, state in global memory")
    wg = hasf.Context(0, grid_min_pixels=2**64 - 1)
    d = dev(X)
    wg.filter(d, None, 3)
    wg.sync()
    assert np.array_equal(host(d), oracle.hasf(X, None, 3))
    say("filter 700x1000 r=3, default")
    assert np.array_equal(_filter_gpu(X, None, 3), oracle.hasf(X, None, 3))


def test_filter_4096_r10_matches_oracle_digest():
    # full size: the oracle's result (about four minutes on one core) is stored
    # as a digest by tests/golden/make_large_digest.py
    gold = json.load(open(os.path.join(GOLDEN, "hasf_4096x4096_r10.json")))
    X, C, r = synth.workload_large()
    assert hashlib.sha256(X.tobytes()).hexdigest() == gold["input_sha256"]
    d = dev(X)
    say("filter 4096x4096 r=10")
    ctx().filter(d, None, r)
    ctx().sync()
    Y = host(d)
    assert int(Y.sum()) == gold["ones"]
    assert hashlib.sha256(np.ascontiguousarray(Y).tobytes()).hexdigest() == gold["sha256"]


def test_batch_uneven_images():
    items = [synth.batch_item(k, lo=40, hi=400) for k in range(24)]
    dX = [dev(X) for X, _, _ in items]
    say("batch 24 images")
    ctx().filter_batch([(d, None, r) for d, (_, _, r) in zip(dX, items)])
    ctx().sync()
    for k, ((X, C, r), d) in enumerate(zip(items, dX)):
        assert np.array_equal(host(d), oracle.hasf(X, C, r)), "image %d" % k


def test_batch_equals_single_and_handles_mixed_radii_and_constraints():
    rng = np.random.default_rng(3)
    imgs = []
    for k in range(10):
        H, W = int(rng.integers(20, 200)), int(rng.integers(20, 200))
        X = synth.random_binary(H, W, 0.5, 500 + k)
        C = synth.random_binary(H, W, 0.05, 600 + k) if k % 2 else None
        imgs.append((X, C, int(rng.integers(0, 7))))
    dX = [dev(X) for X, _, _ in imgs]
    dC = [dev(C) if C is not None else None for _, C, _ in imgs]
    say("batch mixed")
    ctx().filter_batch([(x, c, r) for x, c, (_, _, r) in zip(dX, dC, imgs)])
    ctx().sync()
    for (X, C, r), x in zip(imgs, dX):
        single = _filter_gpu(X, C, r)
        assert np.array_equal(host(x), single)
        assert np.array_equal(single, oracle.hasf(X, C, r))


TOPO_SHAPES = [(1, 5), (9, 1), (16, 16), (40, 65), (63, 64), (100, 70)]


@pytest.mark.parametrize("shape", TOPO_SHAPES)
def test_homotopic_thin(shape):
    H, W = shape
    X = synth.random_binary(H, W, 0.6, 40 + H + W)
    K = synth.random_binary(H, W, 0.04, 41)
    for KK in (None, K):
        Xd = dev(X)
        ctx().homotopic_thin(Xd, dev(KK) if KK is not None else None)
        ctx().sync()
        say("thin", shape, KK is not None)
        assert np.array_equal(host(Xd), oracle.homotopic_thin(X, KK))


@pytest.mark.parametrize("shape", TOPO_SHAPES)
def test_homotopic_thicken(shape):
    H, W = shape
    Y = synth.random_binary(H, W, 0.2, 60 + H + W)
    V = synth.random_binary(H, W, 0.7, 61)
    Yd = dev(Y)
    ctx().homotopic_thicken(Yd, dev(V))
    ctx().sync()
    say("thicken", shape)
    assert np.array_equal(host(Yd), oracle.homotopic_thicken(Y, V))


def test_homotopic_thin_generated_image():
    X, _, _ = synth.workload_disks(H=256, W=200)
    Xd = dev(X)
    ctx().homotopic_thin(Xd, None)
    ctx().sync()
    assert np.array_equal(host(Xd), oracle.homotopic_thin(X, None))


def test_thicken_empty_set_adds_nothing():
    Y = np.zeros((30, 40), np.uint8)
    V = np.ones((30, 40), np.uint8)
    Yd = dev(Y)
    ctx().homotopic_thicken(Yd, dev(V))
    ctx().sync()
    assert not host(Yd).any()


# H + W at the limit (65535): the widest rows take the uint16 row pass of the
# EDT and 1024-word rows in the filter; the tallest columns take 2048 segments
EXTREME_SHAPES = [(1, 65534), (65534, 1), (3, 65532), (65532, 3)]


@pytest.mark.parametrize("shape", EXTREME_SHAPES)
def test_edt_extreme_shapes(shape):
    for k, d in enumerate((0.0, 0.0005, 0.3)):
        F = synth.random_binary(shape[0], shape[1], d, 71 + k)
        say("edt extreme", shape, d)
        for frame in (False, True):
            assert np.array_equal(_edt_gpu(F, frame), oracle.edt_sq(F, frame)), (shape, d, frame)


@pytest.mark.parametrize("shape", EXTREME_SHAPES)
def test_filter_extreme_shapes(shape):
    X = synth.random_binary(shape[0], shape[1], 0.55, 81)
    C = synth.random_binary(shape[0], shape[1], 0.02, 82)
    say("filter extreme", shape)
    assert np.array_equal(_filter_gpu(X, C, 3), oracle.hasf(X, C, 3))


def test_thicken_from_one_pixel_over_a_long_row():
    # priorities up to 15999^2: the distinct-value ranking spans a 256 M range
    Y = np.zeros((1, 16000), np.uint8)
    Y[0, 0] = 1
    V = np.ones((1, 16000), np.uint8)
    Yd = dev(Y)
    say("thicken 1x16000 from one pixel")
    ctx().homotopic_thicken(Yd, dev(V))
    ctx().sync()
    assert np.array_equal(host(Yd), oracle.homotopic_thicken(Y, V))


def test_grid_extreme_shapes():
    from test_gpu_grid import grid_ctx
    for shape in [(3, 65532), (65532, 3)]:
        X = synth.random_binary(shape[0], shape[1], 0.55, 91)
        d = dev(X)
        say("grid extreme", shape)
        grid_ctx().filter(d, None, 3)
        grid_ctx().sync()
        assert np.array_equal(host(d), oracle.hasf(X, None, 3)), shape
