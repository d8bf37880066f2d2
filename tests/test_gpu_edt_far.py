"""Parity of the exact squared EDT on inputs whose features are far from most
pixels: few features, empty columns, features only at one edge, with and
without the frame. These strips go to the envelope row pass (the windowed
search would cost each pixel about its distance to the nearest feature), and
images whose features lie in at most 32 columns to its direct minimum over
those columns (both sides of that threshold are checked); the rest of the
image keeps the windowed search, so images that mix both are checked too. Bit-exact against the oracle's transform; the sparse 4096^2
case is also timed against the dense workload."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import synth

pytestmark = pytest.mark.gpu


def _edt(F, frame, pitch=None):
    out = ctx().edt_sq(dev(F, pitch), frame)
    ctx().sync()
    return host(out).view(np.uint32)


def _sparse(H, W, n, seed):
    rng = np.random.default_rng(seed)
    F = np.zeros((H, W), np.uint8)
    F[rng.integers(0, H, n), rng.integers(0, W, n)] = 1
    return F


@pytest.mark.parametrize("shape", [(37, 300), (300, 37), (64, 2049), (513, 700), (1000, 1000), (96, 16384),
                                   (40, 16385), (3, 20000)])
@pytest.mark.parametrize("frame", [False, True])
def test_edt_sparse(shape, frame):
    H, W = shape
    for n in (1, 3, 17):
        F = _sparse(H, W, n, H * 7 + W + n)
        say("edt sparse", shape, n, "frame" if frame else "")
        assert np.array_equal(_edt(F, frame), oracle.edt_sq(F, frame)), (shape, n)


@pytest.mark.parametrize("ncols", [31, 32, 33, 64])
@pytest.mark.parametrize("frame", [False, True])
def test_edt_rows_with_few_feature_columns(ncols, frame):
    # every row of a far strip has exactly ncols columns with a feature: up to
    # 32 the row takes the direct minimum over them, beyond it the envelope
    rng = np.random.default_rng(600 + ncols)
    F = np.zeros((600, 2000), np.uint8)
    cols = rng.choice(2000, ncols, replace=False)
    F[rng.integers(0, 600, ncols), cols] = 1
    F[rng.integers(0, 600, ncols), cols] = 1  # a second feature in some columns
    say("edt few feature columns", ncols, "frame" if frame else "")
    assert np.array_equal(_edt(F, frame), oracle.edt_sq(F, frame))


@pytest.mark.parametrize("frame", [False, True])
def test_edt_far_edges_and_mixed_strips(frame):
    # features only on the top row: every column has one, far from most rows
    F = np.zeros((700, 900), np.uint8)
    F[0, :] = 1
    assert np.array_equal(_edt(F, frame), oracle.edt_sq(F, frame))
    # a dense band (near strips) above an empty band (far strips)
    G = synth.random_binary(800, 640, 0.3, 5)
    G[300:, :] = 0
    G[700, 17] = 1
    assert np.array_equal(_edt(G, frame), oracle.edt_sq(G, frame))
    assert np.array_equal(_edt(G, frame, pitch=700), oracle.edt_sq(G, frame))
    # ties between columns at equal distance
    T = np.zeros((300, 400), np.uint8)
    T[150, ::37] = 1
    T[10, 200] = 1
    assert np.array_equal(_edt(T, frame), oracle.edt_sq(T, frame))


@pytest.mark.parametrize("frame", [False, True])
def test_edt_random_low_densities(frame):
    # every column has features but far apart (long runs of distinct column
    # distances: large hulls with many vertices removed in the merges), and
    # the empty image (no feature at all: only the frame, or nothing)
    for dens, seed in ((0.001, 1), (0.005, 2), (0.02, 3)):
        F = synth.random_binary(1024, 1500, dens, 300 + seed)
        say("edt random density", dens, "frame" if frame else "")
        assert np.array_equal(_edt(F, frame), oracle.edt_sq(F, frame)), dens
    Z = np.zeros((300, 1100), np.uint8)
    assert np.array_equal(_edt(Z, frame), oracle.edt_sq(Z, frame))
    # one feature row in the middle: constant column distances on most rows
    R = np.zeros((900, 700), np.uint8)
    R[450, :] = 1
    R[450, 300:340] = 0
    assert np.array_equal(_edt(R, frame), oracle.edt_sq(R, frame))


def test_edt_sparse_4096_parity_and_timing():
    X, _, _ = synth.workload_large()
    S = _sparse(4096, 4096, 16, 4096)
    say("edt 4096^2: 16 features, no frame, against the oracle")
    assert np.array_equal(_edt(S, False), oracle.edt_sq(S, False))
    xd, sd = dev(X), dev(S)
    out = torch.empty((4096, 4096), dtype=torch.int32, device="cuda")

    def t(x, frame):
        for _ in range(3):
            ctx().edt_sq(x, frame, out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            ctx().edt_sq(x, frame, out)
        e1.record()
        ctx().sync()
        return e0.elapsed_time(e1) / 10

    dense, sparse, sparse_f = t(xd, True), t(sd, False), t(sd, True)
    say("edt 4096^2 ms: dense %.4f, sparse %.4f, sparse with frame %.4f" % (dense, sparse, sparse_f))
    # 16 features lie in at most 16 columns: every row takes the direct
    # minimum over those columns, linear in the row length, so the sparse
    # image costs less than twice the dense one on MI355X (not the sum of
    # its pixels' distances, thousands of times the dense cost); the bound
    # leaves room for a busy device
    assert sparse < 4 * dense and sparse_f < 4 * dense


@pytest.mark.parametrize("case", ["density 0.001", "2000 features, frame", "empty right quarter",
                                  "empty band of 96 columns"])
def test_edt_4096_scattered_features(case):
    # scattered features: every column holds some, so the column distances
    # are large while each pixel's nearest feature is near; a strip is then
    # sampled, and its rows take the windowed search when the sample is
    # short, else the envelope. An empty quarter or band of columns leaves
    # some strips' samples long and others short.
    rng = np.random.default_rng(9100)
    frame = False
    if case == "density 0.001":
        F = (rng.random((4096, 4096)) < 0.001).astype(np.uint8)
    elif case == "2000 features, frame":
        F, frame = _sparse(4096, 4096, 2000, 9101), True
    elif case == "empty right quarter":
        F = (rng.random((4096, 4096)) < 0.005).astype(np.uint8)
        F[:, 3072:] = 0
    else:
        F = (rng.random((4096, 4096)) < 0.005).astype(np.uint8)
        F[:, 2000:2096] = 0
    say("edt 4096^2 scattered:", case)
    assert np.array_equal(_edt(F, frame), oracle.edt_sq(F, frame))
