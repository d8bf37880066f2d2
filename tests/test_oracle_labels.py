"""Pins of the per-label oracle (hasf_labels): each plane is the filter of one
label's pixels, checked against closed forms that do not use the oracle's
filter: r = 0 leaves every label's mask as a per-pixel comparison gives it,
labels absent from the image give empty planes, and well separated digital
disks of (R, r) pairs left unchanged by the classical opening and closing come
back unchanged, each in its own plane."""
import numpy as np

import oracle
import topo_checks as tc


def test_r0_planes_are_the_label_masks():
    rng = np.random.default_rng(5)
    Lab = rng.integers(0, 5, size=(23, 31)).astype(np.uint8)
    values = [3, 0, 4, 1, 2]
    P = oracle.hasf_labels(Lab, values, 0)
    assert P.shape == (5, 23, 31)
    for k, v in enumerate(values):
        for i in range(23):
            for j in range(31):
                assert P[k, i, j] == (1 if Lab[i, j] == v else 0)


def test_absent_label_gives_an_empty_plane():
    Lab = np.full((20, 20), 7, np.uint8)
    Lab[5:15, 5:15] = 9
    P = oracle.hasf_labels(Lab, [200, 9], 3)
    assert not P[0].any()
    # a 10 x 10 square keeps its topology: one component, no hole
    assert tc.components8(P[1]) == 1


def test_separated_smooth_disks_come_back_unchanged():
    # (R, r) pairs that the classical opening and closing by B_r leave
    # unchanged: in 2D the homotopic filter then leaves the disk unchanged too
    pairs = [(6, 2), (10, 3), (9, 2)]
    tiles = [tc.disk_image(R) for R, _ in pairs]
    h = max(t.shape[0] for t in tiles)
    Lab = np.zeros((h, sum(t.shape[1] for t in tiles)), np.uint8)
    x = 0
    spans = []
    for k, t in enumerate(tiles):
        Lab[:t.shape[0], x:x + t.shape[1]][t > 0] = k + 1
        spans.append((x, t))
        x += t.shape[1]
    for k, (R, r) in enumerate(pairs):
        P = oracle.hasf_labels(Lab, [k + 1], r)[0]
        expect = np.zeros_like(Lab)
        x0, t = spans[k]
        expect[:t.shape[0], x0:x0 + t.shape[1]] = t
        assert np.array_equal(P, expect), (R, r)
