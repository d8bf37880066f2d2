"""The two forms of a subfield pass against the oracle. A sub-image of at most
2 x (workgroup threads) words is listed and tested wave by wave; a larger one
through one list shared by the workgroup. Images at the boundary mix both
forms: with an odd number of rows the two row parities of the sub-images
differ in size. A lone image (or a batch of at most one image per CU) runs on
1024-thread workgroups, a larger batch on 512-thread ones."""
import numpy as np
import pytest

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import synth

pytestmark = pytest.mark.gpu

# W = 512: 8 words per sub-image row. At 1024 threads the per-wave form takes
# up to 2048 words (256 sub-image rows): 512 rows both forms per-wave, 513 rows
# one parity each, 514 rows both shared.
LONE = [(512, 512, 3), (513, 512, 4), (514, 512, 2), (511, 512, 3), (300, 1100, 3)]


@pytest.mark.parametrize("case", LONE)
def test_lone_image_at_the_boundary(case):
    H, W, r = case
    X = synth.disks_image(H, W, np.random.default_rng(H * 3 + W))
    C = synth.constraint_pixels(X, 50, np.random.default_rng(H + W))
    say("lone filter", case)
    d = dev(X)
    ctx().filter(d, dev(C), r)
    ctx().sync()
    assert np.array_equal(host(d), oracle.hasf(X, C, r))


def test_large_batch_at_the_boundary():
    # more images than CUs: 512 threads, so the per-wave form takes up to 1024
    # words (128 sub-image rows at W = 512)
    import torch
    nfill = torch.cuda.get_device_properties(0).multi_processor_count + 4
    big = [(256, 512, 3), (257, 512, 3), (258, 512, 2), (255, 512, 4)]
    items = []
    for k, (H, W, r) in enumerate(big):
        items.append((synth.disks_image(H, W, np.random.default_rng(700 + k)), r))
    for k in range(nfill):
        items.append((synth.random_binary(8, 8, 0.5, 7100 + k), 1))
    say("batch of %d images, 4 at the boundary" % len(items))
    ds = [dev(X) for X, _ in items]
    ctx().filter_batch([(d, None, r) for d, (_, r) in zip(ds, items)])
    ctx().sync()
    for k, (d, (X, r)) in enumerate(zip(ds, items)):
        assert np.array_equal(host(d), oracle.hasf(X, None, r)), "image %d" % k


@pytest.mark.parametrize("H", [512, 513, 514])
def test_thin_and_thicken_at_the_boundary(H):
    W = 512
    X = synth.random_binary(H, W, 0.6, 90 + H)
    K = synth.random_binary(H, W, 0.03, 91)
    say("thin", H)
    Xd = dev(X)
    ctx().homotopic_thin(Xd, dev(K))
    ctx().sync()
    assert np.array_equal(host(Xd), oracle.homotopic_thin(X, K))
    Y = synth.random_binary(H, W, 0.2, 92 + H)
    V = synth.random_binary(H, W, 0.7, 93)
    say("thicken", H)
    Yd = dev(Y)
    ctx().homotopic_thicken(Yd, dev(V))
    ctx().sync()
    assert np.array_equal(host(Yd), oracle.homotopic_thicken(Y, V))
