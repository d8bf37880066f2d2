"""Parity of the topological watershed's lowering (hasf_watershed,
hasf_watershed_batch: grey-level W-thinning, lower sections 4-connected) with
the oracle, bit-exact: smooth and random grey images of ragged sizes, single
rows and columns, constant images, pitched buffers, an uneven batch in one
launch, and a tall image whose per-word flags do not fit LDS (every word then
tested in every pass); plus the separation of every lower section and the
argument checks."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth
from test_oracle_wshed import separation_ok

pytestmark = pytest.mark.gpu


def _ws(F, pitch=None):
    d = dev(F, pitch)
    ctx().watershed(d)
    ctx().sync()
    return host(d)


CASES = [
    # (kind, H, W, seed)
    ("grey", 1, 300, 1), ("grey", 300, 1, 2), ("grey", 2, 2, 3), ("grey", 37, 130, 4),
    ("grey", 64, 64, 5), ("grey", 129, 191, 6), ("grey", 256, 256, 7), ("grey", 100, 700, 8),
    ("rand", 50, 77, 9), ("rand", 200, 65, 10), ("grey", 512, 512, 11),
]


def _image(kind, H, W, seed):
    if kind == "grey":
        return synth.grey_image(H, W, 5000 + seed)
    return np.random.default_rng(seed).integers(0, 9, (H, W)).astype(np.uint8)


@pytest.mark.parametrize("case", CASES)
def test_watershed_matches_oracle(case):
    F = _image(*case)
    say("watershed", case)
    got = _ws(F)
    assert np.array_equal(got, oracle.wshed(F))
    if F.size <= 70000:
        assert separation_ok(F, got)


def test_watershed_pitch_constant_and_no_flags():
    F = synth.grey_image(90, 140, 5100)
    say("watershed pitch")
    assert np.array_equal(_ws(F, pitch=203), oracle.wshed(F))
    C = np.full((40, 70), 9, np.uint8)
    assert np.array_equal(_ws(C), C)
    # 24577 rows of one word: the flags would need more LDS than allowed
    T = np.random.default_rng(12).integers(0, 40, (24577, 1)).astype(np.uint8)
    say("watershed, no flags")
    assert np.array_equal(_ws(T), oracle.wshed(T))


def test_watershed_batch_of_uneven_images():
    rng = np.random.default_rng(13)
    imgs = [_image("grey" if k % 3 else "rand", int(rng.integers(1, 200)), int(rng.integers(1, 300)), 200 + k)
            for k in range(20)]
    ds = [dev(F) for F in imgs]
    say("watershed batch of 20")
    ctx().watershed_batch(ds)
    ctx().sync()
    for k, (F, d) in enumerate(zip(imgs, ds)):
        assert np.array_equal(host(d), oracle.wshed(F)), k


def test_watershed_arguments():
    lib = hasf.lib()
    h = ctx()._h
    p = ctypes.c_void_p(0x1000)
    assert lib.hasf_watershed(h, p, 0, 4, 4) == hasf.HASF_EINVAL
    assert lib.hasf_watershed(h, p, 4, 4, 3) == hasf.HASF_EINVAL
    assert lib.hasf_watershed(h, None, 4, 4, 4) == hasf.HASF_EINVAL
    assert lib.hasf_watershed(h, p, 65536, 65536, 65536) == hasf.HASF_EINVAL
    assert lib.hasf_watershed(None, p, 4, 4, 4) == hasf.HASF_EINVAL
