"""Parity of the standalone thinning and thickening for the (4,8) pair
(hasf_homotopic_thin_conn / hasf_homotopic_thicken_conn) with the oracle,
bit-exact, with the state in LDS and in global memory."""
import numpy as np
import pytest

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu

CASES = [(1, 70, 0.6), (60, 1, 0.6), (37, 130, 0.5), (100, 127, 0.45), (256, 256, 0.5), (600, 700, 0.5)]


@pytest.mark.parametrize("case", CASES)
def test_thin_48(case):
    H, W, dens = case
    X = synth.random_binary(H, W, dens, 3000 + H + W)
    K = synth.random_binary(H, W, 0.03, 3100 + H)
    say("thin (4,8)", case)
    x, k = dev(X, W + 5), dev(K, W + 5)
    ctx().homotopic_thin(x, k, conn=4)
    ctx().sync()
    assert np.array_equal(host(x), oracle.homotopic_thin(X, K, n=4))


@pytest.mark.parametrize("case", CASES)
def test_thicken_48(case):
    H, W, dens = case
    X = synth.random_binary(H, W, dens * 0.4, 3200 + H + W)
    V = synth.random_binary(H, W, 0.7, 3300 + W)
    say("thicken (4,8)", case)
    y, v = dev(X), dev(V)
    ctx().homotopic_thicken(y, v, conn=4)
    ctx().sync()
    assert np.array_equal(host(y), oracle.homotopic_thicken(X, V, n=4))


def test_disks_both_pairs():
    X = synth.disks_image(300, 280, np.random.default_rng(8))
    for n in (8, 4):
        say("thin, disks, pair", n)
        x = dev(X)
        ctx().homotopic_thin(x, None, conn=n)
        ctx().sync()
        assert np.array_equal(host(x), oracle.homotopic_thin(X, None, n=n))


def test_bad_conn_is_refused():
    X = synth.random_binary(30, 40, 0.5, 3400)
    x = dev(X)
    with pytest.raises(hasf.HasfError) as e:
        ctx().homotopic_thin(x, None, conn=6)
    assert e.value.status == hasf.HASF_EINVAL
    ctx().sync()
    assert np.array_equal(host(x), X)
