"""hasf_filter_labels against the oracle's per-label filter (bit-exact), with
pitched inputs and outputs, many labels, and argument errors."""
import numpy as np
import pytest

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", [(97, 130, 4, 2), (300, 257, 6, 3), (1, 40, 2, 1), (64, 64, 3, 0)])
def test_labels_match_oracle(case):
    H, W, n, r = case
    Lab = synth.label_image(H, W, n, 4000 + H + W)
    values = list(range(n))[::-1]
    say("labels", case)
    P = ctx().filter_labels(dev(Lab), values, r)
    ctx().sync()
    assert np.array_equal(host(P), oracle.hasf_labels(Lab, values, r))


def test_labels_pitched_input_and_output():
    import torch
    H, W, n, r = 120, 90, 3, 3
    Lab = synth.label_image(H, W, n, 4100)
    buf = torch.full((n, H + 2, W + 24), 0xAA, dtype=torch.uint8, device="cuda:0")
    out = buf[:, :H, 5:5 + W]
    say("labels pitched")
    ctx().filter_labels(dev(Lab, pitch=W + 13), [2, 0, 1], r, out=out)
    ctx().sync()
    assert np.array_equal(host(out), oracle.hasf_labels(Lab, [2, 0, 1], r))
    b = host(buf)
    assert (b[:, :, :5] == 0xAA).all() and (b[:, :, 5 + W:] == 0xAA).all() and (b[:, H:, :] == 0xAA).all()


def test_many_labels_in_one_call():
    H, W, n, r = 512, 512, 40, 2
    Lab = synth.label_image(H, W, n, 4200)
    values = list(range(n))
    say("labels 512x512, 40 labels")
    P = host(ctx().filter_labels(dev(Lab), values, r))
    ctx().sync()
    assert np.array_equal(P, oracle.hasf_labels(Lab, values, r))


def test_labels_argument_errors():
    Lab = synth.label_image(30, 40, 3, 4300)
    L = dev(Lab)
    for values, r in (([1, 1], 2), ([], 2), ([0, 1], 16), ([0, 1], -1)):
        with pytest.raises(hasf.HasfError) as e:
            ctx().filter_labels(L, values, r)
        assert e.value.status == hasf.HASF_EINVAL
    with pytest.raises(hasf.HasfError) as e:  # out overlapping L
        ctx().filter_labels(L, [0], 1, out=L.view(1, 30, 40))
    assert e.value.status == hasf.HASF_EINVAL
    ctx().sync()
    assert np.array_equal(host(L), Lab)
