"""A context's calls on different streams: the library orders a new stream
after the work already queued on the previous one (the calls share the
context's scratch memory), and a call does not wait on the host for the work
queued before it."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu


def test_calls_on_two_streams_do_not_overlap():
    c = hasf.Context(0)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    X1 = synth.disks_image(700, 1000, np.random.default_rng(5))   # global state, long
    X2 = synth.disks_image(300, 280, np.random.default_rng(6))
    X3 = synth.random_binary(200, 150, 0.5, 7)
    d1, d2, d3 = dev(X1), dev(X2), dev(X3)
    torch.cuda.synchronize()
    say("filters on two streams, no host sync between them")
    with torch.cuda.stream(sa):
        c.filter(d1, None, 4)
    with torch.cuda.stream(sb):
        c.filter(d2, None, 3)
        c.filter_batch([(d3, None, 2)])
    with torch.cuda.stream(sa):
        out = c.edt_sq(d2, True)  # after the filters of d2 (stream order across the switch)
    c.sync()
    torch.cuda.synchronize()
    Y2 = oracle.hasf(X2, None, 3)
    assert np.array_equal(host(d1), oracle.hasf(X1, None, 4))
    assert np.array_equal(host(d2), Y2)
    assert np.array_equal(host(d3), oracle.hasf(X3, None, 2))
    assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle.edt_sq(Y2, True))


def test_many_calls_queued_then_one_sync():
    c = hasf.Context(0)
    imgs = [synth.random_binary(64 + 9 * k, 80, 0.5, 50 + k) for k in range(12)]
    ds = [dev(X) for X in imgs]
    torch.cuda.synchronize()
    say("12 filters queued, one sync")
    for k, d in enumerate(ds):
        if k % 3 == 2:
            c.filter_batch([(d, None, 1 + k % 4)])
        else:
            c.filter(d, None, 1 + k % 4)
    c.sync()
    for k, (d, X) in enumerate(zip(ds, imgs)):
        assert np.array_equal(host(d), oracle.hasf(X, None, 1 + k % 4)), "image %d" % k
