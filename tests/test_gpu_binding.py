"""The binding's argument checks: every malformed tensor is refused before a
pointer reaches the library (a wrong dtype, a host tensor, a mismatched
plane or an undersized output would otherwise be read or written out of
bounds by a kernel)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu


def _x(H=40, W=50, seed=1):
    return dev(synth.random_binary(H, W, 0.5, seed))


def test_companion_planes_are_checked():
    say("binding: companion planes")
    x = _x()
    bad = [x.float(), x.cpu(), _x(40, 51), x[:, :49].contiguous(), torch.zeros(40, 50, 2, dtype=torch.uint8,
                                                                                  device="cuda")]
    for C in bad:
        with pytest.raises(ValueError):
            ctx().filter(x, C, 2)
        with pytest.raises(ValueError):
            ctx().filter(x, None, 2, D=C, conn=4)
        with pytest.raises(ValueError):
            ctx().homotopic_thin(x, C)
        with pytest.raises(ValueError):
            ctx().homotopic_thicken(x, C)
        with pytest.raises(ValueError):
            ctx().filter_batch([(x, C, 2)])
    with pytest.raises(ValueError):
        ctx().homotopic_thicken(x, None)


def test_edt_output_is_checked():
    say("binding: edt output")
    x = _x()
    for out in (torch.empty(40, 49, dtype=torch.int32, device="cuda"),
                torch.empty(40, 50, dtype=torch.float32, device="cuda"),
                torch.empty(40, 50, dtype=torch.int32),
                torch.empty(50, 40, dtype=torch.int32, device="cuda").t(),
                torch.empty(40 * 50, dtype=torch.int32, device="cuda")):
        with pytest.raises(ValueError):
            ctx().edt_sq(x, True, out)
    # a pitched output is fine
    big = torch.full((40, 64), -7, dtype=torch.int32, device="cuda")
    out = ctx().edt_sq(x, True, big[:, :50])
    ctx().sync()
    X = host(x)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle.edt_sq((X != 0).astype(np.uint8), True))
    assert (big[:, 50:] == -7).all()


def test_rows_must_not_overlap():
    say("binding: overlapping rows")
    base = torch.zeros(64 * 40, dtype=torch.uint8, device="cuda")
    x = base.as_strided((40, 50), (32, 1))
    with pytest.raises(ValueError):
        ctx().filter(x, None, 1)


def test_valid_call_after_refusals_still_works():
    say("binding: valid call after refusals")
    X = synth.random_binary(37, 61, 0.5, 9)
    x = dev(X)
    with pytest.raises(ValueError):
        ctx().filter(x, x.float(), 2)
    ctx().filter(x, None, 2)
    ctx().sync()
    assert np.array_equal(host(x), oracle.hasf(X, None, 2))


def test_server_checks_frames():
    say("binding: server frames")
    srv = hasf.Server(ctx(), lanes=2)
    try:
        x = _x()
        with pytest.raises(ValueError):
            srv.submit(x, x.cpu(), 2)
        with pytest.raises(ValueError):
            srv.submit(x.cpu(), None, 2)
    finally:
        srv.stop()
