"""The allocation-free EDT entry point (hasf_edt_sq_noalloc) through the C
ABI: bit-exact against hasf_edt_sq on two calls in a row, the second on a
smaller image (the shared scratch keeps the first call's contents), and
against the oracle; sizes beyond its scratch are rejected before any device
work."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu


def _pair(F, frame, pitch=None):
    import torch
    H, W = F.shape
    d = dev(F, pitch)
    a = torch.full((H, W + 5), 123, dtype=torch.int32, device="cuda:0")[:, :W]
    b = torch.full((H, W + 5), 77, dtype=torch.int32, device="cuda:0")[:, :W]
    ctx().edt_sq(d, frame, out=a)
    ctx().edt_sq(d, frame, out=b, noalloc=True)
    ctx().sync()
    return host(a).view(np.uint32), host(b).view(np.uint32)


@pytest.mark.parametrize("frame", [False, True])
def test_noalloc_equals_edt_sq_on_two_calls_the_second_smaller(frame):
    rng = np.random.default_rng(2024 + frame)
    big = synth.workload_disks(H=1000, W=1300)[0] == 0  # background of a disks image: features
    small = rng.random((77, 333)) < 0.02
    for F in (big, small):
        say("noalloc EDT", F.shape, "frame" if frame else "no frame")
        a, b = _pair(F.astype(np.uint8), frame, pitch=F.shape[1] + 64)
        assert np.array_equal(a, b)
        assert np.array_equal(b, oracle.edt_sq(F.astype(np.uint8), frame))


def test_noalloc_at_4096_and_sparse_features():
    F = np.zeros((4096, 4096), np.uint8)
    rng = np.random.default_rng(7)
    F[rng.integers(0, 4096, 16), rng.integers(0, 4096, 16)] = 1
    say("noalloc EDT 4096^2, 16 features, then 3x5")
    a, b = _pair(F, False)
    assert np.array_equal(a, b)
    a, b = _pair(np.eye(3, 5, dtype=np.uint8), True)
    assert np.array_equal(a, b)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    lib = hasf.lib()
    p = ctypes.c_void_p(0x1000)
    # at most ceil(H / 32) * W * 12 + 4 H + W / 8 + 6144 bytes of scratch: 8192 x 8192 needs 24 MiB
    st = lib.hasf_edt_sq_noalloc(ctx()._h, p, 8192, 8192, 8192, 0, p, 8192)
    assert st == hasf.HASF_EINVAL
    assert b"HASF_NOALLOC_SCRATCH_BYTES" in lib.hasf_last_error(ctx()._h)
    # and the device is still usable
    a, b = _pair(np.eye(40, 50, dtype=np.uint8), False)
    assert np.array_equal(a, b)
