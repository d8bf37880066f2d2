"""Served stream through the persistent polling kernel (HASF_SERVE_PERSISTENT):
every frame's result is the same in the mix as alone (and as the oracle), also
when admission is throttled by a tiny memory pool, with an invalid frame in
the middle, and with a full queue.

That kernel's workgroups stopped making progress on the GPU, the cause has not
been found, and the mode is switched off (hasf_serve returns HASF_EINTERNAL for
it). These tests stay, skipped. The served stream in use is the launch-lane
server, tested in test_gpu_stream.py."""
import numpy as np
import pytest

import oracle
from gpu_util import ctx, dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="persistent polling serve kernel hung on the GPU (workgroup waves out of "
                                      "step, cause not found); the mode is switched off")]


def _frames(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        H, W = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        X = synth.disks_image(H, W, np.random.default_rng(seed * 100 + k))
        C = synth.random_binary(H, W, 0.02, seed + k) if k % 3 == 0 else None
        out.append((X, C, int(rng.integers(0, 9))))
    return out


def _run(server, frames):
    dX = [dev(X) for X, _, _ in frames]
    dC = [dev(C) if C is not None else None for _, C, _ in frames]
    tickets = [server.submit(x, c, r) for x, c, (_, _, r) in zip(dX, dC, frames)]
    res = [server.wait(t, 60000) for t in tickets]
    assert all(r is not None for r in res)
    return [host(x) for x in dX], res


def test_mix_equals_alone_and_oracle():
    frames = _frames(40, 30, 300, 11)
    srv = hasf.Server(ctx(), pool_bytes=256 << 20, persistent=True)
    say("serve mix 40")
    got, res = _run(srv, frames)
    st = srv.stats()
    srv.stop()
    assert st["completed"] == 40 and st["p99_ms"] > 0
    for k, ((X, C, r), g) in enumerate(zip(frames, got)):
        assert np.array_equal(g, oracle.hasf(X, C, r)), "frame %d" % k
    # alone: the same frames through hasf_filter one by one
    for k, (X, C, r) in enumerate(frames[:8]):
        x = dev(X)
        ctx().filter(x, dev(C) if C is not None else None, r)
        ctx().sync()
        assert np.array_equal(host(x), got[k])


def test_tiny_pool_queues_but_completes():
    frames = _frames(12, 100, 260, 23)
    # room for one or two frames' scratch at a time (~0.5 MiB each)
    srv = hasf.Server(ctx(), pool_bytes=1 << 20, persistent=True)
    say("serve tiny pool")
    got, _ = _run(srv, frames)
    st = srv.stats()
    srv.stop()
    assert st["pool_peak_bytes"] <= 1 << 20
    for (X, C, r), g in zip(frames, got):
        assert np.array_equal(g, oracle.hasf(X, C, r))


def test_invalid_frame_does_not_poison_others():
    frames = _frames(6, 40, 120, 31)
    srv = hasf.Server(ctx(), persistent=True)
    dX = [dev(X) for X, _, _ in frames]
    t = []
    for k, (x, (_, _, r)) in enumerate(zip(dX, frames)):
        t.append(srv.submit(x, None, r))
        if k == 2:
            st = srv.submit(x, None, 99, check=False)  # r out of range
            assert st == hasf.HASF_EINVAL
    for tk in t:
        assert srv.wait(tk, 60000) is not None
    s = srv.stats()
    srv.stop()
    assert s["rejected"] == 1
    for (X, _, r), x in zip(frames, dX):
        assert np.array_equal(host(x), oracle.hasf(X, None, r))


def test_full_queue_returns_eagain():
    frames = _frames(10, 200, 260, 41)
    # one or two frames' scratch fit at a time and at most one frame may wait
    srv = hasf.Server(ctx(), pool_bytes=1 << 20, max_pending=1, persistent=True)
    dX = [dev(X) for X, _, _ in frames]
    accepted, saw_eagain = [], False
    for x, (_, _, r) in zip(dX, frames):
        st = srv.submit(x, None, r, check=False)
        if st == hasf.HASF_EAGAIN:
            saw_eagain = True
        else:
            accepted.append(st)
    for tk in accepted:
        assert srv.wait(tk, 60000) is not None
    srv.stop()
    assert saw_eagain
