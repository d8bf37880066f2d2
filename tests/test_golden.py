"""Stored expected values: the input generator still draws the inputs they were
computed from."""
import hashlib
import json
import os

from paper_1603_09337_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_large_workload_input_is_the_one_the_digest_was_made_from():
    gold = json.load(open(os.path.join(GOLDEN, "hasf_4096x4096_r10.json")))
    X, C, r = synth.workload_large()
    assert (X.shape, r, C) == ((gold["H"], gold["W"]), gold["r"], None)
    assert int(X.sum()) == gold["input_ones"]
    assert hashlib.sha256(X.tobytes()).hexdigest() == gold["input_sha256"]


def test_batch_and_stream_inputs_are_the_ones_the_digests_were_made_from():
    gold = json.load(open(os.path.join(GOLDEN, "batch_and_stream_digests.json")))
    imgs = gold["batch"]["images"]
    assert [g["k"] for g in imgs] == list(range(256))
    for k in (0, 1, 100, 255):
        X, C, r = synth.batch_item(k)
        assert (X.shape, r) == ((imgs[k]["H"], imgs[k]["W"]), imgs[k]["r"])
        assert hashlib.sha256(X.tobytes()).hexdigest() == imgs[k]["input_sha256"]
    frames = gold["stream_bank"]["frames"]
    assert [g["k"] for g in frames] == list(range(64))
    sched = synth.stream_schedule()
    for k in (0, 63):
        _, H, W, r, fs = sched[k]
        assert (H, W, r) == (frames[k]["H"], frames[k]["W"], frames[k]["r"])
        X = synth.stream_frame(H, W, fs)
        assert hashlib.sha256(X.tobytes()).hexdigest() == frames[k]["input_sha256"]
