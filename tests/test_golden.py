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
