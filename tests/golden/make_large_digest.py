"""Writes hasf_4096x4096_r10.json: the oracle's result on the 4096x4096, r=10
workload (synth.workload_large, its fixed seed), as a SHA-256 digest of the
H x W uint8 0/1 output (row-major, no padding) and its object-pixel count.

The full image is too large to store; the GPU test compares the digest of its
own output. Runs the oracle only (about four minutes on one core):

    python tests/golden/make_large_digest.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1603_09337_amd import synth  # noqa: E402


def main():
    X, C, r = synth.workload_large()
    t = time.time()
    Y = oracle.hasf(X, C, r)
    dt = time.time() - t
    out = {
        "workload": "synth.workload_large (4096x4096, 3000 shapes, r=10, C empty), seed %d" % synth.SEED_LARGE,
        "H": int(Y.shape[0]), "W": int(Y.shape[1]), "r": r,
        "input_sha256": hashlib.sha256(X.tobytes()).hexdigest(),
        "input_ones": int(X.sum()),
        "sha256": hashlib.sha256(Y.tobytes()).hexdigest(),
        "ones": int(Y.sum()),
        "oracle_seconds": round(dt, 1),
    }
    with open(os.path.join(HERE, "hasf_4096x4096_r10.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
