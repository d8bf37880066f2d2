"""Writes batch_and_stream_digests.json: the oracle's result on every image of
the 256-image uneven batch (synth.workload_batch(256): sides U[128, 1024], r
U{2..8}) and on every frame of the mixed-stream bank (the first 64 frames of
synth.stream_schedule(2000 frames/s, 10 s): sides U[256, 2048], r U{2..8},
the frames the benchmark's mixed stream cycles through), as the SHA-256 of
each H x W uint8 0/1 output (row-major, no padding), with the input's digest.

Runs the oracle only, in worker processes (a few minutes on 8 cores):

    python tests/golden/make_batch_digests.py [workers]
"""
import hashlib
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1603_09337_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "batch_and_stream_digests.json")
BANK = 64


def _batch(k):
    X, C, r = synth.batch_item(k)
    Y = oracle.hasf(X, C, r)
    return {"k": k, "H": int(X.shape[0]), "W": int(X.shape[1]), "r": r,
            "input_sha256": hashlib.sha256(X.tobytes()).hexdigest(),
            "sha256": hashlib.sha256(Y.tobytes()).hexdigest(), "ones": int(Y.sum())}


def _frame(k):
    _, H, W, r, fs = synth.stream_schedule()[k]
    X = synth.stream_frame(H, W, fs)
    Y = oracle.hasf(X, None, r)
    return {"k": k, "H": H, "W": W, "r": r,
            "input_sha256": hashlib.sha256(X.tobytes()).hexdigest(),
            "sha256": hashlib.sha256(Y.tobytes()).hexdigest(), "ones": int(Y.sum())}


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 1)
    oracle.build(force=False)
    t = time.time()
    with Pool(workers) as p:
        frames = p.map(_frame, range(BANK), chunksize=1)
        batch = p.map(_batch, range(256), chunksize=1)
    out = {
        "batch": {"workload": "synth.workload_batch(256): sides U[128,1024], r U{2..8}, 12-disk recipe, "
                              "image k seeded %d*1000+k" % synth.SEED_BATCH,
                  "images": batch},
        "stream_bank": {"workload": "first %d frames of synth.stream_schedule(2000 frames/s, 10 s), seed %d: "
                                    "sides U[256,2048], r U{2..8}, 12-disk recipe" % (BANK, synth.SEED_STREAM),
                        "frames": frames},
        "oracle_seconds": round(time.time() - t, 1),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print("wrote", OUT, out["oracle_seconds"], "s")


if __name__ == "__main__":
    main()
