"""bench.py's CPU baseline leg runs end to end on the host (the oracle on a
few 512x512 r=5 frames, one watershed image and one 64^3 volume), so the
bench's JSON line cannot fail on it; the GPU legs are exercised on the GPU."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_cpu_baseline_runs_and_reports_its_sample():
    Xs, Cs = bench.make_inputs(2)
    out = bench.cpu_baseline(Xs, Cs, 1, 2, max_cores=2, per=1)
    assert out["kind"] == "oracle" and out["unit"] == "Mpixel/s"
    assert out["value"] > 0 and 1 <= out["cores"] <= 2
    assert out["one_core"]["value"] > 0
    assert out["watershed_one_core"]["value"] > 0 and out["volumes_one_core"]["value"] > 0
    assert "512x512" in out["sample"]
