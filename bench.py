"""Benchmark: HASF on 512x512 binary images, r = 5: batched, plain and served.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--plain P]
                [--serve-seconds S] [--mixed-seconds M] [--no-serve] [--no-cpu]
python bench.py --only-edt      (the 4096x4096 exact EDT alone, for profiling)
python bench.py --only-volumes  (the 3D leg alone, for profiling)
python bench.py --only-watershed (the watershed leg alone, for profiling)

A step filters one batch of B synthetic 512x512 images (the 40-shape recipe
with a 200-pixel constraint set each) in one persistent launch
(hasf_filter_batch); the batch is first restored from a pristine device copy,
since the filter works in place. Inputs are resident in HBM before timing.
The value is the batched path's Mpixel/s over the K timed steps.

Beside it, on the same GPU:
* plain: one hasf_filter launch per image, serially, on P images (frames/s and
  per-frame latency from HIP events);
* served (hasf_serve): a Poisson stream of 512x512 r=5 frames at 2000
  frames/s for S seconds (frames/s, p50/p99 latency from submission to
  completion), a burst of 4096 such frames submitted at once (the server's
  capacity), and the mixed stream -- Poisson 2000 frames/s for M seconds,
  sides U[256,2048], r U{2..8}, the 12-disk recipe; its frames cycle through
  64 distinct drawn frames of the schedule -- with the plain path timed on
  those 64 frames;
* edt: the exact squared EDT (hasf_edt_sq) of the 4096x4096 r=10 input, as
  HBM GB/s against the 8 TB/s peak, on 9 bytes per pixel (a two-pass EDT
  that writes and reads its column distances) and on the 5 bytes per pixel
  this layout moves (read the features once, write the squared distances);
* large: the whole filter on that 4096x4096 r=10 image alone;
* roofline: the thinning and thickening rounds of that filter against HBM:
  1.375 bytes per pixel per round (object and constraint bits read, a 1-byte
  level map read, object bits written) times the rounds of the schedule,
  counted on the device (hasf_get_grid_counts), over the kernel's time from
  HIP events on the stream it runs on;
* batch_kernel: diagnostics of the batched kernel (VALU lane operations from
  the committed rocprofv3 counter summary against the int32 VALU peak);
* cpu_baseline: the CPU oracle on a sample of the 512x512 images, on one
  core and as independent processes on up to 16 host cores.
Prints one JSON line.

The served streams run one launch lane per hardware queue. --hw-queues Q
(default 16; 0 keeps the environment's) sets GPU_MAX_HW_QUEUES for this
process before torch, and so the HIP runtime, starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# hardware queues of the process, set from --hw-queues before the HIP runtime
# starts (the served streams run one launch lane per queue)
HW_QUEUES = 4

H = W = 512
R = 5
# int32 VALU lanes: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (ops/s)
VALU_INT32_PEAK = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8.0e12  # bytes/s
# VALU instructions and HBM bytes per 512x512 r=5 image of the filter kernel,
# from rocprofv3 --pmc (SQ_INSTS_VALU, FETCH_SIZE, WRITE_SIZE); each wave64
# VALU instruction is 64 lane-ops
PROFILE_COUNTS = os.path.join(ROOT, "profiles", "filter_512x512_r5_counters.json")
# exact EDT: a two-pass EDT reads the features (1 B), writes and reads the
# column distances g (uint16, 2 + 2 B) and writes d^2 (uint32, 4 B); this
# layout keeps g on chip, so its compulsory bytes are 1 B read + 4 B written
EDT_BYTES_PER_PX = 9
EDT_BYTES_PER_PX_LAYOUT = 5
# one round of thinning or thickening (four subfield passes over the window):
# object bits and constraint or limit bits read (1/8 + 1/8 B), a 1-byte level
# map read, object bits written (1/8 B)
ROUND_BYTES_PER_PX = 1.375
# HBM bytes per hasf_edt_sq call on the 4096x4096 input, from rocprofv3 --pmc
# (FETCH_SIZE, WRITE_SIZE of the EDT kernels of the same calls as bench_edt)
EDT_COUNTS = os.path.join(ROOT, "profiles", "edt_4096_counters.json")
# HBM bytes of one whole 4096x4096 r=10 filter (the tile kernel), from the
# same rocprofv3 --pmc runs
LARGE_COUNTS = os.path.join(ROOT, "profiles", "filter_4096x4096_r10_counters.json")


def sources_sha256():
    """SHA-256 over the kernel sources (paper_1603_09337_amd/csrc, sorted by
    name): the counter files record the value they were taken at, and their
    figures are used only while it still matches."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1603_09337_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def load_counts(path):
    """A counter file's figures, or None when it is missing or was taken on
    other kernel sources."""
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    return d if d.get("sources_sha256") == sources_sha256() else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--distinct", type=int, default=64)
    ap.add_argument("--plain", type=int, default=64)
    ap.add_argument("--cpu-sample", type=int, default=12)
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--mixed-seconds", type=float, default=10.0)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--high-rate", type=float, default=20000.0)
    ap.add_argument("--high-seconds", type=float, default=2.0)
    ap.add_argument("--lanes", type=int, default=0)  # 0: one per hardware queue
    ap.add_argument("--hw-queues", type=int, default=16)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-edt", action="store_true")
    ap.add_argument("--only-volumes", action="store_true")
    ap.add_argument("--only-watershed", action="store_true")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(n_distinct):
    import numpy as np
    from paper_1603_09337_amd import synth
    Xs, Cs = [], []
    for k in range(n_distinct):
        X, C, r = synth.workload_shapes(seed=synth.SEED_SHAPES + 7919 * k)
        assert r == R
        Xs.append(X)
        Cs.append(C)
    return np.stack(Xs), np.stack(Cs)


def bench_edt(ctx, reps=20):
    """Exact squared EDT of the 4096x4096 input, HBM GB/s."""
    import torch
    from paper_1603_09337_amd import synth
    X, _, _ = synth.workload_large()
    Hn, Wn = X.shape
    x = torch.from_numpy(X).cuda()
    d2 = torch.empty((Hn, Wn), dtype=torch.int32, device="cuda")
    for _ in range(3):
        ctx.edt_sq(x, True, d2)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        ctx.edt_sq(x, True, d2)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    bytes_ = EDT_BYTES_PER_PX * Hn * Wn
    bytes_l = EDT_BYTES_PER_PX_LAYOUT * Hn * Wn
    ec = load_counts(EDT_COUNTS)
    traffic = ec.get("hbm_bytes_per_call") if ec else None
    return {"bound": "hbm", "achieved": round(bytes_ / t / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": round(bytes_ / t / HBM_PEAK, 4), "traffic": traffic, "us_per_call": round(t * 1e6, 1),
            "workload": "hasf_edt_sq 4096x4096, border is feature (the 4096x4096 r=10 input)",
            "bytes_per_px": EDT_BYTES_PER_PX, "bytes_per_call": bytes_,
            "layout": {"bytes_per_px": EDT_BYTES_PER_PX_LAYOUT, "bytes_per_call": bytes_l,
                       "achieved": round(bytes_l / t / 1e9, 1), "frac": round(bytes_l / t / HBM_PEAK, 4)}}


def bench_large(ctx, reps=3):
    """The whole filter on the 4096x4096 r=10 image alone (the large-image path: tiles in LDS)."""
    import torch
    from paper_1603_09337_amd import hasf, synth
    X, C, r = synth.workload_large()
    src = torch.from_numpy(X).cuda()
    d = src.clone()
    ctx.filter(d, None, r)
    ctx.sync()
    ctx.grid_counts(reset=True)
    # the filter runs on the current stream, where the events are recorded
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        d.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.filter(d, None, r)
        e1.record(stream)
        ctx.sync()
        ts.append(e0.elapsed_time(e1))
    counts = ctx.grid_counts(reset=True)
    ms = min(ts)
    ms_avg = sum(ts) / len(ts)
    tiled = ctx.tile_rows >= 0
    # the library's default tile shape for an image of this size (the bands
    # cut into column tiles of whole 64-column words that fill the CUs)
    dth, dhalo = hasf.default_tile_shape(*X.shape)
    th = ctx.tile_rows or dth
    halo = ctx.tile_halo or dhalo
    out = {"workload": "hasf 4096x4096 r=10, C empty, one image (%s)" %
           ("tiles in LDS: bands of %d rows, %d halo rows, cut into column tiles" % (th, halo) if tiled
            else "grid of workgroups"),
           "ms": round(ms, 2), "ms_avg": round(ms_avg, 2),
           "Mpixel_per_s": round(X.size / ms / 1e3, 2), "frames_per_s": round(1e3 / ms, 3),
           "per_filter": {k: v / counts["launches"] for k, v in counts.items() if k != "launches"}}
    # the thinning and thickening rounds against HBM: algorithmic bytes of the
    # schedule's rounds (counted on the device) over the kernel's mean time
    # (which also holds the distance stages)
    rounds = counts["rounds"] / counts["launches"]
    alg = ROUND_BYTES_PER_PX * X.size * rounds
    traffic = None
    lc = load_counts(LARGE_COUNTS)
    if lc and lc.get("kernel") == ("hasf_tile_kernel" if tiled else "hasf_grid_kernel"):
        traffic = lc.get("hbm_bytes_per_filter")
    out["roofline"] = {"bound": "hbm", "achieved": round(alg / (ms_avg / 1e3) / 1e9, 1), "peak": HBM_PEAK / 1e9,
                       "unit": "GB/s", "frac": round(alg / (ms_avg / 1e3) / HBM_PEAK, 4), "traffic": traffic,
                       "kernel": "hasf_tile_kernel" if tiled else "hasf_grid_kernel",
                       "workload": out["workload"], "rounds": rounds, "bytes_per_px_round": ROUND_BYTES_PER_PX,
                       "px": X.size, "algorithmic_bytes": alg, "kernel_ms": round(ms_avg, 3)}
    return out


def run_stream(srv, frames, arrivals):
    """Submit frames[k] at arrivals[k] seconds (host clock) and wait for all."""
    t0 = time.perf_counter()
    tickets = []
    for (x, c, r), ta in zip(frames, arrivals):
        while True:
            dt = ta - (time.perf_counter() - t0)
            if dt <= 0:
                break
            if dt > 1e-3:
                time.sleep(dt - 5e-4)
        tickets.append(srv.submit(x, c, r))
    t_sub = time.perf_counter() - t0
    res = [srv.wait(t, 120000) for t in tickets]
    if any(r is None for r in res):
        raise RuntimeError("served frame did not complete in 120 s")
    st = srv.stats()
    return st, res, t_sub


def stream_summary(st, res, npx, t_sub, rate=None):
    import numpy as np
    lat = np.array([r["latency_ms"] for r in res])
    t_first = min(r["submit_s"] for r in res)
    t_last = max(r["done_s"] for r in res)
    out = {"frames": len(res), "frames_per_s": round(len(res) / (t_last - t_first), 1),
           "Mpixel_per_s": round(npx / (t_last - t_first) / 1e6, 2),
           "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
           "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
           "latency_ms_max": round(float(lat.max()), 3),
           "kernel_launches": int(st["kernel_launches"]),
           "frames_per_launch": round(float(st["frames_per_launch"]), 2),
           "pool_peak_MiB": round(st["pool_peak_bytes"] / 2**20, 1)}
    if rate is not None:
        out["offered_frames_per_s"] = rate
        out["submit_seconds"] = round(t_sub, 3)
    return out


def bench_served(ctx, a, src, Cd):
    """Served streams: 512x512 Poisson, 512x512 burst, mixed-size Poisson."""
    import numpy as np
    import torch
    from paper_1603_09337_amd import hasf, synth
    out = {"hw_queues": HW_QUEUES, "lanes": a.lanes or min(hasf.HASF_SERVE_LANES_MAX, HW_QUEUES)}
    rng = np.random.Generator(np.random.PCG64(synth.SEED_STREAM + 1))

    # 512x512 r=5 at the offered rate
    gaps = rng.exponential(1.0 / a.rate, size=int(a.rate * a.serve_seconds * 1.5) + 16)
    arr = np.cumsum(gaps)
    arr = arr[arr < a.serve_seconds]
    n = len(arr)
    D = src.shape[0]
    X = src[torch.arange(n, device=src.device) % D].clone()
    torch.cuda.synchronize()
    frames = [(X[k], Cd[k % D], R) for k in range(n)]
    srv = hasf.Server(ctx, lanes=a.lanes)
    # warm the server's lanes
    w = src[:8].clone()
    torch.cuda.synchronize()
    for t in [srv.submit(w[k], Cd[k], R) for k in range(8)]:
        srv.wait(t, 60000)
    srv.stop()
    srv = hasf.Server(ctx, lanes=a.lanes)
    log("served 512x512 stream: %d frames" % n)
    st, res, t_sub = run_stream(srv, frames, arr)
    srv.stop()
    out["stream_512"] = stream_summary(st, res, n * H * W, t_sub, a.rate)
    out["stream_512"]["workload"] = "Poisson %g frames/s for %g s, 512x512 r=5, C = 200 pixels" % (
        a.rate, a.serve_seconds)
    del X, frames

    # 512x512 r=5 at a rate well above the plain path's capacity
    if a.high_rate > 0 and a.high_seconds > 0:
        gaps = rng.exponential(1.0 / a.high_rate, size=int(a.high_rate * a.high_seconds * 1.5) + 16)
        arr = np.cumsum(gaps)
        arr = arr[arr < a.high_seconds]
        n = len(arr)
        X = src[torch.arange(n, device=src.device) % D].clone()
        torch.cuda.synchronize()
        frames = [(X[k], Cd[k % D], R) for k in range(n)]
        srv = hasf.Server(ctx, lanes=a.lanes)
        log("served 512x512 stream at %g frames/s: %d frames" % (a.high_rate, n))
        st, res, t_sub = run_stream(srv, frames, arr)
        srv.stop()
        out["stream_512_high"] = stream_summary(st, res, n * H * W, t_sub, a.high_rate)
        out["stream_512_high"]["workload"] = "Poisson %g frames/s for %g s, 512x512 r=5, C = 200 pixels" % (
            a.high_rate, a.high_seconds)
        del X, frames

    # burst: the server's capacity on 512x512 r=5
    nb = 4096
    Xb = src[torch.arange(nb, device=src.device) % D].clone()
    torch.cuda.synchronize()
    srv = hasf.Server(ctx, lanes=a.lanes)
    log("served 512x512 burst: %d frames" % nb)
    st, res, t_sub = run_stream(srv, [(Xb[k], Cd[k % D], R) for k in range(nb)], np.zeros(nb))
    srv.stop()
    out["burst_512"] = stream_summary(st, res, nb * H * W, t_sub)
    out["burst_512"]["workload"] = "4096 frames 512x512 r=5 submitted at once"
    del Xb

    # mixed sizes
    sched = synth.stream_schedule(rate=a.rate, seconds=a.mixed_seconds)
    nbank = min(64, len(sched))
    bank = []
    for k in range(nbank):
        _, Hk, Wk, rk, fs = sched[k]
        bank.append((torch.from_numpy(synth.stream_frame(Hk, Wk, fs)).cuda(), rk))
    offs, tot = [], 0
    for k in range(len(sched)):
        Hk, Wk = bank[k % nbank][0].shape
        offs.append(tot)
        tot += (Hk * Wk + 255) // 256 * 256
    flat = torch.empty(tot, dtype=torch.uint8, device="cuda")
    frames, npx = [], 0
    for k in range(len(sched)):
        b, rk = bank[k % nbank]
        Hk, Wk = b.shape
        v = flat[offs[k]:offs[k] + Hk * Wk].view(Hk, Wk)
        v.copy_(b)
        frames.append((v, None, rk))
        npx += Hk * Wk
    torch.cuda.synchronize()
    srv = hasf.Server(ctx, lanes=a.lanes)
    log("served mixed stream: %d frames, %.2f Gpx" % (len(frames), npx / 1e9))
    st, res, t_sub = run_stream(srv, frames, [s[0] for s in sched])
    srv.stop()
    mixed = stream_summary(st, res, npx, t_sub, a.rate)
    mixed["workload"] = ("Poisson %g frames/s for %g s, H and W U[256,2048], r U{2..8}, 12-disk recipe "
                         "(frames cycle through %d drawn frames)" % (a.rate, a.mixed_seconds, nbank))
    # latency by frame size (pixels)
    px = np.array([f[0].shape[0] * f[0].shape[1] for f in frames])
    lat = np.array([r["latency_ms"] for r in res])
    buckets = {}
    for lo, hi, name in [(0, 2**19, "<=0.5Mpx"), (2**19, 2**21, "0.5-2Mpx"), (2**21, 2**23, ">2Mpx")]:
        m = (px > lo) & (px <= hi)
        if m.any():
            buckets[name] = {"frames": int(m.sum()), "latency_ms_p50": round(float(np.percentile(lat[m], 50)), 2),
                             "latency_ms_p99": round(float(np.percentile(lat[m], 99)), 2)}
    mixed["by_size"] = buckets
    out["stream_mixed"] = mixed
    del frames, flat

    # plain path on the mixed stream's distinct frames
    stream = torch.cuda.current_stream()
    work = [(b.clone(), rk) for b, rk in bank]
    torch.cuda.synchronize()
    ev = []
    t0 = time.perf_counter()
    for x, rk in work:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.filter(x, None, rk)
        e1.record(stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pl = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    ppx = sum(x.shape[0] * x.shape[1] for x, _ in work)
    out["plain_mixed"] = {"frames": nbank, "frames_per_s": round(nbank / (t1 - t0), 2),
                          "Mpixel_per_s": round(ppx / (t1 - t0) / 1e6, 2),
                          "latency_ms_p50": round(float(np.percentile(pl, 50)), 2),
                          "latency_ms_p99": round(float(np.percentile(pl, 99)), 2)}
    return out


def bench_labels(ctx, reps=5):
    """Per-label smoothing of a 512x512 label image with 16 labels at r=5: the
    label planes are extracted and filtered in one batched call."""
    import torch
    from paper_1603_09337_amd import synth
    Hn = Wn = 512
    n, r = 16, 5
    Lab = torch.from_numpy(synth.label_image(Hn, Wn, n, synth.SEED_SHAPES + 16)).cuda()
    values = list(range(n))
    out = torch.empty((n, Hn, Wn), dtype=torch.uint8, device="cuda")
    ctx.filter_labels(Lab, values, r, out=out)
    ctx.sync()
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.filter_labels(Lab, values, r, out=out)
        e1.record(stream)
        ctx.sync()
        ts.append(e0.elapsed_time(e1))
    ms = min(ts)
    return {"workload": "hasf_filter_labels 512x512, 16 labels (nearest of 48 sites, 1 % noise), r=5",
            "ms": round(ms, 3), "label_planes_per_s": round(n / ms * 1e3, 1),
            "Mpixel_per_s": round(n * Hn * Wn / ms / 1e3, 2)}


def bench_volumes(ctx, reps=3):
    """3D HASF ((26,6)) on a batch of 256 volumes of 64^3 at r = 3 (balls with
    cavities and 2 % noise, 16 distinct volumes): one hasf_filter3_batch launch
    per call, inputs restored before each call outside the timed region (the
    3D oracle is timed in the CPU baseline leg)."""
    import torch
    from paper_1603_09337_amd import synth
    vols, r = synth.workload_volumes()
    src = [torch.from_numpy(v).cuda() for v in vols[:16]]
    work = [src[k % 16].clone() for k in range(len(vols))]
    items = [(w, None, r) for w in work]
    ctx.filter3_batch(items)
    ctx.sync()
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        for k, w in enumerate(work):
            w.copy_(src[k % 16])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.filter3_batch(items)
        e1.record(stream)
        ctx.sync()
        ts.append(e0.elapsed_time(e1))
    ms = min(ts)
    nvox = sum(v.size for v in vols)
    return {"workload": "hasf_filter3_batch: 256 volumes of 64^3, r = 3, (26,6), balls with cavities, 2 % noise",
            "ms": round(ms, 2), "volumes_per_s": round(len(vols) / ms * 1e3, 1),
            "Mvoxel_per_s": round(nvox / ms / 1e3, 1)}


def bench_watershed(ctx, reps=3):
    """The topological watershed's lowering on 64 grey-level 512x512 images
    (synth.grey_image: Gaussian bumps and pits with noise, 16 distinct) in one
    hasf_watershed_batch launch per call, inputs restored before each call
    outside the timed region; and one image alone."""
    import torch
    from paper_1603_09337_amd import synth
    n, Hn, Wn = 64, 512, 512
    bank = [torch.from_numpy(synth.grey_image(Hn, Wn, synth.SEED_GREY + k)).cuda() for k in range(16)]
    work = [bank[k % 16].clone() for k in range(n)]
    ctx.watershed_batch(work)
    ctx.sync()
    stream = torch.cuda.current_stream()

    def timed(imgs, src):
        ts = []
        for _ in range(reps):
            for k, w in enumerate(imgs):
                w.copy_(src[k % len(src)])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.watershed_batch(imgs)
            e1.record(stream)
            ctx.sync()
            ts.append(e0.elapsed_time(e1))
        return min(ts)
    ms = timed(work, bank)
    one = timed(work[:1], bank[:1])
    return {"workload": "hasf_watershed_batch: 64 grey-level 512x512 images (Gaussian bumps and pits, noise)",
            "ms": round(ms, 2), "images_per_s": round(n / ms * 1e3, 1),
            "Mpixel_per_s": round(n * Hn * Wn / ms / 1e3, 1), "one_image_ms": round(one, 2)}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_share(args):
    """One worker of the multi-process leg: the oracle on its images."""
    import oracle
    Xs, Cs = args
    t0 = time.perf_counter()
    for X, C in zip(Xs, Cs):
        oracle.hasf(X, C, R)
    return time.perf_counter() - t0


def cpu_baseline(Xs, Cs, n, distinct, max_cores=16, per=3):
    """The oracle (plain C, one thread per process, as it stands) on n of the
    512x512 r=5 images on one core, then on up to max_cores host cores as
    independent processes with `per` images each (images are independent)."""
    import multiprocessing as mp
    import oracle
    from paper_1603_09337_amd import synth
    log("cpu oracle: %d frames on one core" % n)
    t0 = time.perf_counter()
    for k in range(n):
        oracle.hasf(Xs[k % distinct], Cs[k % distinct], R)
    t1 = time.perf_counter()
    one = n * H * W / (t1 - t0) / 1e6
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(max_cores, avail))
    shares = [([Xs[(c * per + j) % distinct] for j in range(per)], [Cs[(c * per + j) % distinct] for j in range(per)])
              for c in range(cores)]
    log("cpu oracle: %d frames on %d processes" % (cores * per, cores))
    ctx_mp = mp.get_context("spawn")
    with ctx_mp.Pool(cores) as pool:
        pool.map(_oracle_share, shares[:cores])  # start-up and library load outside the timing
        t2 = time.perf_counter()
        pool.map(_oracle_share, shares)
        t3 = time.perf_counter()
    multi = cores * per * H * W / (t3 - t2) / 1e6
    # the watershed oracle on one image of the watershed leg, one core
    Gw = synth.grey_image(512, 512, synth.SEED_GREY)
    log("cpu oracle: one 512x512 watershed")
    t6 = time.perf_counter()
    oracle.wshed(Gw)
    t7 = time.perf_counter()
    # the 3D oracle on one volume of the 3D leg's workload, one core
    vols, r3 = synth.workload_volumes(n=1)
    log("cpu oracle: one 64^3 volume, r=3")
    t4 = time.perf_counter()
    oracle.hasf3(vols[0], None, r3)
    t5 = time.perf_counter()
    return {"value": round(multi, 3), "unit": "Mpixel/s", "cores": cores, "kind": "oracle",
            "watershed_one_core": {"value": round(Gw.size / (t7 - t6) / 1e6, 4), "unit": "Mpixel/s",
                                   "sample": "one 512x512 image of the watershed leg", "cores": 1},
            "volumes_one_core": {"value": round(vols[0].size / (t5 - t4) / 1e6, 4), "unit": "Mvoxel/s",
                                 "sample": "one 64^3 volume of the 3D leg, r = 3", "cores": 1},
            "frames_per_s": round(cores * per / (t3 - t2), 3),
            "sample": "%d of the 512x512 r=5 images (C = 200 px), %d per process on %d processes; "
                      "one core: %d images" % (cores * per, per, cores, n),
            "one_core": {"value": round(one, 4), "unit": "Mpixel/s", "frames_per_s": round(n / (t1 - t0), 3),
                         "cores": 1},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "affinity": avail,
            "paper": "32 images/s at 512x512 on 8 cores of 2x Xeon E5405 (2 GHz), radius not stated"}


def main():
    global HW_QUEUES
    a = parse()
    if a.hw_queues > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(a.hw_queues)
    HW_QUEUES = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    if a.gpus != 1:
        print("bench.py: libhasf runs on one GPU; --gpus %d is not supported (use --gpus 1)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1603_09337_amd import hasf

    dev = torch.device("cuda:0")
    ctx = hasf.Context(0)
    if a.only_edt:
        print(json.dumps({"edt": bench_edt(ctx, reps=a.steps)}), flush=True)
        return
    if a.only_volumes:
        print(json.dumps({"volumes": bench_volumes(ctx, reps=a.steps)}), flush=True)
        return
    if a.only_watershed:
        print(json.dumps({"watershed": bench_watershed(ctx, reps=a.steps)}), flush=True)
        return
    Xs, Cs = make_inputs(a.distinct)
    B = a.batch
    idx = np.arange(B) % a.distinct
    src = torch.from_numpy(Xs[idx]).to(dev)
    Cd = torch.from_numpy(Cs[idx]).to(dev)
    work = src.clone()
    plan = ctx.plan_batch([(work[k], Cd[k], R) for k in range(B)])
    stream = torch.cuda.current_stream(dev)

    def step(kernel_events=None):
        work.copy_(src)
        if kernel_events is not None:
            kernel_events[0].record(stream)
        ctx.run_plan(plan)
        if kernel_events is not None:
            kernel_events[1].record(stream)

    log("batched: %d steps of %d images" % (a.steps, B))
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kern_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    frames = B * a.steps
    px = frames * H * W

    # plain path: one launch per frame
    log("plain: %d frames" % a.plain)
    lat = []
    pw = src[: a.plain].clone()
    pc = Cd[: a.plain]
    for k in range(min(4, a.plain)):
        ctx.filter(pw[k], pc[k], R)
    torch.cuda.synchronize()
    pw.copy_(src[: a.plain])
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for k in range(a.plain):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.filter(pw[k], pc[k], R)
        e1.record(stream)
        lat.append((e0, e1))
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    lat_ms = np.array([e0.elapsed_time(e1) for e0, e1 in lat])
    plain_fps = a.plain / (tp1 - tp0)

    # diagnostics of the batched kernel: an image's state lives in LDS and
    # its compulsory HBM traffic is 3 B/px, so it is not held to a roofline;
    # how busy its vector ALUs are comes from the committed instruction counts
    kern_s = float(np.mean(kern_ms)) / 1e3
    batch_diag = {"kernel": "hasf_filter_kernel<512>", "kernel_ms": round(kern_s * 1e3, 3),
                  "compulsory_bytes": 3 * H * W * B,
                  "compulsory_GB_per_s": round(3 * H * W * B / kern_s / 1e9, 1)}
    counts = load_counts(PROFILE_COUNTS)
    if counts and counts.get("valu_insts_per_image"):
        ops = counts["valu_insts_per_image"] * 64.0 * B
        batch_diag["valu_busy"] = round(ops / kern_s / VALU_INT32_PEAK, 4)
        batch_diag["valu_lane_ops_per_s"] = round(ops / kern_s / 1e12, 3)
        if counts.get("hbm_bytes_per_image") is not None:
            batch_diag["traffic"] = counts["hbm_bytes_per_image"] * B

    log("edt 4096x4096")
    edt = bench_edt(ctx)
    log("filter 4096x4096 r=10")
    large = bench_large(ctx)
    log("labels 512x512, 16 labels")
    labels = bench_labels(ctx)
    log("volumes 256 x 64^3 r=3")
    volumes = bench_volumes(ctx)
    log("watershed 64 x 512x512")
    watershed = bench_watershed(ctx)

    served = None
    if not a.no_serve:
        served = bench_served(ctx, a, src, Cd)

    cpu = None
    if not a.no_cpu and a.cpu_sample > 0:
        cpu = cpu_baseline(Xs, Cs, a.cpu_sample, a.distinct)

    out = {
        "metric": "Mpixel/s and frames/s for HASF 512^2 r=5 (batched vs plain); p50/p99 frame latency",
        "value": round(px / wall / 1e6, 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "hasf 512x512 r=5, C = 200 pixels, batched (one persistent launch per step)",
                   "batch": B, "distinct_images": a.distinct, "H": H, "W": W, "r": R},
        "frames_per_s": round(frames / wall, 1),
        "plain": {"frames_per_s": round(plain_fps, 1), "Mpixel_per_s": round(plain_fps * H * W / 1e6, 2),
                  "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
                  "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3), "frames": a.plain},
        "batched_over_plain": round((frames / wall) / plain_fps, 2),
        "batch_kernel_ms": round(float(np.mean(kern_ms)), 3),
        "served": served,
        "served_over_plain": (round(served["stream_512"]["frames_per_s"] / plain_fps, 2) if served else None),
        # the same frames offered at a rate far above the plain path's capacity
        "served_high_over_plain": (round(served["stream_512_high"]["frames_per_s"] / plain_fps, 1)
                                   if served and "stream_512_high" in served else None),
        # the stream above is capped by its offered rate; the burst measures the server's capacity
        "served_capacity_over_plain": (round(served["burst_512"]["frames_per_s"] / plain_fps, 1)
                                       if served else None),
        "edt": edt,
        "large": large,
        "labels": labels,
        "volumes": volumes,
        "watershed": watershed,
        "batch_kernel": batch_diag,
        "roofline": large["roofline"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
