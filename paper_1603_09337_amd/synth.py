"""Seeded synthetic binary images standing in for the paper's test images.

The paper measures on 2D binary images (200x200, 168x288 and 512x512) that are
not published. These generators draw images with the same kind of content: a
few filled disks and convex polygons, some with a concentric hole, with a noisy
boundary and isolated salt-and-pepper pixels, which is what a smoothing filter
is meant to clean up.

This module only draws inputs. It holds none of the filter's arithmetic and is
shared by the oracle-side tests and the GPU-side tests and benchmark, so that
both sides see byte-identical inputs for a given seed.

Recipes (seeds are fixed per workload):

* ``disks``   256x256, 12 disks of radius U[8,40], 3 of them with a concentric
  hole of radius round(U[0.3,0.6]*R) >= 2, boundary flip p=0.15, 0.5 % salt and
  pepper, no constraint set.
* ``shapes``  512x512, 40 shapes (disk or convex polygon with 3..8 vertices, p=0.5)
  of radius U[10,80], 10 with holes, boundary flip p=0.2, 1 % salt and pepper,
  constraint set = 200 distinct object pixels.
* ``large``   4096x4096, 3000 shapes of radius U[5,150], each with a hole with
  probability 0.3, boundary flip p=0.2, 1 % salt and pepper.
* ``batch``   256 images, H and W independent U[128,1024], r uniform in {2..8},
  each drawn with the ``disks`` recipe.
* ``stream``  Poisson arrivals at 2000 frames/s for 10 s, H and W independent
  U[256,2048], r uniform in {2..8}, each frame drawn with the ``disks`` recipe.
"""
from __future__ import annotations

import numpy as np

SEED_DISKS = 1603093371
SEED_SHAPES = 1603093372
SEED_LARGE = 1603093373
SEED_BATCH = 1603093374
SEED_STREAM = 1603093375
SEED_VOLUMES = 1603093376
SEED_GREY = 1603093377


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _paint_disk(img, cy, cx, R, value):
    H, W = img.shape
    y0, y1 = max(0, int(np.floor(cy - R))), min(H, int(np.ceil(cy + R)) + 1)
    x0, x1 = max(0, int(np.floor(cx - R))), min(W, int(np.ceil(cx + R)) + 1)
    if y0 >= y1 or x0 >= x1:
        return
    yy, xx = np.mgrid[y0:y1, x0:x1]
    m = (yy - cy) ** 2 + (xx - cx) ** 2 <= R * R
    img[y0:y1, x0:x1][m] = value


def _paint_polygon(img, cy, cx, R, nv, rng, value):
    """Convex polygon: nv vertices at sorted random angles on a circle of radius R."""
    H, W = img.shape
    ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, size=nv))
    vy = cy + R * np.sin(ang)
    vx = cx + R * np.cos(ang)
    y0, y1 = max(0, int(np.floor(vy.min()))), min(H, int(np.ceil(vy.max())) + 1)
    x0, x1 = max(0, int(np.floor(vx.min()))), min(W, int(np.ceil(vx.max())) + 1)
    if y0 >= y1 or x0 >= x1:
        return
    yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float64)
    inside = np.ones(yy.shape, dtype=bool)
    for k in range(nv):
        ay, ax = vy[k], vx[k]
        by, bx = vy[(k + 1) % nv], vx[(k + 1) % nv]
        # vertices are in counter-clockwise angle order: inside is to the left
        cross = (bx - ax) * (yy - ay) - (by - ay) * (xx - ax)
        inside &= cross >= 0.0
    img[y0:y1, x0:x1][inside] = value


def _boundary_flip(img, p, rng):
    """Flip each pixel that has a 4-neighbour of the other value with probability p."""
    b = np.zeros(img.shape, dtype=bool)
    d = img[1:, :] != img[:-1, :]
    b[1:, :] |= d
    b[:-1, :] |= d
    d = img[:, 1:] != img[:, :-1]
    b[:, 1:] |= d
    b[:, :-1] |= d
    flip = b & (rng.random(img.shape) < p)
    img[flip] ^= 1


def _salt_pepper(img, frac, rng):
    n = int(np.floor(frac * img.size))
    if n == 0:
        return
    idx = rng.choice(img.size, size=n, replace=False)
    flat = img.reshape(-1)
    flat[idx] ^= 1


def draw(H, W, rng, n_shapes, rmin, rmax, p_polygon, n_holes=None, p_hole=None,
         p_flip=0.15, sp_frac=0.005):
    """Draw one image (uint8, values 0/1) with the shape/hole/noise recipe."""
    img = np.zeros((H, W), dtype=np.uint8)
    if n_holes is not None:
        holed = set(rng.choice(n_shapes, size=min(n_holes, n_shapes), replace=False).tolist())
    for k in range(n_shapes):
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        R = rng.uniform(rmin, rmax)
        if p_polygon > 0 and rng.random() < p_polygon:
            nv = int(rng.integers(3, 9))
            _paint_polygon(img, cy, cx, R, nv, rng, 1)
        else:
            _paint_disk(img, cy, cx, R, 1)
        has_hole = (k in holed) if n_holes is not None else (rng.random() < p_hole)
        if has_hole:
            rh = max(2, int(round(rng.uniform(0.3, 0.6) * R)))
            _paint_disk(img, cy, cx, rh, 0)
    _boundary_flip(img, p_flip, rng)
    _salt_pepper(img, sp_frac, rng)
    return img


def disks_image(H, W, rng):
    return draw(H, W, rng, 12, 8, 40, 0.0, n_holes=3, p_flip=0.15, sp_frac=0.005)


def shapes_image(H, W, rng):
    return draw(H, W, rng, 40, 10, 80, 0.5, n_holes=10, p_flip=0.2, sp_frac=0.01)


def constraint_pixels(X, n, rng):
    """Constraint set: n distinct object pixels drawn uniformly from X."""
    obj = np.flatnonzero(X.reshape(-1))
    C = np.zeros(X.size, dtype=np.uint8)
    if obj.size:
        C[rng.choice(obj, size=min(n, obj.size), replace=False)] = 1
    return C.reshape(X.shape)


def workload_disks(seed=SEED_DISKS, H=256, W=256):
    """256x256, r=2, no constraint set."""
    rng = _rng(seed)
    return disks_image(H, W, rng), None, 2


def workload_shapes(seed=SEED_SHAPES, H=512, W=512):
    """512x512, r=5, 200 constrained object pixels."""
    rng = _rng(seed)
    X = shapes_image(H, W, rng)
    C = constraint_pixels(X, 200, rng)
    return X, C, 5


def workload_large(seed=SEED_LARGE, H=4096, W=4096):
    """4096x4096, r=10, no constraint set."""
    rng = _rng(seed)
    X = draw(H, W, rng, 3000, 5, 150, 0.5, p_hole=0.3, p_flip=0.2, sp_frac=0.01)
    return X, None, 10


def batch_item(k, seed=SEED_BATCH, lo=128, hi=1024, rlo=2, rhi=8):
    """Image k of the uneven batch: H, W independent U[lo, hi], r U{rlo..rhi}."""
    rng = _rng(seed * 1000 + k)
    H = int(rng.integers(lo, hi + 1))
    W = int(rng.integers(lo, hi + 1))
    r = int(rng.integers(rlo, rhi + 1))
    return disks_image(H, W, rng), None, r


def workload_batch(n=256, seed=SEED_BATCH, lo=128, hi=1024):
    return [batch_item(k, seed, lo, hi) for k in range(n)]


def stream_schedule(rate=2000.0, seconds=10.0, seed=SEED_STREAM, lo=256, hi=2048):
    """Poisson arrivals: list of (arrival_s, H, W, r, frame_seed)."""
    rng = _rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        H = int(rng.integers(lo, hi + 1))
        W = int(rng.integers(lo, hi + 1))
        r = int(rng.integers(2, 9))
        out.append((t, H, W, r, int(rng.integers(0, 2**62))))
    return out


def stream_frame(H, W, frame_seed):
    return disks_image(H, W, _rng(frame_seed))


def random_binary(H, W, density, seed):
    """Plain Bernoulli image, for edge cases and brute-force checks."""
    rng = _rng(seed)
    return (rng.random((H, W)) < density).astype(np.uint8)


def label_image(H, W, n_labels, seed, n_sites=None, noise=0.01):
    """Label image for the per-label filter: the nearest of n_sites random
    sites (squared distance, ties to the lower site) gives each pixel one of
    n_labels values 0..n_labels-1 (drawn per site), then a fraction `noise`
    of the pixels takes a random label."""
    rng = _rng(seed)
    n_sites = n_sites or 3 * n_labels
    sy = rng.integers(0, H, n_sites)
    sx = rng.integers(0, W, n_sites)
    lab_of = rng.integers(0, n_labels, n_sites).astype(np.uint8)
    ii = np.arange(H)[:, None]
    jj = np.arange(W)[None, :]
    best = np.full((H, W), np.iinfo(np.int64).max, np.int64)
    out = np.zeros((H, W), np.uint8)
    for k in range(n_sites):
        d = (ii - sy[k]) ** 2 + (jj - sx[k]) ** 2
        m = d < best
        best[m] = d[m]
        out[m] = lab_of[k]
    flip = rng.random((H, W)) < noise
    out[flip] = rng.integers(0, n_labels, int(flip.sum())).astype(np.uint8)
    return out


def balls_volume(D, H, W, seed, n=8, noise=0.02):
    """3D stand-in (the paper gives no 3D workload): the union of n balls of
    radius U[3, 0.3 min(D, H, W)] (every third one hollow: a cavity of 0.45
    of its radius), then a fraction `noise` of the voxels flipped."""
    rng = _rng(seed)
    zz, yy, xx = np.mgrid[0:D, 0:H, 0:W]
    V = np.zeros((D, H, W), bool)
    for k in range(n):
        c = rng.uniform(0, (D, H, W))
        R = rng.uniform(3, max(3.5, 0.3 * min(D, H, W)))
        d2 = (zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2
        b = d2 <= R * R
        if k % 3 == 2:
            b &= d2 > (0.45 * R) ** 2
        V |= b
    return (V ^ (rng.random(V.shape) < noise)).astype(np.uint8)


def workload_volumes(n=256, S=64, seed=SEED_VOLUMES, distinct=16):
    """The 3D benchmark workload: n volumes of S^3 (cycling through `distinct`
    drawn ones), r = 3."""
    bank = [balls_volume(S, S, S, seed + k) for k in range(distinct)]
    return [bank[k % distinct] for k in range(n)], 3


def grey_image(H, W, seed, n_bumps=None, noise=6.0):
    """Grey-level stand-in for the watershed (the paper gives no grey-level
    workload): a sum of Gaussian bumps and pits (amplitude U[-1, 1], width
    U[4, max(5, min(H, W) / 4)], about one per 4000 pixels) scaled to 0..255,
    plus Gaussian noise of deviation `noise`, rounded and clipped."""
    rng = _rng(seed)
    n = n_bumps if n_bumps is not None else max(4, (H * W) // 4000)
    yy, xx = np.mgrid[0:H, 0:W]
    F = np.zeros((H, W))
    for _ in range(n):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        s = rng.uniform(4, max(5.0, min(H, W) / 4))
        a = rng.uniform(-1, 1)
        F += a * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
    lo, hi = F.min(), F.max()
    F = (F - lo) / (hi - lo + 1e-12) * (255 - 2 * noise) + noise + rng.normal(0, noise, F.shape)
    return np.clip(np.rint(F), 0, 255).astype(np.uint8)
