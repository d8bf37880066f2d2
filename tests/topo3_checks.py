"""Independent 3D checks for the oracle's (26,6) filter: topology of a volume
by component labelling (scipy) and the Euler characteristic of its voxel
complex, ball stamping, brute-force distances and a raster-order schedule.
Nothing here is shared with the oracle."""
import functools

import numpy as np
from scipy import ndimage

S26 = np.ones((3, 3, 3), dtype=bool)
S6 = ndimage.generate_binary_structure(3, 1)


def offsets26():
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dz, dy, dx) != (0, 0, 0)]


OFF26 = offsets26()


def euler3(V):
    """Euler characteristic of the union of the closed unit cubes of the
    object voxels: vertices - edges + faces - cubes of the cubical complex."""
    v = np.pad(np.asarray(V) != 0, 1)
    C = int(v.sum())
    # faces: normal to axis a, between voxel layers k-1 and k along a
    F = 0
    for a in range(3):
        F += int(np.logical_or(np.take(v, range(0, v.shape[a] - 1), axis=a),
                               np.take(v, range(1, v.shape[a]), axis=a)).sum())
    # edges parallel to axis a: any of the 4 voxels around it in the other two axes
    E = 0
    for a in range(3):
        b, c = [x for x in range(3) if x != a]
        w = np.moveaxis(v, (a, b, c), (0, 1, 2))
        E += int((w[:, :-1, :-1] | w[:, 1:, :-1] | w[:, :-1, 1:] | w[:, 1:, 1:]).sum())
    Vt = int((v[:-1, :-1, :-1] | v[1:, :-1, :-1] | v[:-1, 1:, :-1] | v[:-1, :-1, 1:] | v[1:, 1:, :-1]
              | v[1:, :-1, 1:] | v[:-1, 1:, 1:] | v[1:, 1:, 1:]).sum())
    return Vt - E + F - C


def topology3(V):
    """(26-components of the object, 6-components of the background with the
    outside of the box, Euler characteristic)."""
    v = np.asarray(V) != 0
    _, n_obj = ndimage.label(v, structure=S26)
    bg = np.pad(~v, 1, constant_values=True)
    _, n_bg = ndimage.label(bg, structure=S6)
    return n_obj, n_bg, euler3(v)


def code_of(S, z, y, x):
    D, H, W = S.shape
    code = 0
    for b, (dz, dy, dx) in enumerate(OFF26):
        zz, yy, xx = z + dz, y + dy, x + dx
        if 0 <= zz < D and 0 <= yy < H and 0 <= xx < W and S[zz, yy, xx]:
            code |= 1 << b
    return code


@functools.lru_cache(maxsize=None)
def simple_by_topology(code: int) -> bool:
    """x is simple iff removing it from X leaves the topology of X unchanged:
    the same number of object 26-components and background 6-components and
    the same Euler characteristic, evaluated on the 3x3x3 neighbourhood with
    x set, inside an empty 5x5x5 box."""
    box = np.zeros((5, 5, 5), dtype=bool)
    for b, (dz, dy, dx) in enumerate(OFF26):
        box[2 + dz, 2 + dy, 2 + dx] = (code >> b) & 1
    box[2, 2, 2] = True
    before = topology3(box)
    box[2, 2, 2] = False
    return topology3(box) == before


def ball_offsets3(r):
    return [(a, b, c) for a in range(-r, r + 1) for b in range(-r, r + 1) for c in range(-r, r + 1)
            if a * a + b * b + c * c <= r * r]


def dilate3(X, r):
    D, H, W = X.shape
    out = np.zeros(X.shape, bool)
    x = np.asarray(X) != 0
    for a, b, c in ball_offsets3(r):
        z0, z1 = max(0, -a), min(D, D - a)
        y0, y1 = max(0, -b), min(H, H - b)
        x0, x1 = max(0, -c), min(W, W - c)
        if z0 < z1 and y0 < y1 and x0 < x1:
            out[z0 + a:z1 + a, y0 + b:y1 + b, x0 + c:x1 + c] |= x[z0:z1, y0:y1, x0:x1]
    return out


def erode3(X, r):
    """points whose whole ball lies in X (outside the box is background)"""
    D, H, W = X.shape
    x = np.asarray(X) != 0
    out = x.copy()
    for a, b, c in ball_offsets3(r):
        sh = np.zeros(X.shape, bool)
        z0, z1 = max(0, a), min(D, D + a)
        y0, y1 = max(0, b), min(H, H + b)
        x0, x1 = max(0, c), min(W, W + c)
        if z0 < z1 and y0 < y1 and x0 < x1:
            sh[z0 - a:z1 - a, y0 - b:y1 - b, x0 - c:x1 - c] = x[z0:z1, y0:y1, x0:x1]
        out &= sh
    return out


def edt3_brute(F, frame):
    D, H, W = F.shape
    pts = np.argwhere(np.asarray(F) != 0)
    zz, yy, xx = np.mgrid[0:D, 0:H, 0:W]
    best = np.full(F.shape, np.iinfo(np.int64).max, dtype=np.int64)
    for (a, b, c) in pts:
        best = np.minimum(best, (zz - a) ** 2 + (yy - b) ** 2 + (xx - c) ** 2)
    if frame:
        e = np.minimum.reduce([zz + 1, D - zz, yy + 1, H - yy, xx + 1, W - xx])
        best = np.minimum(best, e * e)
    best[best == np.iinfo(np.int64).max] = np.iinfo(np.uint32).max
    return best.astype(np.uint32)


def schedule3_raster(mode, S, B, P, simple):
    """The 3D schedule with voxels of a subfield taken one at a time in raster
    order on the current state (equal to the simultaneous pass, since voxels
    of one subfield are never 26-adjacent)."""
    S = (np.asarray(S) != 0).astype(np.uint8).copy()
    Bm = np.zeros(S.shape, bool) if B is None else np.asarray(B) != 0
    D, H, W = S.shape
    cand = (S == 1) & ~Bm if mode == 0 else (S == 0) & Bm
    for d in np.unique(P[cand]):
        while True:
            changed = False
            for s in range(8):
                pz, py, px = s >> 2, (s >> 1) & 1, s & 1
                for z in range(pz, D, 2):
                    for y in range(py, H, 2):
                        for x in range(px, W, 2):
                            c = (S[z, y, x] == 1 and not Bm[z, y, x]) if mode == 0 else \
                                (S[z, y, x] == 0 and Bm[z, y, x])
                            if c and P[z, y, x] <= d and simple(code_of(S, z, y, x)):
                                S[z, y, x] = mode
                                changed = True
            if not changed:
                break
    return S


def edt3_lib(F, frame):
    """Squared distance to the nearest nonzero voxel (and, with frame, the
    outside of the box) from scipy's exact transform: the nearest feature's
    indices give the distance in integers."""
    D, H, W = F.shape
    if frame:
        G = np.ones((D + 2, H + 2, W + 2), dtype=bool)
        G[1:-1, 1:-1, 1:-1] = np.asarray(F) != 0
        off = 1
    else:
        G = np.asarray(F) != 0
        off = 0
    if not G.any():
        return np.full(F.shape, np.iinfo(np.uint32).max, dtype=np.uint32)
    _, ind = ndimage.distance_transform_edt(~G, return_indices=True)
    zz, yy, xx = np.mgrid[0:G.shape[0], 0:G.shape[1], 0:G.shape[2]]
    d2 = (zz - ind[0]) ** 2 + (yy - ind[1]) ** 2 + (xx - ind[2]) ** 2
    return d2[off:off + D, off:off + H, off:off + W].astype(np.uint32)


def hasf3_composed(X, C, r):
    """The 3D filter from the parts above (ball stamping, scipy's transform,
    the raster schedule with the global definition of a simple voxel): per
    radius HC_i (thin by the distance to the background and the outside,
    keeping eps_i(X) u C; thicken inside delta_i(Y) n X by the distance to Y)
    then HF_i (thicken inside delta_i(X) by the distance to X; thin keeping
    eps_i(Z) u X by the distance to the background of Z and the outside).
    Returns an (r, 4, D, H, W) stage array."""
    x = (np.asarray(X) != 0).astype(np.uint8)
    Cn = np.zeros(x.shape, bool) if C is None else (np.asarray(C) != 0) & (x != 0)
    simple = simple_by_topology
    out = []
    for i in range(1, r + 1):
        K = erode3(x, i) | Cn
        Y = schedule3_raster(0, x, K, edt3_lib(x == 0, True), simple)
        Xc = schedule3_raster(1, Y, dilate3(Y, i) & (x != 0), edt3_lib(Y, False), simple)
        Z = schedule3_raster(1, Xc, dilate3(Xc, i), edt3_lib(Xc, False), simple)
        Xf = schedule3_raster(0, Z, erode3(Z, i) | (Xc != 0), edt3_lib(Z == 0, True), simple)
        out.append(np.stack([Y, Xc, Z, Xf]))
        x = Xf
    return np.stack(out)
