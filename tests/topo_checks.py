"""Independent checks used to pin the oracle: brute force, textbook formulas and
topological invariants, written with numpy/scipy only (nothing from oracle/ or
from the HIP library)."""
from __future__ import annotations

import numpy as np
from scipy import ndimage

# neighbour k -> (dy, dx): E NE N NW W SW S SE
NB = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]

EIGHT = np.ones((3, 3), dtype=int)
FOUR = ndimage.generate_binary_structure(2, 1)


def yokoi_simple(m: int) -> bool:
    """Yokoi's 8-connectivity number N8 = sum over the 4-neighbours k of
    xb_k - xb_k * xb_{k+1} * xb_{k+2} (xb = 1 - x, indices mod 8 counter-clockwise
    from E); an object point is (8,4)-simple iff N8 == 1."""
    x = [(m >> k) & 1 for k in range(8)]
    xb = [1 - v for v in x]
    n8 = sum(xb[k] - xb[k] * xb[(k + 1) % 8] * xb[(k + 2) % 8] for k in (0, 2, 4, 6))
    return n8 == 1


def global_simple(m: int) -> bool:
    """Global definition of a simple point (Sec. 2): removing x from X changes
    the number of 8-components of X and of 4-components of the complement by
    nothing. Evaluated on the 3x3 configuration padded with background."""
    img = np.zeros((5, 5), dtype=np.uint8)
    img[2, 2] = 1
    for k, (dy, dx) in enumerate(NB):
        img[2 + dy, 2 + dx] = (m >> k) & 1
    before_o = ndimage.label(img, EIGHT)[1]
    before_b = ndimage.label(1 - img, FOUR)[1]
    img[2, 2] = 0
    after_o = ndimage.label(img, EIGHT)[1]
    after_b = ndimage.label(1 - img, FOUR)[1]
    return before_o == after_o and before_b == after_b


def neighbourhood_codes(S: np.ndarray) -> np.ndarray:
    """Code m of every pixel (outside the window = background)."""
    H, W = S.shape
    P = np.zeros((H + 2, W + 2), dtype=np.uint16)
    P[1:-1, 1:-1] = S != 0
    m = np.zeros((H, W), dtype=np.uint16)
    for k, (dy, dx) in enumerate(NB):
        m |= P[1 + dy:1 + dy + H, 1 + dx:1 + dx + W] << k
    return m


def simple_mask(S: np.ndarray) -> np.ndarray:
    table = np.array([yokoi_simple(m) for m in range(256)], dtype=bool)
    return table[neighbourhood_codes(S)]


def components8(X: np.ndarray) -> int:
    return ndimage.label(X != 0, EIGHT)[1]


def components4_complement(X: np.ndarray) -> int:
    """4-components of the complement, the outside of the window included
    (one pixel of background padding joins everything that touches the border)."""
    P = np.ones((X.shape[0] + 2, X.shape[1] + 2), dtype=np.uint8)
    P[1:-1, 1:-1] = X == 0
    return ndimage.label(P, FOUR)[1]


def euler84_quads(X: np.ndarray) -> int:
    """Euler number of X under 8-adjacency from Gray's 2x2 quad counts:
    E = (n(Q1) - n(Q3) - 2 n(QD)) / 4 on the image padded with background."""
    P = np.zeros((X.shape[0] + 2, X.shape[1] + 2), dtype=np.int32)
    P[1:-1, 1:-1] = X != 0
    a, b, c, d = P[:-1, :-1], P[:-1, 1:], P[1:, :-1], P[1:, 1:]
    s = a + b + c + d
    q1 = int((s == 1).sum())
    q3 = int((s == 3).sum())
    qd = int(((s == 2) & (a == d)).sum())
    e4 = q1 - q3 - 2 * qd
    assert e4 % 4 == 0
    return e4 // 4


def topology(X: np.ndarray):
    return components8(X), components4_complement(X), euler84_quads(X)


def edt_brute(F: np.ndarray, frame: bool) -> np.ndarray:
    """O(N^2) brute force: min over feature pixels (and, with frame, over the
    one-pixel ring just outside the window) of the squared distance."""
    H, W = F.shape
    pts = np.argwhere(F != 0)
    if frame:
        ring = [(-1, j) for j in range(-1, W + 1)] + [(H, j) for j in range(-1, W + 1)] + \
               [(i, -1) for i in range(H)] + [(i, W) for i in range(H)]
        pts = np.concatenate([pts.reshape(-1, 2), np.array(ring, dtype=np.int64)])
    if pts.size == 0:
        return np.full((H, W), np.iinfo(np.uint32).max, dtype=np.uint32)
    ii, jj = np.mgrid[0:H, 0:W]
    d = (ii[..., None] - pts[:, 0]) ** 2 + (jj[..., None] - pts[:, 1]) ** 2
    return d.min(axis=-1).astype(np.uint32)


def ball_offsets(r: int):
    return [(a, b) for a in range(-r, r + 1) for b in range(-r, r + 1) if a * a + b * b <= r * r]


def dilate_stamp(X: np.ndarray, r: int) -> np.ndarray:
    """Dilation by the Euclidean ball B_r (Sec. 2), restricted to the window."""
    H, W = X.shape
    out = np.zeros((H, W), dtype=bool)
    for a, b in ball_offsets(r):
        ys0, ys1 = max(0, -a), min(H, H - a)
        xs0, xs1 = max(0, -b), min(W, W - b)
        if ys0 < ys1 and xs0 < xs1:
            out[ys0 + a:ys1 + a, xs0 + b:xs1 + b] |= X[ys0:ys1, xs0:xs1] != 0
    return out


def erode_stamp(X: np.ndarray, r: int) -> np.ndarray:
    """Erosion by B_r as the dual of dilation: points whose whole ball lies in X
    (the outside of the window is background)."""
    H, W = X.shape
    out = X != 0
    for a, b in ball_offsets(r):
        sh = np.zeros((H, W), dtype=bool)
        ys0, ys1 = max(0, a), min(H, H + a)
        xs0, xs1 = max(0, b), min(W, W + b)
        if ys0 < ys1 and xs0 < xs1:
            sh[ys0 - a:ys1 - a, xs0 - b:xs1 - b] = X[ys0:ys1, xs0:xs1] != 0
        out &= sh
    return out


def opening(X, r):
    return dilate_stamp(erode_stamp(X, r).astype(np.uint8), r)


def closing(X, r):
    return erode_stamp(dilate_stamp(X, r).astype(np.uint8), r)


def disk_image(R: int, margin: int = 12) -> np.ndarray:
    n = 2 * R + 1 + 2 * margin
    c = R + margin
    ii, jj = np.mgrid[0:n, 0:n]
    return (((ii - c) ** 2 + (jj - c) ** 2) <= R * R).astype(np.uint8)


def sequential_schedule(mode: int, S: np.ndarray, B, P: np.ndarray, table=None) -> np.ndarray:
    """Second, structurally different implementation of the distance-ordered
    subfield schedule: inside each subfield pass, points are updated in place in
    raster order (no separate deletion list). Same result as the simultaneous
    pass because two points of one subfield are never 8-adjacent. table: the
    simple-point predicate per neighbourhood code (default: (8,4), Yokoi)."""
    S = (np.asarray(S) != 0).astype(np.uint8).copy()
    H, W = S.shape
    Bm = np.zeros((H, W), dtype=bool) if B is None else (np.asarray(B) != 0)
    if table is None:
        table = [yokoi_simple(m) for m in range(256)]
    cand = (S == 1) & ~Bm if mode == 0 else (S == 0) & Bm
    levels = sorted(set(P[cand].tolist()))

    def code(i, j):
        m = 0
        for k, (dy, dx) in enumerate(NB):
            y, x = i + dy, j + dx
            if 0 <= y < H and 0 <= x < W and S[y, x]:
                m |= 1 << k
        return m

    for d in levels:
        while True:
            changed = False
            for si, sj in ((0, 0), (0, 1), (1, 0), (1, 1)):
                for i in range(si, H, 2):
                    for j in range(sj, W, 2):
                        if P[i, j] > d:
                            continue
                        if mode == 0 and S[i, j] and not Bm[i, j] and table[code(i, j)]:
                            S[i, j] = 0
                            changed = True
                        elif mode == 1 and not S[i, j] and Bm[i, j] and table[code(i, j)]:
                            S[i, j] = 1
                            changed = True
            if not changed:
                break
    return S


# the (4,8) pair: object 4-adjacency, background 8-adjacency (Sec. 2)
def components4(X: np.ndarray) -> int:
    return ndimage.label(X != 0, FOUR)[1]


def components8_complement(X: np.ndarray) -> int:
    """8-components of the complement, the outside of the window included."""
    P = np.ones((X.shape[0] + 2, X.shape[1] + 2), dtype=np.uint8)
    P[1:-1, 1:-1] = X == 0
    return ndimage.label(P, EIGHT)[1]


def euler48_quads(X: np.ndarray) -> int:
    """Euler number of X under 4-adjacency from Gray's 2x2 quad counts:
    E = (n(Q1) - n(Q3) + 2 n(QD)) / 4 on the image padded with background."""
    P = np.zeros((X.shape[0] + 2, X.shape[1] + 2), dtype=np.int32)
    P[1:-1, 1:-1] = X != 0
    a, b, c, d = P[:-1, :-1], P[:-1, 1:], P[1:, :-1], P[1:, 1:]
    s = a + b + c + d
    q1 = int((s == 1).sum())
    q3 = int((s == 3).sum())
    qd = int(((s == 2) & (a == d)).sum())
    e4 = q1 - q3 + 2 * qd
    assert e4 % 4 == 0
    return e4 // 4


def topology48(X: np.ndarray):
    return components4(X), components8_complement(X), euler48_quads(X)


def global_simple48(m: int) -> bool:
    """The global definition for the (4,8) pair: removing x changes neither the
    number of 4-components of X nor that of 8-components of the complement, on
    the 3x3 configuration padded with background."""
    img = np.zeros((5, 5), dtype=np.uint8)
    img[2, 2] = 1
    for k, (dy, dx) in enumerate(NB):
        img[2 + dy, 2 + dx] = (m >> k) & 1
    before_o = ndimage.label(img, FOUR)[1]
    before_b = ndimage.label(1 - img, EIGHT)[1]
    img[2, 2] = 0
    after_o = ndimage.label(img, FOUR)[1]
    after_b = ndimage.label(1 - img, EIGHT)[1]
    return before_o == after_o and before_b == after_b


# ---------------------------------------------------------------------------
# An independent composition of the cutting HC_i and the filling HF_i (Sec. 2,
# eq. (i) and eq. (ii)) from parts that share nothing with the oracle: ball
# stamping for the thresholds, scipy's exact Euclidean transform (nearest
# feature indices, squared distances in integers) for the priorities, and a
# numpy subfield schedule. It fixes which distance map orders each of the four
# thinnings and thickenings of a radius:
#   HC thinning    priority d^2(., complement of X u outside)
#   HC thickening  priority d^2(., Y), Y the thinned set
#   HF thickening  priority d^2(., X)
#   HF thinning    priority d^2(., complement of Z u outside), Z the thickened set
# ---------------------------------------------------------------------------
def edt_sq_lib(F: np.ndarray, frame: bool) -> np.ndarray:
    """Squared distance to the nearest nonzero pixel of F (with frame: or to
    any pixel outside the window), from scipy's exact transform: the nearest
    feature's indices give the distance in integers."""
    H, W = F.shape
    if frame:
        G = np.ones((H + 2, W + 2), dtype=bool)
        G[1:-1, 1:-1] = F != 0
        off = 1
    else:
        G = F != 0
        off = 0
    if not G.any():
        return np.full((H, W), np.iinfo(np.uint32).max, dtype=np.uint32)
    _, ind = ndimage.distance_transform_edt(~G, return_indices=True)
    ii, jj = np.mgrid[0:G.shape[0], 0:G.shape[1]]
    d2 = (ii - ind[0]) ** 2 + (jj - ind[1]) ** 2
    return d2[off:off + H, off:off + W].astype(np.uint32)


def schedule_np(mode: int, S: np.ndarray, B, P: np.ndarray, table) -> np.ndarray:
    """The distance-ordered subfield schedule with whole-subfield numpy passes:
    levels = distinct P over the candidates, ascending; at level d, rounds of
    the passes (even,even) (even,odd) (odd,even) (odd,odd) over the points with
    P <= d until a round changes nothing. mode 0 deletes simple points of
    S \\ B, mode 1 adds simple points of B \\ S."""
    S = (np.asarray(S) != 0).astype(np.uint8).copy()
    H, W = S.shape
    Bm = np.zeros((H, W), dtype=bool) if B is None else (np.asarray(B) != 0)
    tab = np.asarray(table, dtype=bool)
    cand = (S == 1) & ~Bm if mode == 0 else (S == 0) & Bm
    ii, jj = np.mgrid[0:H, 0:W]
    par = [((ii % 2) == si) & ((jj % 2) == sj) for si, sj in ((0, 0), (0, 1), (1, 0), (1, 1))]
    for d in np.unique(P[cand]):
        act = P <= d
        while True:
            changed = False
            for sub in par:
                ok = tab[neighbourhood_codes(S)]
                if mode == 0:
                    hit = sub & act & (S == 1) & ~Bm & ok
                else:
                    hit = sub & act & (S == 0) & Bm & ok
                if hit.any():
                    S[hit] = mode
                    changed = True
            if not changed:
                break
    return S


def simple_table(n: int = 8):
    return [global_simple(m) if n == 8 else global_simple48(m) for m in range(256)]


def hc_composed(X, C, i: int, table):
    """HC_i (eq. (i)): Y = H(X, eps_i(X) u C) ordered by d^2 to the background
    (outside included); X' = *H(Y, delta_i(Y) n X) ordered by d^2 to Y.
    Returns (Y, X')."""
    X = (np.asarray(X) != 0).astype(np.uint8)
    K = erode_stamp(X, i) | (np.zeros(X.shape, bool) if C is None else (np.asarray(C) != 0))
    Y = schedule_np(0, X, K, edt_sq_lib(X == 0, True), table)
    V = dilate_stamp(Y, i) & (X != 0)
    return Y, schedule_np(1, Y, V, edt_sq_lib(Y, False), table)


def hf_composed(X, D, i: int, table):
    """HF_i (eq. (ii), W read as eps_i(Z) u X): Z = *H(X, delta_i(X) \\ D)
    ordered by d^2 to X; X' = H(Z, eps_i(Z) u X) ordered by d^2 to the
    background of Z (outside included). Returns (Z, X')."""
    X = (np.asarray(X) != 0).astype(np.uint8)
    L = dilate_stamp(X, i) & ~(np.zeros(X.shape, bool) if D is None else (np.asarray(D) != 0))
    Z = schedule_np(1, X, L, edt_sq_lib(X, False), table)
    Wc = erode_stamp(Z, i) | (X != 0)
    return Z, schedule_np(0, Z, Wc, edt_sq_lib(Z == 0, True), table)


def hasf_composed(X, C, D, r: int, n: int = 8, order: int = 0):
    """HASF of order r from the parts above: per radius HC_i then HF_i (order
    0) or HF_i then HC_i (order 1), with C <- C n X and D <- D \\ X taken from
    the input. Returns an (r, 4, H, W) array of the states in the order they
    are produced (thinned, cut, thickened, filled for order 0)."""
    X = (np.asarray(X) != 0).astype(np.uint8)
    Cn = None if C is None else ((np.asarray(C) != 0) & (X != 0))
    Dn = None if D is None else ((np.asarray(D) != 0) & (X == 0))
    table = simple_table(n)
    out = []
    x = X
    for i in range(1, r + 1):
        st = []
        ops = (("c", "f") if order == 0 else ("f", "c"))
        for op in ops:
            if op == "c":
                a, x = hc_composed(x, Cn, i, table)
            else:
                a, x = hf_composed(x, Dn, i, table)
            st += [a, x]
        out.append(np.stack(st))
    return np.stack(out) if out else np.zeros((0, 4) + X.shape, np.uint8)


def hasf_inf_composed(X, C, D, n: int = 8, order: int = 0, r_max: int = 0):
    """"r = infinity" from the parts above: radii 1, 2, ... until the first
    radius that leaves the set unchanged, at most r_max (0: the least i with
    i^2 >= (H-1)^2 + (W-1)^2, past which the thresholds and level tests of a
    radius no longer depend on it). Returns (result, last radius applied)."""
    x = (np.asarray(X) != 0).astype(np.uint8)
    H, W = x.shape
    Cn = None if C is None else ((np.asarray(C) != 0) & (x != 0))
    Dn = None if D is None else ((np.asarray(D) != 0) & (x == 0))
    cap = r_max if r_max > 0 else int(np.ceil(np.sqrt((H - 1) ** 2 + (W - 1) ** 2 - 1e-9)))
    cap = max(cap, 1)
    table = simple_table(n)
    i = 0
    for i in range(1, cap + 1):
        prev = x
        for op in (("c", "f") if order == 0 else ("f", "c")):
            x = hc_composed(x, Cn, i, table)[1] if op == "c" else hf_composed(x, Dn, i, table)[1]
        x = x.astype(np.uint8)
        if np.array_equal(x, prev):
            break
    return x, i
