"""Pins of the watershed oracle (oracle.wshed, the grey-level W-thinning:
W-destructible pixels -- a lower neighbour, and T-bar = 1 for the binary
image "not lower" against "lower" in the 8-neighbourhood, lower sections
4-connected -- lowered to their largest lower neighbour, in rounds of the four
parity subfields until stable). Pinned to what the definitions fix:
  - the destructibility table against component labelling of the 3 x 3
    neighbourhood (scipy), on all 256 codes;
  - the result is a fixed point (no W-destructible pixel left), only lowers,
    and keeps grey levels of the input;
  - separation: at every level k, each 4-component of the result's lower
    section {F' < k} holds exactly one 4-component of the input's (no merge,
    no new minimum), by labelling (scipy);
  - bit for bit, an independent numpy implementation of the same schedule;
  - closed forms: a constant image is left alone, a cone or a ramp with one
    minimum drains to it;
  - a plausible mistake (lowering to the smallest lower neighbour, or
    counting 8-components of the lower pixels) gives other images."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1603_09337_amd import synth

S4 = ndimage.generate_binary_structure(2, 1)
S8 = ndimage.generate_binary_structure(2, 2)
# neighbour k: E NE N NW W SW S SE, as (row, column) offsets
NB = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]
FOUR = [0, 2, 4, 6]


def tbar_brute(code, structure=S4):
    """4-components (or those of `structure`) of the neighbourhood's lower
    pixels (bits clear) that contain a 4-neighbour of the centre."""
    low = np.zeros((3, 3), bool)
    for k, (dy, dx) in enumerate(NB):
        low[1 + dy, 1 + dx] = not (code >> k) & 1
    lab, _ = ndimage.label(low, structure=structure)
    return len({lab[1 + NB[k][0], 1 + NB[k][1]] for k in FOUR} - {0})


TBAR1 = np.array([tbar_brute(m) == 1 for m in range(256)])
TBAR1_8 = np.array([tbar_brute(m, S8) == 1 for m in range(256)])


def codes_and_delta(F):
    """Per pixel: the code (bit k: neighbour k is not lower, or outside) and
    the largest lower neighbour level (-1 if none)."""
    H, W = F.shape
    P = np.full((H + 2, W + 2), 256, np.int32)
    P[1:-1, 1:-1] = F
    v = P[1:-1, 1:-1]
    code = np.zeros((H, W), np.int32)
    delta = np.full((H, W), -1, np.int32)
    for k, (dy, dx) in enumerate(NB):
        n = P[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
        code |= (n >= v).astype(np.int32) << k
        delta = np.where(n < v, np.maximum(delta, n), delta)
    return code, delta


def schedule_numpy(F, table=TBAR1, lower_to="max"):
    F = F.astype(np.int32).copy()
    H, W = F.shape
    while True:
        changed = False
        for s in range(4):
            si, sj = s >> 1, s & 1
            code, delta = codes_and_delta(F)
            if lower_to == "min":
                Pm = np.full((H + 2, W + 2), 256, np.int32)
                Pm[1:-1, 1:-1] = F
                mn = np.full((H, W), 256, np.int32)
                for dy, dx in NB:
                    n = Pm[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
                    mn = np.minimum(mn, n)
                delta = np.where(delta >= 0, mn, -1)
            sel = np.zeros((H, W), bool)
            sel[si::2, sj::2] = True
            go = sel & (delta >= 0) & table[code]
            if go.any():
                F[go] = delta[go]
                changed = True
        if not changed:
            return F.astype(np.uint8)


def separation_ok(F0, F1):
    for k in np.unique(np.concatenate([F0.ravel(), F1.ravel()])).astype(int) + 1:
        lab1, n1 = ndimage.label(F1 < k, structure=S4)
        lab0, n0 = ndimage.label(F0 < k, structure=S4)
        if n1 == 0:
            continue
        # the input's components inside each result component
        pairs = np.unique(np.stack([lab1[F0 < k], lab0[F0 < k]]), axis=1)
        per = np.bincount(pairs[0], minlength=n1 + 1)[1:]
        if not (per == 1).all():
            return False
    return True


def test_destructibility_table_is_the_definition():
    for m in range(256):
        T, Tb = oracle.topo_numbers(8, m)
        assert (Tb == 1) == TBAR1[m], m
    # the 4- and 8-adjacent readings of the lower pixels differ on some codes
    assert (TBAR1 != TBAR1_8).any()


IMAGES = [
    ("grey", 40, 50, 1), ("grey", 1, 60, 2), ("grey", 70, 1, 3), ("grey", 33, 33, 4),
    ("grey", 64, 96, 5), ("rand", 30, 30, 6), ("rand", 17, 41, 7), ("grey", 120, 90, 8),
]


def _image(kind, H, W, seed):
    if kind == "grey":
        return synth.grey_image(H, W, 4000 + seed)
    return np.random.default_rng(seed).integers(0, 12, (H, W)).astype(np.uint8)


@pytest.mark.parametrize("case", IMAGES)
def test_fixed_point_lower_only_same_levels_and_separation(case):
    F = _image(*case)
    G = oracle.wshed(F)
    assert (G <= F).all()
    assert set(np.unique(G)) <= set(np.unique(F))
    code, delta = codes_and_delta(G)
    assert not ((delta >= 0) & TBAR1[code]).any(), "a W-destructible pixel is left"
    assert separation_ok(F, G)


@pytest.mark.parametrize("case", IMAGES)
def test_equals_an_independent_schedule(case):
    F = _image(*case)
    assert np.array_equal(oracle.wshed(F), schedule_numpy(F))


def test_closed_forms():
    C = np.full((20, 30), 77, np.uint8)
    assert np.array_equal(oracle.wshed(C), C)
    yy, xx = np.mgrid[0:41, 0:37]
    cone = (np.abs(yy - 20) + np.abs(xx - 11)).astype(np.uint8)
    assert (oracle.wshed(cone) == 0).all()
    ramp = np.tile(np.arange(60, dtype=np.uint8), (25, 1))
    assert (oracle.wshed(ramp) == 0).all()
    # two minima: two basins at their levels and a divide between them
    two = np.minimum(np.abs(yy - 20) + np.abs(xx - 5), 3 + np.abs(yy - 20) + np.abs(xx - 31)).astype(np.uint8)
    G = oracle.wshed(two)
    assert separation_ok(two, G)
    lab, n = ndimage.label(G < G.max(), structure=S4)
    assert n == 2


def test_plausible_mistakes_differ():
    F = synth.grey_image(60, 70, 4100)
    G = oracle.wshed(F)
    assert not np.array_equal(G, schedule_numpy(F, lower_to="min"))
    assert not np.array_equal(G, schedule_numpy(F, table=TBAR1_8))
