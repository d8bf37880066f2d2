"""Parity of the row-tile path (one large image over row tiles whose state
stays in LDS, halo rows exchanged every two rounds) with the oracle, bit
exact. Contexts with grid_min_pixels = 1 and a chosen tile_rows send small,
ragged and degenerate images down this path with many tiles (down to tiles
of 8 own rows and a last tile shorter than the halo), so the exchange and the
level ends decided across tiles are checked at sizes the oracle finishes
quickly. The grid kernel (tile_rows = -1) and the tiles run the same
schedule: besides equal images, they report the same number of rounds and
activated levels."""
import numpy as np
import pytest

import oracle
import topo_checks as tc
from gpu_util import dev, host, say
from paper_1603_09337_amd import hasf, synth

pytestmark = pytest.mark.gpu

_CTX = {}


def tctx(th):
    """Every image on the large-image path: row tiles of th rows (-1: the grid kernel)."""
    if th not in _CTX:
        _CTX[th] = hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1, tile_rows=th, tile_halo=12)
    return _CTX[th]


def _filter(c, X, C, r, pitch=None, D=None, n=8, order=0):
    d = dev(X, pitch)
    cd = dev(C, pitch) if C is not None else None
    dd = dev(D, pitch) if D is not None else None
    c.filter(d, cd, r, D=dd, conn=n, order=order)
    c.sync()
    return host(d)


TILE_CASES = [
    # (H, W, r, density, with C, tile rows, seed)
    (40, 90, 2, 0.6, False, 8, 1),     # five tiles of 8 rows
    (37, 130, 3, 0.55, True, 8, 2),    # last tile of 5 rows, shorter than the halo
    (64, 64, 5, 0.5, False, 16, 3),
    (100, 300, 4, 0.45, True, 10, 4),
    (257, 65, 6, 0.5, False, 32, 5),   # odd height
    (129, 191, 8, 0.5, True, 24, 6),
    (300, 200, 3, 0.5, False, 8, 7),   # 38 tiles
    (18, 700, 2, 0.5, False, 8, 8),    # three tiles, wide rows
    (90, 1000, 3, 0.5, True, 30, 9),
    (61, 77, 12, 0.5, True, 8, 10),    # radius beyond the halo
]


@pytest.mark.parametrize("case", TILE_CASES)
def test_tiles_random(case):
    H, W, r, dens, withC, th, seed = case
    X = synth.random_binary(H, W, dens, 700 + seed)
    C = synth.random_binary(H, W, 0.05, 750 + seed) if withC else None
    say("tiles random", case)
    assert np.array_equal(_filter(tctx(th), X, C, r), oracle.hasf(X, C, r))


@pytest.mark.parametrize("th", [8, 32])
def test_tiles_disks_and_shapes_workloads(th):
    X, C, r = synth.workload_disks()
    say("tiles of %d rows, 256x256 r=2" % th)
    assert np.array_equal(_filter(tctx(th), X, C, r), oracle.hasf(X, C, r))
    X, C, r = synth.workload_shapes()
    say("tiles of %d rows, 512x512 r=5, C = 200 px" % th)
    assert np.array_equal(_filter(tctx(th), X, C, r), oracle.hasf(X, C, r))


def test_tiles_background_constraint_pairs_and_order():
    X = synth.disks_image(150, 170, np.random.default_rng(11))
    C = synth.random_binary(150, 170, 0.03, 12)
    rng = np.random.default_rng(13)
    D = ((rng.random(X.shape) < 0.3) & (X == 0)).astype(np.uint8)
    for n in (8, 4):
        for order in (0, 1):
            say("tiles with C and D, pair", n, "order", order)
            got = _filter(tctx(8), X, C, 4, D=D, n=n, order=order)
            assert np.array_equal(got, oracle.hasf(X, C, 4, D=D, n=n, order=order))


def test_tiles_pitch_r0_empty_full():
    X = synth.disks_image(90, 140, np.random.default_rng(3))
    say("tiles pitch, r = 0, empty, full")
    assert np.array_equal(_filter(tctx(8), X, None, 3, pitch=201), oracle.hasf(X, None, 3))
    assert np.array_equal(_filter(tctx(8), X, None, 0), (X != 0).astype(np.uint8))
    Z = np.zeros((70, 80), np.uint8)
    assert np.array_equal(_filter(tctx(8), Z, None, 4), Z)
    F = np.ones((70, 80), np.uint8)
    assert np.array_equal(_filter(tctx(8), F, None, 4), oracle.hasf(F, None, 4))


def test_tiles_and_grid_run_the_same_schedule():
    X, _, _ = synth.workload_disks(H=700, W=1000)
    exp = oracle.hasf(X, None, 3)
    counts = {}
    for th in (-1, 8, 32, 64):
        c = tctx(th)
        c.grid_counts(reset=True)
        say("700x1000 r=3, tile rows", th)
        assert np.array_equal(_filter(c, X, None, 3), exp), th
        counts[th] = c.grid_counts(reset=True)
        assert counts[th]["launches"] == 1
    for th in (8, 32, 64):
        assert counts[th]["rounds"] == counts[-1]["rounds"], counts
        assert counts[th]["levels"] == counts[-1]["levels"], counts
        # one barrier per two rounds at most, against one per pass
        assert counts[th]["barriers"] < counts[-1]["barriers"] / 2, counts


def test_batch_with_tile_and_workgroup_images():
    c = hasf.Context(0, batch_grid_min_pixels=60000, tile_rows=8)
    items = [synth.batch_item(k, lo=60, hi=420) for k in range(10)]
    dX = [dev(X) for X, _, _ in items]
    say("batch, tile and workgroup images:", sum(X.size >= 60000 for X, _, _ in items), "on tiles")
    c.filter_batch([(d, None, r) for d, (_, _, r) in zip(dX, items)])
    c.sync()
    for k, ((X, C, r), d) in enumerate(zip(items, dX)):
        assert np.array_equal(host(d), oracle.hasf(X, C, r)), "image %d" % k


def test_tiles_keep_topology_on_a_2048_square():
    X = synth.workload_disks(H=2048, W=2048)[0]
    say("2048x2048 r=6 on tiles and on the grid kernel")
    a = _filter(tctx(32), X, None, 6)
    b = _filter(tctx(-1), X, None, 6)
    assert np.array_equal(a, b)
    assert tc.topology(a) == tc.topology(X)


def test_bad_tile_rows_is_refused():
    for th in (-2, 2, 3, 7, 9):
        with pytest.raises(hasf.HasfError):
            hasf.Context(0, tile_rows=th)


_HCTX = {}


@pytest.mark.parametrize("halo", [4, 12, 16, 24, 32])
def test_tiles_other_halo_depths(halo):
    # halo / 4 rounds between exchanges; tiles at least as tall as the halo
    if halo not in _HCTX:
        _HCTX[halo] = hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1, tile_rows=8, tile_halo=halo)
    c = _HCTX[halo]
    for (H, W, r, dens, withC, seed) in [(37, 130, 3, 0.55, True, 21), (129, 191, 6, 0.5, True, 22),
                                         (300, 200, 4, 0.5, False, 23)]:
        X = synth.random_binary(H, W, dens, 800 + seed)
        C = synth.random_binary(H, W, 0.05, 850 + seed) if withC else None
        say("tiles, halo", halo, (H, W, r))
        assert np.array_equal(_filter(c, X, C, r), oracle.hasf(X, C, r))
    X, C, r = synth.workload_shapes()
    say("tiles, halo", halo, "512x512 r=5")
    assert np.array_equal(_filter(c, X, C, r), oracle.hasf(X, C, r))
    for bad in (2, 6, 30, 36):
        with pytest.raises(hasf.HasfError):
            hasf.Context(0, tile_halo=bad)
    # the same with column tiles (one word of halo covers up to 32 passes)
    key = ("cols", halo)
    if key not in _HCTX:
        _HCTX[key] = hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1, tile_rows=8, tile_halo=halo,
                                  tile_cols=3)
    X = synth.random_binary(150, 500, 0.5, 824)
    say("column tiles, halo", halo)
    assert np.array_equal(_filter(_HCTX[key], X, None, 5), oracle.hasf(X, None, 5))


_CTX2 = {}


def t2ctx(th, nc):
    """Every image on the large-image path: bands of th rows cut into nc column tiles."""
    if (th, nc) not in _CTX2:
        _CTX2[(th, nc)] = hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1, tile_rows=th, tile_halo=12,
                                       tile_cols=nc)
    return _CTX2[(th, nc)]


TILE2D_CASES = [
    # (H, W, r, density, with C, tile rows, column tiles, seed): column tiles of
    # whole 64-column words, one word of halo on each side
    (40, 200, 2, 0.6, False, 8, 2, 1),     # 4 words: column tiles of 2 words
    (37, 130, 3, 0.55, True, 8, 3, 2),     # 3 words, 3 tiles of one word each; last row band short
    (100, 300, 4, 0.45, True, 10, 5, 3),   # 5 words, one per tile
    (129, 700, 6, 0.5, False, 24, 4, 4),   # ragged last word (700 = 10 * 64 + 60)
    (64, 1000, 8, 0.5, True, 16, 3, 5),
    (300, 520, 3, 0.5, False, 8, 2, 6),    # 38 bands x 2
    (18, 1500, 2, 0.5, False, 8, 7, 7),
    (61, 400, 12, 0.5, True, 8, 2, 8),     # radius beyond the halo
    (20, 4000, 3, 0.5, False, 12, 16, 9),  # one band of 20 rows, 16 column tiles
]


@pytest.mark.parametrize("case", TILE2D_CASES)
def test_column_tiles_random(case):
    H, W, r, dens, withC, th, nc, seed = case
    X = synth.random_binary(H, W, dens, 800 + seed)
    C = synth.random_binary(H, W, 0.05, 850 + seed) if withC else None
    say("column tiles", case)
    assert np.array_equal(_filter(t2ctx(th, nc), X, C, r), oracle.hasf(X, C, r))


@pytest.mark.parametrize("n", [8, 4])
def test_column_tiles_cd_order_pitch(n):
    X = synth.disks_image(90, 450, np.random.default_rng(31))
    rng = np.random.default_rng(32)
    C = ((rng.random(X.shape) < 0.03) & (X != 0)).astype(np.uint8)
    D = ((rng.random(X.shape) < 0.05) & (X == 0)).astype(np.uint8)
    for order in (0, 1):
        say("column tiles C, D, conn", n, "order", order)
        exp = oracle.hasf(X, C, 4, D=D, n=n, order=order)
        assert np.array_equal(_filter(t2ctx(12, 3), X, C, 4, pitch=467, D=D, n=n, order=order), exp)


def test_column_tiles_same_schedule_counts():
    # the same rounds and levels as one band per row tile and as the grid kernel
    X, _, _ = synth.workload_disks(H=300, W=1000)
    outs, counts = [], []
    for c in (t2ctx(16, 1), t2ctx(16, 4), tctx(-1)):
        c.grid_counts(reset=True)
        outs.append(_filter(c, X, None, 5))
        counts.append(c.grid_counts(reset=True))
    assert np.array_equal(outs[0], oracle.hasf(X, None, 5))
    assert all(np.array_equal(o, outs[0]) for o in outs[1:])
    assert counts[0]["rounds"] == counts[1]["rounds"] == counts[2]["rounds"]
    assert counts[0]["levels"] == counts[1]["levels"] == counts[2]["levels"]


def test_bad_tile_cols_is_refused():
    with pytest.raises(hasf.HasfError) as e:
        hasf.Context(0, tile_cols=-1)
    assert e.value.status == hasf.HASF_EINVAL


_FCTX = {}


@pytest.mark.parametrize("th", [96, 98, 240])
def test_tiles_pass_forms_at_their_boundaries(th):
    # A tile's pass tests one word per thread in place when its sub-image has
    # at most 1024 words, lists them wave by wave up to 2048, and through one
    # shared list beyond. W = 1024 (16 words), halo 16, one column tile: bands
    # of 96 rows keep 128 rows (64 x 16 = 1024 words, in place), of 98 rows
    # 130 (1040, per wave) and of 240 rows 272 (2176, shared list); the first
    # band is 16 rows shorter and the last band (H odd) has two sub-image
    # sizes, so each launch mixes two forms.
    if th not in _FCTX:
        _FCTX[th] = hasf.Context(0, grid_min_pixels=1, batch_grid_min_pixels=1, tile_rows=th, tile_halo=16,
                                 tile_cols=1)
    X = synth.random_binary(701, 1024, 0.5, 900 + th)
    C = synth.random_binary(701, 1024, 0.05, 950 + th)
    say("tile pass forms, tile rows", th)
    assert np.array_equal(_filter(_FCTX[th], X, C, 3), oracle.hasf(X, C, 3))
