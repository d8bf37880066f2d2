"""Host-side models of two pieces of device logic that no GPU test can take
apart on its own.

1. The tile kernel's grid barrier with the level-end decision folded into it.
   Each tile adds 1 + (chg << 32) to a 64-bit arrival word (chg: its epoch's
   last round changed one of its own pixels); the last arrival (the one whose
   add brings the low half to (gen + 1) * tiles) stores gen + 1 with the high
   half of its new sum in the barrier word; every tile then says "quiet" when
   the barrier word's high half equals the one it saw at its previous barrier.
   The model runs many barriers with random arrival orders and random chg
   flags and checks that every tile's decision is "no tile set chg at this
   barrier", that all tiles decide alike, and that a tile never reads a
   barrier word of another generation.

2. The direct minimum of the EDT's few-column rows. For parabolas
   (j - k)^2 + g_k^2 with distinct k sorted increasingly, the first column
   that is lowest at a pixel never moves left as the pixel moves right, so
   over a run of pixels [j0, j1] the minimum at each pixel is found among the
   columns between the first lowest at j0 and the first lowest at j1. Checked
   against the plain minimum over all columns on random column sets, runs and
   ties."""
import random

import numpy as np
import pytest


def run_barriers(ntiles, nbar, seed):
    rng = random.Random(seed)
    arrive = 0           # the 64-bit arrival word
    word = 0             # the barrier word: gen | cum << 32
    cchg = [0] * ntiles  # each tile's high half seen at its previous barrier
    for gen in range(nbar):
        chg = [rng.random() < 0.3 if rng.random() < 0.7 else False for _ in range(ntiles)]
        order = list(range(ntiles))
        rng.shuffle(order)
        last_word = None
        seen = {}
        for pos, t in enumerate(order):
            add = 1 | ((1 if chg[t] else 0) << 32)
            old = arrive
            arrive = (arrive + add) & ((1 << 64) - 1)
            if (old & 0xFFFFFFFF) + 1 == (gen + 1) * ntiles:
                assert pos == ntiles - 1  # only the last arrival completes it
                word = (gen + 1) | ((old + add) & 0xFFFFFFFF00000000)
                last_word = word
        # every tile waits for the new generation and reads the same word
        for t in range(ntiles):
            w = word
            assert (w & 0xFFFFFFFF) == gen + 1
            cum = w >> 32
            quiet = cum == cchg[t]
            cchg[t] = cum
            seen[t] = quiet
        assert last_word is not None
        want = not any(chg)
        assert all(q == want for q in seen.values()), (gen, chg)


@pytest.mark.parametrize("ntiles", [1, 2, 7, 256])
def test_tile_barrier_quiet_word(ntiles):
    run_barriers(ntiles, 300 if ntiles < 256 else 60, 1000 + ntiles)


def test_tile_barrier_words_do_not_overflow_in_long_runs():
    # arrivals stay in the low half for (gen + 1) * tiles < 2^32 and the
    # change count in the high half; a long run of 256 tiles all changing
    ntiles, nbar = 256, 5000
    arrive = 0
    for gen in range(nbar):
        arrive += ntiles * (1 | (1 << 32))
    assert (arrive & 0xFFFFFFFF) == ntiles * nbar and (arrive >> 32) == ntiles * nbar


def direct_run_minimum(cols, g, j0, j1):
    """The kernel's rule: first lowest columns at the run's ends, then the
    minimum over the columns between them at each pixel."""
    def f(q, j):
        return (j - cols[q]) ** 2 + g[q] ** 2
    qa = min(range(len(cols)), key=lambda q: (f(q, j0), q))
    qb = min(range(len(cols)), key=lambda q: (f(q, j1), q))
    return [min(f(q, j) for q in range(qa, qb + 1)) for j in range(j0, j1 + 1)]


@pytest.mark.parametrize("seed", range(40))
def test_few_columns_run_minimum(seed):
    rng = np.random.default_rng(seed)
    W = int(rng.integers(2, 400))
    n = int(rng.integers(1, min(W, 32) + 1))
    cols = sorted(rng.choice(W, n, replace=False).tolist())
    # small g values make many ties between columns
    g = rng.integers(0, 4 if seed % 3 == 0 else W, n).tolist()
    B = int(rng.integers(1, 40))
    for j0 in range(0, W, B):
        j1 = min(W, j0 + B) - 1
        want = [min((j - k) ** 2 + gg ** 2 for k, gg in zip(cols, g)) for j in range(j0, j1 + 1)]
        assert direct_run_minimum(cols, g, j0, j1) == want, (seed, j0)


def test_few_columns_rule_needs_sorted_columns():
    # the rule relies on increasing columns: with the columns out of order the
    # range between the two ends can miss the lowest column (a plausible
    # mistake in the kernel's listing that the ordering step prevents)
    cols, g = [10, 0, 20], [0, 0, 0]
    got = direct_run_minimum(cols, g, 0, 20)
    want = [min((j - k) ** 2 for k in cols) for j in range(0, 21)]
    assert got != want
    order = sorted(range(3), key=lambda q: cols[q])
    assert direct_run_minimum([cols[q] for q in order], [g[q] for q in order], 0, 20) == want
