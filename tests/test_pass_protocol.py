"""A host-side model of the control protocol that the waves of one workgroup
follow through the subfield rounds of a distance level (the per-wave pass
form of the kernels' run_rounds, whose waves meet one barrier per executed
pass), run under adversarial and random interleavings of the waves.

Every wave keeps its own copy of the scheduling state (serial, the prod value
each sub-image's pass last consumed) and takes the skip decisions itself from
the shared words prod[4] and chg. The protocol is correct when every wave
takes the same decisions, i.e. every barrier is reached by all waves with the
same pass. The model shows that a single copy of prod is not enough: after a
level's activation, or after a pass that changed nothing, the waves may skip
pass s and run a later pass t; a wave that runs ahead stores prod[s] in pass
t while a slower wave has still to decide whether to skip pass s, so the
slower wave runs pass s alone. It also shows that the double copy by executed-pass
parity, with the read copy carried into the written one, keeps the waves in
step under every interleaving tried."""
import random

import pytest

SUBS = 4


def targets(s):
    """Sub-images whose words read sub-image s (E/W, N/S, diagonal)."""
    si, sj = s >> 1, s & 1
    so, co = 1 - si, 1 - sj
    return [si * 2 + co, so * 2 + sj, so * 2 + co]


def wave(w, double, changed, levels):
    """One wave's run of the levels of a phase: per level, the activation of
    the sub-images listed (wave 0 stores their prod words: both copies in the
    double protocol), a barrier, then rounds of the four passes until a round
    changes nothing, then a barrier. Yields memory operations and barriers;
    receives the values of its reads."""
    consumed = [0] * SUBS
    serial = 0
    rd = 0
    for act in levels:
        serial += 1
        if w == 0:
            for t in act:
                yield ("write", t, serial)
                if double:
                    yield ("write", t + 4, serial)
        yield ("barrier", ("activate", serial))
        while True:
            round_start = serial
            for s in range(SUBS):
                rd_off = rd if double else 0
                wr_off = (rd ^ 4) if double else 0
                p = yield ("read", rd_off + s)
                if p <= consumed[s]:
                    continue
                consumed[s] = p
                serial += 1
                ser = serial
                if double and w == 0:
                    for t in range(SUBS):
                        v = yield ("read", rd_off + t)
                        yield ("max", wr_off + t, v)
                if changed(ser, w):
                    yield ("write", "chg", ser)
                    for t in targets(s):
                        yield ("write", wr_off + t, ser)
                yield ("barrier", ("pass", ser, s))
                if double:
                    rd ^= 4
            c = yield ("read", "chg")
            if c <= round_start:
                break
        yield ("barrier", ("level end", serial))


class OutOfStep(Exception):
    pass


def run(nwaves, double, changed, pick, levels, max_steps=400000):
    """Runs the waves, choosing the next wave to step with pick(runnable).
    Returns the list of passes (serial, sub-image) the workgroup executed."""
    mem = {"chg": 0}
    for k in range(8):
        mem[k] = 0
    gens = [wave(w, double, changed, levels) for w in range(nwaves)]
    pending = [None] * nwaves  # operation each wave waits to perform
    reply = [None] * nwaves
    for w in range(nwaves):
        pending[w] = next(gens[w])
    at_barrier = {}
    done = set()
    passes = []
    for _ in range(max_steps):
        if len(done) == nwaves:
            return passes
        runnable = [w for w in range(nwaves) if w not in done and w not in at_barrier]
        if not runnable:
            labels = set(at_barrier.values())
            if len(labels) != 1:
                raise OutOfStep("barrier reached with different passes: %s" % sorted(map(str, labels)))
            lab = labels.pop()
            if lab[0] == "pass":
                passes.append(lab[1:])
            for w in list(at_barrier):
                del at_barrier[w]
                try:
                    pending[w] = gens[w].send(None)
                except StopIteration:
                    done.add(w)
            continue
        w = pick(runnable)
        op = pending[w]
        val = None
        if op[0] == "read":
            val = mem[op[1]]
        elif op[0] == "write":
            mem[op[1]] = op[2]
        elif op[0] == "max":
            mem[op[1]] = max(mem[op[1]], op[2])
        elif op[0] == "barrier":
            at_barrier[w] = op[1]
            continue
        try:
            pending[w] = gens[w].send(val)
        except StopIteration:
            done.add(w)
    raise AssertionError("model did not finish")


def changes_script(pattern):
    """changed(ser, w): wave 0 changes a pixel in the passes whose serials are
    listed (the other waves' chunks hold nothing to change)."""
    return lambda ser, w: w == 0 and ser in pattern


def fast_wave_first(runnable):
    """Adversarial order: a wave moves only when every lower-numbered wave is
    waiting at a barrier, so wave 0 runs ahead between barriers."""
    return runnable[0]


# A level activates only sub-image 2: after the activation's barrier the waves
# skip passes 0 and 1 and run pass 2 (serial 2), which changes a pixel and
# stores prod[0], prod[1] and prod[3].
SKIP_THEN_RUN = [[2]]


@pytest.mark.parametrize("double", [False, True])
def test_skip_then_later_pass(double):
    changed = changes_script({2})
    if not double:
        # wave 1 decides on pass 0 only after wave 0 stored prod[0] in pass 2:
        # it runs pass 0, which wave 0 skipped
        with pytest.raises(OutOfStep):
            run(2, False, changed, fast_wave_first, SKIP_THEN_RUN)
    else:
        ref = run(1, True, changed, fast_wave_first, SKIP_THEN_RUN)
        assert ref[0] == (2, 2)
        assert run(2, True, changed, fast_wave_first, SKIP_THEN_RUN) == ref


def _random_levels(rng, n):
    return [sorted(rng.sample(range(SUBS), rng.randint(1, SUBS))) for _ in range(n)]


def test_random_interleavings_single_copy_goes_out_of_step():
    """With one copy of prod, random interleavings of random levels put the
    waves out of step."""
    bad = 0
    for seed in range(300):
        rng = random.Random(seed)
        levels = _random_levels(rng, 4)
        pat = {s for s in range(2, 60) if rng.random() < 0.35}
        try:
            run(4, False, changes_script(pat), lambda r: rng.choice(r), levels)
        except OutOfStep:
            bad += 1
    assert bad > 0


@pytest.mark.parametrize("nwaves", [2, 4, 8, 16])
def test_random_interleavings_double_copy_stays_in_step(nwaves):
    """With the double copy every interleaving runs the same passes as one
    wave alone (which has no one to race with)."""
    for seed in range(300):
        rng = random.Random(1000 * nwaves + seed)
        levels = _random_levels(rng, 4)
        pat = {s for s in range(2, 60) if rng.random() < 0.35}
        changed = lambda ser, w, pat=pat: w == (ser % nwaves) and ser in pat
        ref = run(1, True, lambda ser, w, pat=pat: ser in pat, lambda r: r[0], levels)
        bias = rng.random()
        got = run(nwaves, True, changed, lambda r: r[0] if rng.random() < bias else rng.choice(r), levels)
        assert got == ref, seed
