"""Model of the boundary ring between segments of one workgroup (engine.hpp,
segment_forward with per-group flow control): segment w publishes a_t of its
top state for every frame into slot bslot(t) of its ring, and the segment
above reads them one frame ahead.  A segment starts an 8-frame group once the
segment below has published one value past the group and the segment above
has consumed all but kFlowWin frames of what this group will overwrite.

Run under random interleavings, every value a segment reads must be the one
published for that frame (no slot overwritten too early), and every schedule
must finish (no deadlock).  Constants come from the kernels' own header."""
import os
import random
import re

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(HERE, "..", "paper_2310_17864_amd", "csrc", "internal.hpp")


def constant(name):
    txt = open(HDR).read()
    m = re.search(r"constexpr int %s = (\d+);" % name, txt)
    assert m, name
    return int(m.group(1))


BND, WIN, UNROLL, BLK = constant("kBnd"), constant("kFlowWin"), constant("kUnroll"), constant("kBlk")


def bslot(t):
    return 0 if t == 0 else ((t - 1) % BND) + 1


def run(T, W, win, seed):
    rng = random.Random(seed)
    nsteps = T - 1
    ring = [dict() for _ in range(W)]            # slot -> frame whose value it holds
    prod = [0] * W                               # values 0 .. prod-1 published
    cons = [0] * W                               # values of the segment below consumed
    nxt = [0] * W                                # next frame group per segment
    ngrp = (nsteps + UNROLL - 1) // UNROLL
    for w in range(W):                           # frame 0
        if w + 1 < W:
            ring[w][0] = 0
            prod[w] = 1
    while True:
        ready = []
        for w in range(W):
            g = nxt[w]
            if g >= ngrp:
                continue
            ubase = UNROLL * g
            ne = min(UNROLL, nsteps - ubase)
            if w > 0 and prod[w - 1] < ubase + ne + 1:
                continue
            if w + 1 < W and ubase + ne - win + 1 > 0 and cons[w + 1] < ubase + ne - win + 1:
                continue
            ready.append(w)
        if not ready:
            return all(nxt[w] >= ngrp for w in range(W))   # False: deadlock
        w = rng.choice(ready)
        g = nxt[w]
        ubase = UNROLL * g
        ne = min(UNROLL, nsteps - ubase)
        if w > 0:
            # the block's first frame at its first group, then one frame ahead
            frames = ([ubase] if ubase % BLK == 0 else []) + list(range(ubase + 1, ubase + ne + 1))
            for t in frames:
                if ring[w - 1].get(bslot(t)) != t:
                    raise AssertionError(f"segment {w} read slot {bslot(t)} for frame {t}: "
                                         f"holds {ring[w - 1].get(bslot(t))}")
            cons[w] = ubase + ne
        if w + 1 < W:
            for t in range(ubase + 1, ubase + ne + 1):
                ring[w][bslot(t)] = t
            prod[w] = ubase + ne + 1
        nxt[w] = g + 1


def test_slots_of_a_group_are_consecutive():
    for g in range(40):
        base = bslot(UNROLL * g + 1)
        assert [bslot(UNROLL * g + 1 + i) for i in range(UNROLL)] == list(range(base, base + UNROLL))
    assert bslot(0) == 0 and {bslot(t) for t in range(1, 5 * BND)} == set(range(1, BND + 1))


def test_window_never_overwrites_a_value_in_use_and_never_deadlocks():
    assert 2 * UNROLL <= WIN <= BND
    for T in (2, 9, 33, 100, 517, 3000):
        for W in (2, 4, 8):
            for seed in range(6):
                assert run(T, W, WIN, seed), (T, W, seed)


def test_a_window_past_the_ring_overwrites_values():
    # a producer allowed to run more than the ring's frames ahead overwrites
    # a slot before the segment above has read it
    failed = False
    for seed in range(40):
        try:
            run(3000, 2, BND + 3 * UNROLL, seed)
        except AssertionError:
            failed = True
            break
    assert failed
