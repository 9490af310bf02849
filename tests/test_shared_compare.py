"""Model of the kernels' per-frame update (engine.hpp, dp_frame) and of the
backtrack's decoding of its one-bit backpointers, against the strict rule of
the recursion written out directly (first maximum over s, s-1, s-2 with a
strict '>', paper Sec. 4 "CTC-based forced alignment").

The kernel lets a blank state s-1 pick the better of a(s-2) and a(s-1) (ties
to s-1), gives the label state s that winner when it may skip and a(s-1)
when it may not, compares it once with a(s), and stores one bit per state;
the decoder recovers s-2 from the blank's bit.  Checked here in float32 on
inputs full of ties, signed zeros and -inf: the same predecessor and the
bitwise same a_t for every state."""
import numpy as np

NINF = np.float32(-np.inf)


def strict_step(a, e, skip):
    """a_t and the predecessor offset k (0, 1, 2) per state, by the rule."""
    S = a.shape[0]
    out = np.empty_like(a)
    k = np.zeros(S, np.int64)
    for s in range(S):
        best, kk = a[s], 0
        if s >= 1 and a[s - 1] > best:
            best, kk = a[s - 1], 1
        if s >= 2 and skip[s] and a[s - 2] > best:
            best, kk = a[s - 2], 2
        out[s] = np.float32(e[s] + best)
        k[s] = kk
    return out, k


def shared_step(a, e, skip):
    """a_t and one bit per state, as the kernel computes them."""
    S = a.shape[0]
    out = np.empty_like(a)
    bit = np.zeros(S, np.int64)
    for s in range(0, S, 2):                      # blank s, label s+1
        y = a[s]
        z = a[s - 1] if s >= 1 else NINF
        cb = z > y
        wb = z if cb else y
        out[s] = np.float32(e[s] + wb)
        bit[s] = int(cb)
        if s + 1 < S:
            x = a[s + 1]
            fb = wb if skip[s + 1] else y
            cl = fb > x
            out[s + 1] = np.float32(e[s + 1] + (fb if cl else x))
            bit[s + 1] = int(cl)
    return out, bit


def decode(bit, skip, s):
    """The backtrack's predecessor offset of state s from the bits."""
    if s % 2 == 0:
        return int(bit[s])
    if not bit[s]:
        return 0
    return 2 if (skip[s] and bit[s - 1]) else 1


def random_case(rng, L):
    S = 2 * L + 1
    lab = rng.integers(1, 4, size=L)              # few classes: repeated labels
    skip = np.zeros(S, bool)
    for s in range(3, S, 2):
        skip[s] = lab[(s - 1) // 2] != lab[(s - 3) // 2]
    pool = np.array([0.0, -0.0, -1.0, -2.0, -3.0, -np.inf, -0.5, -1.5], np.float32)
    a = rng.choice(pool, size=S).astype(np.float32)
    e = rng.choice(pool[:5], size=S).astype(np.float32)
    return a, e, skip


def test_shared_compare_matches_the_strict_rule():
    rng = np.random.default_rng(7)
    for _ in range(4000):
        L = int(rng.integers(0, 6))
        a, e, skip = random_case(rng, L)
        ref, k = strict_step(a, e, skip)
        got, bit = shared_step(a, e, skip)
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32)), (a, e, skip)
        for s in range(a.shape[0]):
            assert decode(bit, skip, s) == k[s], (a, skip, s)


def test_a_label_that_may_not_skip_ignores_the_blank_choice():
    # a(s-2) > a(s-1) > a(s): the blank takes s-2, the repeated label must
    # still come from s-1
    a4 = np.array([-9.0, -1.0, -2.0, -5.0, -9.0], np.float32)   # label 3: z=-1 > y=-2 > x=-5
    skip = np.array([False, False, False, False, False])
    e = np.zeros(5, np.float32)
    ref, k = strict_step(a4, e, skip)
    got, bit = shared_step(a4, e, skip)
    assert k[3] == 1 and decode(bit, skip, 3) == 1 and got[3] == ref[3]
    skip[3] = True
    ref, k = strict_step(a4, e, skip)
    got, bit = shared_step(a4, e, skip)
    assert k[3] == 2 and decode(bit, skip, 3) == 2 and got[3] == ref[3]


def test_a_tie_to_the_farther_state_is_caught():
    # the model is sensitive to the tie rule: a blank compare of z >= y (ties
    # to s-2) diverges from the strict rule on these inputs
    rng = np.random.default_rng(11)
    diverged = False
    for _ in range(2000):
        a, e, skip = random_case(rng, int(rng.integers(1, 6)))
        _, k = strict_step(a, e, skip)
        S = a.shape[0]
        bit = np.zeros(S, np.int64)
        for s in range(0, S, 2):
            z = a[s - 1] if s >= 1 else NINF
            bit[s] = int(z >= a[s])
            if s + 1 < S:
                wb = z if bit[s] else a[s]
                fb = wb if skip[s + 1] else a[s]
                bit[s + 1] = int(fb > a[s + 1])
        if any(decode(bit, skip, s) != k[s] for s in range(S)):
            diverged = True
            break
    assert diverged
