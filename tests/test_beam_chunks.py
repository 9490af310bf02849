"""Model of the decoder kernel's blank-collapse bookkeeping (k_beam.hip,
kept_frames and the next-kept-frame prefetch): blank flags taken one ballot
per 64-frame chunk, the kept frames of a chunk as a bit mask that carries
the previous chunk's last flag, and the next kept frame found in the same
chunk or, past its end, in the next one (farther kept frames are loaded
when they come).  Checked against the plain rule (a
frame whose blank probability exceeds the threshold is dropped when the
frame before it is such a frame too) for every length around the chunk
boundaries; a mask that forgets the carried flag is caught."""
import numpy as np

CH = 64
MASK = (1 << 64) - 1


def plain_kept(flags):
    out, prev = [], False
    for t, f in enumerate(flags):
        if not (f and prev):
            out.append(t)
        prev = f
    return out


def kept_frames(fl, nt, prev, carry=True):
    valid = MASK if nt >= 64 else (1 << nt) - 1
    return valid & ~(fl & (((fl << 1) & MASK) | (1 if (prev and carry) else 0))) & MASK


def ballot(flags, t0):
    return sum(1 << i for i in range(min(CH, len(flags) - t0)) if flags[t0 + i])


def kernel_kept(flags, carry=True):
    """Kept frames in processing order, with the prefetch target of each."""
    T = len(flags)
    order, nexts = [], []
    fl, prev = ballot(flags, 0), False
    for t0 in range(0, T, CH):
        nt = min(T - t0, CH)
        keep = kept_frames(fl, nt, prev, carry)
        last = bool((fl >> (nt - 1)) & 1)
        t1 = t0 + CH
        while keep:
            tt = (keep & -keep).bit_length() - 1
            keep &= keep - 1
            order.append(t0 + tt)
            if keep:
                tn = t0 + (keep & -keep).bit_length() - 1
            elif t1 < T:
                k1 = kept_frames(ballot(flags, t1), T - t1, last, carry)
                tn = t1 + (k1 & -k1).bit_length() - 1 if k1 else -1
            else:
                tn = -1
            nexts.append(tn)
        if t1 < T:
            fl = ballot(flags, t1)
        prev = last
    return order, nexts


def lengths():
    return [1, 2, 3, 63, 64, 65, 127, 128, 129, 191, 200, 257]


def test_kept_frames_and_prefetch_targets_match_the_rule():
    rng = np.random.default_rng(5)
    for T in lengths():
        for p in (0.0, 0.3, 0.7, 0.95, 1.0):
            for _ in range(20):
                flags = list(rng.random(T) < p)
                ref = plain_kept(flags)
                order, nexts = kernel_kept(flags)
                assert order == ref, (T, p)
                # the prefetch names the next kept frame whenever it lies in
                # the same chunk or the next one, and no frame otherwise (the
                # row is then loaded when its frame comes)
                for k, t in enumerate(ref):
                    nxt = ref[k + 1] if k + 1 < len(ref) else -1
                    near = nxt >= 0 and nxt // CH <= t // CH + 1
                    assert nexts[k] == (nxt if near else -1), (T, p, t)


def test_a_mask_without_the_carried_flag_is_caught():
    # a blank run across a chunk boundary keeps the first frame of the next
    # chunk unless the previous chunk's last flag is carried
    flags = [False] * 60 + [True] * 10
    assert kernel_kept(flags, carry=False)[0] != plain_kept(flags)
    assert kernel_kept(flags)[0] == plain_kept(flags)
