"""Model of the decoder kernel's per-frame selection (k_beam.hip, steps
(b2)-(d)) against the plain rule it must reproduce: of all candidates of a
frame (each hypothesis's stay, and its extension by every class but the
blank that does not join a stay), the B with the largest totals, ties to the
smaller index i*V + c.

The kernel bounds the B-th best key from below by the B-th best of 2n
distinct candidates (the stays and each hypothesis's extension by the
frame's most probable class), pairs only the classes with F*y[c] at or above
the bound (F = the beam's largest max(s, p_b)) with the hypotheses, lists the
candidates at or above the bound and ranks the list; keys carry the index as
i*1024 + c.  Run in float32 on tie-heavy inputs (small value pools, zeros,
repeated labels, joins): the same winners in the same order.  Two planted
mistakes (a strict comparison in the class pruning, a bound one rank too
high) are caught."""
import numpy as np

F32 = np.float32


def key_of(total, idx):
    """64-bit key: total's bits above, 2^32-1-idx below; 0 when total <= 0."""
    if not (total > F32(0)):
        return 0
    return (int(np.array(total, np.float32).view(np.uint32)) << 32) | (0xFFFFFFFF - idx)


def random_frame(rng, n, V, blank):
    pool = np.array([0.0, 0.5, 0.25, 0.125, 0.75, 1.0, 0.375], np.float32)
    pb = rng.choice(pool, size=n).astype(np.float32)
    pnb = rng.choice(pool, size=n).astype(np.float32)
    s = (pb + pnb).astype(np.float32)
    # scores are kept below 1 (the best total is rescaled into [0.5, 1))
    s = np.minimum(s, F32(1.0))
    pb = np.minimum(pb, s)
    last = rng.integers(-1, V, size=n)
    last[last == blank] = (blank + 1) % V
    ypool = np.array([0.0, 0.0, 0.5, 0.25, 0.125, 0.0625, 0.5], np.float32)
    y = rng.choice(ypool, size=V).astype(np.float32)
    # a hypothesis's extension by c may join a stay (h_i + c is in the beam)
    merged = np.zeros((n, V), bool)
    for _ in range(int(rng.integers(0, n + 1))):
        merged[int(rng.integers(0, n)), int(rng.integers(0, V))] = True
    merged[:, blank] = False
    stay = rng.choice(pool * F32(0.5), size=n).astype(np.float32)   # stay totals
    return pb, s, last, y, merged, stay


def ext_total(pb, s, last, y, i, c):
    x = (pb[i] if c == last[i] else s[i]) * y[c]
    return F32(F32(0.0) + F32(x))


def plain_rule(B, pb, s, last, y, merged, stay, blank):
    n, V = merged.shape
    cands = []
    for i in range(n):
        for c in range(V):
            if c == blank:
                tot = stay[i]
            elif merged[i, c]:
                continue
            else:
                tot = ext_total(pb, s, last, y, i, c)
            if tot > F32(0):
                cands.append((-float(tot), i * V + c, i, c))
    cands.sort()
    return [(i, c) for _, _, i, c in cands[:B]]


def kernel_model(B, pb, s, last, y, merged, stay, blank, strict_prune=False, bound_shift=0):
    n, V = merged.shape
    idx = lambda i, c: (i << 10) | c
    # the frame's most probable non-blank class, the smallest of equals
    nb = [c for c in range(V) if c != blank]
    ymax = max(y[c] for c in nb)
    cs = min(c for c in nb if y[c] == ymax)
    sk = [key_of(stay[j], idx(j, blank)) for j in range(n)]
    ek = [0 if merged[j, cs] else key_of(ext_total(pb, s, last, y, j, cs), idx(j, cs)) for j in range(n)]
    keys = sorted([k for k in sk + ek if k != 0], reverse=True)
    r = B - 1 - bound_shift
    if r < 0:
        raise IndexError("no rank above the best")
    bound = keys[r] if len(keys) >= B else 1
    bound_f = np.array(bound >> 32, np.uint32).view(np.float32)[()]
    F = max(max(s[i], pb[i]) for i in range(n))
    lst = [k for k in sk if k != 0 and k >= bound]
    for c in range(V):
        if y[c] <= F32(0) or c == blank:
            continue
        fy = F32(y[c] * F)
        if (fy > bound_f) if strict_prune else (fy >= bound_f):
            for i in range(n):
                x = ext_total(pb, s, last, y, i, c)
                if x >= bound_f and not merged[i, c]:
                    k = key_of(x, idx(i, c))
                    if k >= bound:
                        lst.append(k)
    lst.sort(reverse=True)
    out = []
    for k in lst[:B]:
        j = 0xFFFFFFFF - (k & 0xFFFFFFFF)
        out.append((j >> 10, j & 1023))
    return out


def cases(seed, count):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(1, 17))
        V = int(rng.integers(2, 24))
        blank = int(rng.integers(0, V))
        B = int(rng.integers(1, 17))
        yield (B,) + random_frame(rng, n, V, blank) + (blank,)


def test_kernel_selection_equals_the_plain_rule():
    for args in cases(1, 3000):
        assert kernel_model(*args) == plain_rule(*args), args


def test_a_strict_class_pruning_is_caught():
    diverged = any(kernel_model(*a, strict_prune=True) != plain_rule(*a) for a in cases(2, 3000))
    assert diverged


def test_a_bound_one_rank_too_high_is_caught():
    diverged = False
    for a in cases(3, 3000):
        try:
            if kernel_model(*a, bound_shift=1) != plain_rule(*a):
                diverged = True
                break
        except IndexError:
            continue
    assert diverged
