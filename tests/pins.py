"""Pins of the CPU oracle against facts fixed by the mathematics of CTC
forced alignment (no shared code with the oracle's dynamic program).

Each check takes an `align` callable with the oracle's float32 signature
``align(E, labels, blank) -> (status, path, scores, total)`` and returns a
list of failure messages, so the same checks run against the committed
oracle and against deliberately broken copies of it (mutation tests).
"""
from __future__ import annotations

import math

import numpy as np

import brute
from invariants import check_alignment, fold32

F32 = np.float32


def bits(x) -> int:
    return int(np.float32(x).view(np.uint32))


def tiny_cases(seed: int, n: int, integer: bool = False, zeros: bool = False,
               denormal: bool = False, neg_inf_p: float = 0.0):
    """n random tiny problems: T<=7, C<=4, L<=3 (with repeats), random blank."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        C = int(rng.integers(2, 5))
        T = int(rng.integers(1, 8 if C <= 3 else 7))
        L = int(rng.integers(0, 4))
        blank = int(rng.integers(0, C))
        nonblank = [c for c in range(C) if c != blank]
        y = np.array([nonblank[int(rng.integers(0, len(nonblank)))] for _ in range(L)],
                     dtype=np.int32)
        if integer:
            E = -rng.integers(0, 4, size=(T, C)).astype(np.float32)
        elif zeros:
            E = rng.choice(np.array([0.0, -0.0, -1.0], dtype=np.float32), size=(T, C))
        elif denormal:
            E = (rng.standard_normal((T, C)) * 1e-39).astype(np.float32)
        else:
            E = -np.abs(rng.standard_normal((T, C))).astype(np.float32) * F32(3.0)
        if neg_inf_p > 0:
            E[rng.random((T, C)) < neg_inf_p] = -np.inf
        out.append((E, y, blank))
    return out


def check_brute(align, cases) -> list:
    """F1: total == max over all alignments of their float32 left fold
    (bitwise); F2: the returned path is an alignment and its own fold equals
    the total (bitwise); infeasible iff no alignment has a finite score."""
    fails = []
    for i, (E, y, blank) in enumerate(cases):
        st, path, scores, total = align(E, y, blank)
        pis, sc = brute.brute(E, y, blank)
        best = sc.max() if len(sc) else -np.inf
        if best == -np.inf:
            if st != 2 or total != -np.inf or np.any(path != -1) or np.any(scores != -np.inf):
                fails.append(f"case {i}: expected infeasible, got status {st}")
            continue
        if st != 0:
            fails.append(f"case {i}: status {st} for a feasible case")
            continue
        if bits(total) != bits(best):
            fails.append(f"case {i}: total {total!r} != brute max {best!r}")
        errs = check_alignment(E, y, blank, path, scores, total)
        if errs:
            fails.append(f"case {i}: {errs}")
    return fails


def check_tie_rule(align, cases) -> list:
    """F3: with exactly representable sums, the returned path is the optimal
    alignment whose reversed state sequence is lexicographically largest."""
    fails = []
    for i, (E, y, blank) in enumerate(cases):
        st, path, scores, total = align(E, y, blank)
        ref = brute.best_by_tie_rule(E, y, blank)
        if ref is None:
            if st != 2:
                fails.append(f"case {i}: expected infeasible")
            continue
        if st != 0 or not np.array_equal(np.asarray(path, np.int64), ref):
            fails.append(f"case {i}: path {list(path)} != tie-rule path {list(ref)}")
            continue
        if bits(total) != bits(fold32(E[np.arange(E.shape[0]), ref])):
            fails.append(f"case {i}: total bits differ from the tie-rule path's fold")
    return fails


def earliest_path(y, T: int, blank: int) -> np.ndarray:
    """Closed form for uniform emissions: every label as early as possible
    (a blank only between equal neighbours), then blanks to the end."""
    seq = []
    for j, c in enumerate(y):
        if j > 0 and y[j - 1] == c:
            seq.append(blank)
        seq.append(int(c))
    return np.array(seq + [blank] * (T - len(seq)), dtype=np.int64)


def check_closed_forms(align) -> list:
    fails = []
    rng = np.random.default_rng(11)
    # F4: uniform emissions
    for y in ([1, 2, 3], [1, 1, 2], [2, 2, 2], [], [3], [1, 2, 1, 2, 2]):
        R = sum(1 for j in range(1, len(y)) if y[j] == y[j - 1])
        for T in range(max(1, len(y) + R), len(y) + R + 6):
            for val in (-1.5, -0.25, -7.0):
                E = np.full((T, 5), val, dtype=np.float32)
                st, path, scores, total = align(E, np.array(y, np.int32), 0)
                exp = earliest_path(y, T, 0)
                if st != 0 or not np.array_equal(np.asarray(path, np.int64), exp):
                    fails.append(f"uniform y={y} T={T}: {list(path)} != {list(exp)}")
    # L = 0: all blank, total = fold of the blank column
    for blank in (0, 2):
        E = rng.standard_normal((37, 4)).astype(np.float32)
        st, path, scores, total = align(E, np.zeros(0, np.int32), blank)
        if st != 0 or np.any(path != blank) or bits(total) != bits(fold32(E[:, blank])):
            fails.append(f"L=0 blank={blank} wrong")
    # T = L + R: the unique minimal alignment
    for y in ([1, 2, 3, 4], [1, 1, 1], [2, 3, 3, 2]):
        R = sum(1 for j in range(1, len(y)) if y[j] == y[j - 1])
        T = len(y) + R
        E = -np.abs(rng.standard_normal((T, 5))).astype(np.float32)
        st, path, scores, total = align(E, np.array(y, np.int32), 0)
        if st != 0 or not np.array_equal(np.asarray(path, np.int64), earliest_path(y, T, 0)):
            fails.append(f"T=L+R y={y}: {list(path)}")
    # T < L + R: infeasible
    for y, T in (([1, 2, 3], 2), ([1, 1], 2), ([2, 2, 2], 4)):
        E = np.zeros((T, 4), dtype=np.float32)
        st, path, scores, total = align(E, np.array(y, np.int32), 0)
        if st != 2 or total != -np.inf or np.any(path != -1) or np.any(scores != -np.inf):
            fails.append(f"infeasible y={y} T={T} not reported")
    # T = 1
    E = np.array([[-1.0, -2.0, -3.0]], dtype=np.float32)
    for y, exp_st, exp_path in (([], 0, [0]), ([2], 0, [2]), ([1, 2], 2, [-1])):
        st, path, scores, total = align(E, np.array(y, np.int32), 0)
        if st != exp_st or list(path) != exp_path:
            fails.append(f"T=1 y={y}: status {st} path {list(path)}")
    # a -inf mask that leaves one alignment returns exactly that alignment
    from paper_2310_17864_amd import synth
    for seed in range(3):
        r = np.random.default_rng(100 + seed)
        u = synth.utterance(r, 60, 6, 12, blank=0, repeat_p=0.3)
        E = u.emission.copy()
        lab = np.where(u.planted % 2 == 0, 0, u.labels[np.maximum(u.planted - 1, 0) // 2])
        mask = np.ones_like(E, dtype=bool)
        mask[np.arange(60), lab] = False
        E[mask] = -np.inf
        st, path, scores, total = align(E, u.labels, 0)
        if st != 0 or not np.array_equal(np.asarray(path), lab):
            fails.append(f"-inf mask seed {seed}: planted path not returned")
    # invalid labels
    for y in ([0], [5], [-1], [1, 0]):
        E = np.zeros((4, 5), dtype=np.float32)
        st, path, scores, total = align(E, np.array(y, np.int32), 0)
        if st != 1 or np.any(path != -1) or not np.all(np.isnan(scores)):
            fails.append(f"invalid labels {y} not rejected")
    return fails


def ctc_loss_limit(E: np.ndarray, y, blank: int, total64: float, betas=(1.0, 10.0, 100.0, 1000.0)):
    """Library cross-check through torch.nn.functional.ctc_loss (float64,
    CPU): -ctc_loss(beta*E)/beta = (1/beta) log sum_pi exp(beta*score(pi))
    lies in [max score, max score + ln(#alignments)/beta]."""
    import torch
    T, C = E.shape
    fails = []
    lp = torch.from_numpy(E.astype(np.float64)).reshape(T, 1, C)
    tgt = torch.tensor(np.asarray(y, dtype=np.int64)).reshape(1, -1)
    for beta in betas:
        loss = torch.nn.functional.ctc_loss(beta * lp, tgt, torch.tensor([T]),
                                            torch.tensor([len(y)]), blank=blank,
                                            reduction="sum", zero_infinity=False)
        v = -float(loss) / beta
        lo = total64 - 1e-9 * max(1.0, abs(total64))
        hi = total64 + T * math.log(3.0) / beta + 1e-9 * max(1.0, abs(total64))
        if not (lo <= v <= hi):
            fails.append(f"beta={beta}: {v} not in [{lo}, {hi}]")
    return fails
