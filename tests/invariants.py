"""Checks that hold for any correct forced alignment, at any size.

* the label path collapses to the transcript (merge runs, drop blanks);
* the implied trellis states start in {0, 1}, end in {S-1, S-2}, never
  decrease, move by at most 2, and move by 2 only into a label state whose
  label differs from the one two states back;
* scores[t] == E[t, path[t]] bitwise;
* total == float32 left fold of scores, bitwise (the path's own score is the
  maximum, which the dynamic program reaches with the same additions).
"""
from __future__ import annotations

import numpy as np


def fold32(x: np.ndarray) -> np.float32:
    acc = np.float32(x[0])
    for v in x[1:]:
        acc = np.float32(acc + np.float32(v))
    return acc


def path_states(path: np.ndarray, blank: int) -> np.ndarray:
    """Trellis state of every frame of a label path (blank after k tokens ->
    2k; a frame of the k-th token -> 2k-1)."""
    p = np.asarray(path, dtype=np.int64)
    prev = np.concatenate([[-1], p[:-1]])
    new_tok = (p != blank) & (p != prev)
    k = np.cumsum(new_tok)
    return np.where(p == blank, 2 * k, 2 * k - 1)


def check_alignment(E: np.ndarray, labels: np.ndarray, blank: int, path: np.ndarray,
                    scores: np.ndarray, total) -> list:
    """Return a list of violated invariants (empty when the alignment is valid)."""
    errs = []
    E = np.asarray(E, dtype=np.float32)
    T = E.shape[0]
    y = np.asarray(labels, dtype=np.int64)
    L = len(y)
    S = 2 * L + 1
    path = np.asarray(path, dtype=np.int64)
    if path.shape != (T,):
        return [f"path shape {path.shape} != ({T},)"]
    if np.any(path < 0) or np.any(path >= E.shape[1]):
        return ["path holds ids outside [0, C)"]
    prev = np.concatenate([[-1], path[:-1]])
    collapsed = path[(path != blank) & (path != prev)]
    if not np.array_equal(collapsed, y):
        errs.append("path does not collapse to the transcript")
        return errs
    st = path_states(path, blank)
    if st[0] not in (0, 1):
        errs.append(f"first state {st[0]} not in {{0,1}}")
    if S == 1:
        if st[-1] != 0:
            errs.append("last state != 0 for an empty transcript")
    elif st[-1] not in (S - 1, S - 2):
        errs.append(f"last state {st[-1]} not in {{S-1,S-2}}")
    d = np.diff(st)
    if np.any(d < 0) or np.any(d > 2):
        errs.append("state steps outside {0,1,2}")
    for t in np.nonzero(d == 2)[0]:
        s = st[t + 1]
        if s % 2 == 0 or s < 3 or y[(s - 1) // 2] == y[(s - 3) // 2]:
            errs.append(f"illegal skip into state {s} at frame {t + 1}")
            break
    ref_sc = E[np.arange(T), path]
    if not np.array_equal(ref_sc.view(np.uint32), np.asarray(scores, np.float32).view(np.uint32)):
        errs.append("scores[t] != E[t, path[t]] bitwise")
    if np.float32(total).view(np.uint32) != fold32(ref_sc).view(np.uint32):
        errs.append("total != float32 left fold of the path's emissions")
    return errs
