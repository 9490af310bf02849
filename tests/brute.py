"""Brute-force CTC alignment on tiny inputs, from the textbook definition.

A frame labelling pi in [0, C)^T is a CTC alignment of transcript y iff
collapsing it (merge runs of equal symbols, then drop blanks) gives y
(Graves et al. 2006, the CTC formalism the paper builds on).  This module
enumerates every such pi -- no trellis, no recurrence -- and scores each one
by a float32 left fold of its emissions, so it shares nothing with the oracle's
dynamic program.
"""
from __future__ import annotations

import itertools

import numpy as np


def all_sequences(T: int, C: int) -> np.ndarray:
    """Every pi in [0, C)^T as an int64 array [C**T, T]."""
    return np.array(list(itertools.product(range(C), repeat=T)), dtype=np.int64).reshape(-1, T)


def collapses_to(pi: np.ndarray, y: np.ndarray, blank: int) -> np.ndarray:
    """Boolean mask over rows of pi: collapse(pi) == y."""
    n, T = pi.shape
    L = len(y)
    prev = np.concatenate([np.full((n, 1), -1), pi[:, :-1]], axis=1)
    keep = (pi != blank) & (pi != prev)          # first frame of each non-blank run
    count = keep.sum(axis=1)
    ok = count == L
    if L == 0:
        return ok
    k = np.cumsum(keep, axis=1) - 1
    k = np.clip(k, 0, L - 1)
    yk = np.asarray(y, dtype=np.int64)[k]
    ok &= np.all(~keep | (pi == yk), axis=1)
    return ok


def fold32(E: np.ndarray, pi: np.ndarray) -> np.ndarray:
    """float32 left fold fl(..fl(fl(e0+e1)+e2)..) of E[t, pi_t] for each row."""
    E = np.asarray(E, dtype=np.float32)
    n, T = pi.shape
    acc = E[0, pi[:, 0]].astype(np.float32)
    for t in range(1, T):
        acc = (acc + E[t, pi[:, t]]).astype(np.float32)
    return acc


def states_of(pi_row: np.ndarray, blank: int) -> tuple:
    """Trellis state index of every frame of a valid alignment: a blank after
    k emitted tokens is state 2k, a frame of the k-th token is state 2k+1."""
    out = []
    k = 0                       # tokens started so far
    prev = None
    for c in pi_row:
        c = int(c)
        if c == blank:
            out.append(2 * k)
        else:
            if c != prev:
                k += 1
            out.append(2 * k - 1)
        prev = c
    return tuple(out)


def brute(E: np.ndarray, y, blank: int = 0):
    """All valid alignments with their float32 scores.

    Returns (pis [n, T], scores float32 [n]); n = 0 if no alignment exists."""
    E = np.asarray(E, dtype=np.float32)
    T, C = E.shape
    pis = all_sequences(T, C)
    m = collapses_to(pis, np.asarray(y), blank)
    pis = pis[m]
    if len(pis) == 0:
        return pis, np.zeros(0, dtype=np.float32)
    return pis, fold32(E, pis)


def best_by_tie_rule(E: np.ndarray, y, blank: int = 0):
    """The maximal-score alignment whose reversed state sequence is
    lexicographically largest, or None if no finite-score alignment exists."""
    pis, sc = brute(E, y, blank)
    if len(pis) == 0:
        return None
    top = sc.max()
    if top == -np.inf:
        return None
    cands = pis[sc == top]
    return max(cands, key=lambda r: tuple(reversed(states_of(r, blank))))
