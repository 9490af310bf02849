"""Brute force for CTC prefix beam search pins: the exact probability of
every label sequence, summed in float64 over every frame labelling that
collapses to it (merge runs, drop blanks).  Shares nothing with the oracle's
recursion."""
from __future__ import annotations

import itertools
from typing import Dict, Tuple

import numpy as np


def collapse(pi, blank: int) -> Tuple[int, ...]:
    out = []
    prev = None
    for c in pi:
        if c != prev and c != blank:
            out.append(int(c))
        prev = c
    return tuple(out)


def sequence_probs(y: np.ndarray, blank: int) -> Dict[Tuple[int, ...], float]:
    """{label sequence: P(sequence)} over all V**T frame labellings."""
    T, V = y.shape
    yd = y.astype(np.float64)
    probs: Dict[Tuple[int, ...], float] = {}
    for pi in itertools.product(range(V), repeat=T):
        p = 1.0
        for t, c in enumerate(pi):
            p *= yd[t, c]
        if p > 0.0:
            key = collapse(pi, blank)
            probs[key] = probs.get(key, 0.0) + p
    return probs


def random_probs(rng: np.random.Generator, T: int, V: int, conc: float = 0.7) -> np.ndarray:
    """Rows drawn from a Dirichlet distribution, rounded to float32."""
    return rng.dirichlet(np.full(V, conc), size=T).astype(np.float32)
