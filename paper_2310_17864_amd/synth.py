"""Seeded synthetic CTC alignment workloads.

This module only draws inputs: label sequences, a planted feasible CTC
alignment, and frame log-probabilities built around it.  It holds none of the
alignment arithmetic, so both the CPU oracle (in the tests) and the HIP path
consume exactly the arrays produced here.

What the paper fixes (Sec. 4, paragraph "CTC-based forced alignment"): the input
to forced alignment is a matrix of per-frame log-probabilities from a
CTC-trained network plus a transcript.  No dataset or trained model is used;
the workloads below stand in for such emissions with the shapes of the five
benchmark configurations:

* single utterance: T=200, C=32, L=40, ~10% adjacent label repeats;
* 64 utterances, T ~ U{500..1500}, L = round(T/5), C=32;
* long form: T=90,000, C=32, L=15,000, planted +4 over N(0, 1.5);
* 4,096 utterances, T log-uniform in [100, 6000], L ~ U{ceil(T/6)..floor(T/4)},
  exactly half at C=32 and half at C=256, labels i.i.d. over non-blank classes;
* serving: Poisson arrivals at 2,000 req/s, T log-uniform in [100, 30000],
  C in {32, 256} with probability 1/2 each.

Emission recipe (all configurations): logits ~ N(0, sigma) of shape [T, C];
+mu on the class of a random feasible planted CTC path at every frame;
log_softmax in float64; rounded once to float32.

Planted path: every label state lasts at least one frame, a blank between two
equal adjacent labels lasts at least one frame, other blanks may last zero
frames; the T - (L + R) remaining frames (R = number of adjacent repeats) are
spread multinomially and uniformly over the S = 2L + 1 states.

Every utterance i of a configuration draws from its own stream
``SeedSequence(seed).spawn(n + 1)[i]``; configuration-level draws (class
assignment, arrival times) use the extra child ``[n]``.  Results therefore do
not depend on batch order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Utterance", "Workload", "draw_labels", "planted_states", "emissions_around",
    "utterance", "cfg_single", "cfg_plain_batch", "cfg_long", "cfg_batched",
    "cfg_serving", "poisson_arrivals", "pack", "packed_parallel",
    "decode_states", "decode_probs", "decode_packed",
]


@dataclass
class Utterance:
    emission: np.ndarray          # float32 [T, C], row-major
    labels: np.ndarray            # int32 [L]
    blank: int = 0
    planted: Optional[np.ndarray] = None   # int32 [T] state index of the planted path

    @property
    def T(self) -> int:
        return int(self.emission.shape[0])

    @property
    def C(self) -> int:
        return int(self.emission.shape[1])

    @property
    def L(self) -> int:
        return int(self.labels.shape[0])


@dataclass
class Workload:
    name: str
    utts: List[Utterance]
    meta: dict = field(default_factory=dict)

    @property
    def frames(self) -> int:
        return int(sum(u.T for u in self.utts))


def draw_labels(rng: np.random.Generator, L: int, C: int, blank: int,
                repeat_p: Optional[float]) -> np.ndarray:
    """Transcript of L non-blank class ids.

    repeat_p=None: i.i.d. uniform over the C-1 non-blank classes.
    repeat_p=p:    y_0 uniform; y_i = y_{i-1} with probability p, otherwise
                   uniform over the C-2 non-blank classes other than y_{i-1}.
    """
    nonblank = np.array([c for c in range(C) if c != blank], dtype=np.int64)
    if L == 0:
        return np.zeros(0, dtype=np.int32)
    if repeat_p is None or C - 1 < 2:
        return nonblank[rng.integers(0, C - 1, size=L)].astype(np.int32)
    rep = rng.random(L) < repeat_p
    pick = rng.integers(0, C - 2, size=L)     # index among the C-2 "other" classes
    first = int(nonblank[rng.integers(0, C - 1)])
    out = np.empty(L, dtype=np.int64)
    out[0] = first
    # position of each class inside `nonblank`
    pos = np.full(C, -1, dtype=np.int64)
    pos[nonblank] = np.arange(C - 1)
    for i in range(1, L):
        prev = out[i - 1]
        if rep[i]:
            out[i] = prev
        else:
            k = pick[i]
            # skip over prev's slot so the draw is uniform over the others
            k = k + (k >= pos[prev])
            out[i] = nonblank[k]
    return out.astype(np.int32)


def planted_states(rng: np.random.Generator, T: int, labels: np.ndarray) -> np.ndarray:
    """State index (0..2L) of a random feasible CTC path over T frames."""
    L = int(labels.shape[0])
    S = 2 * L + 1
    dur = np.zeros(S, dtype=np.int64)
    dur[1::2] = 1
    if L > 1:
        dur[2:2 * L:2] = (labels[1:] == labels[:-1]).astype(np.int64)
    need = int(dur.sum())
    if T < need:
        raise ValueError(f"T={T} too short for a feasible path (needs {need})")
    dur += rng.multinomial(T - need, np.full(S, 1.0 / S))
    return np.repeat(np.arange(S, dtype=np.int32), dur)


def emissions_around(rng: np.random.Generator, states: np.ndarray, labels: np.ndarray,
                     C: int, blank: int, mu: float, sigma: float) -> np.ndarray:
    """float32 log-probabilities [T, C]: log_softmax(N(0, sigma) + mu at the planted class)."""
    T = int(states.shape[0])
    logits = rng.standard_normal((T, C)) * sigma
    cls = np.where(states % 2 == 0, blank,
                   labels[np.maximum(states - 1, 0) // 2] if labels.size else blank)
    logits[np.arange(T), cls] += mu
    m = logits.max(axis=1, keepdims=True)
    z = logits - m
    lse = np.log(np.exp(z).sum(axis=1, keepdims=True))
    return (z - lse).astype(np.float32)


def utterance(rng: np.random.Generator, T: int, C: int, L: int, blank: int = 0,
              mu: float = 6.0, sigma: float = 1.0,
              repeat_p: Optional[float] = 0.1) -> Utterance:
    labels = draw_labels(rng, L, C, blank, repeat_p)
    states = planted_states(rng, T, labels)
    em = emissions_around(rng, states, labels, C, blank, mu, sigma)
    return Utterance(np.ascontiguousarray(em), labels, blank, states)


def _children(seed: int, n: int):
    ss = np.random.SeedSequence(seed).spawn(n + 1)
    return [np.random.default_rng(s) for s in ss[:n]], np.random.default_rng(ss[n])


def _log_uniform_T(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def _L_quarter_sixth(rng: np.random.Generator, T: int) -> int:
    return int(rng.integers(math.ceil(T / 6), T // 4 + 1))


def cfg_single(T: int = 200, C: int = 32, L: int = 40, seed: int = 1) -> Workload:
    """Single utterance, plain method (T=200, C=32, L=40, ~10% repeats)."""
    rngs, _ = _children(seed, 1)
    u = utterance(rngs[0], T, C, L, 0, 6.0, 1.0, 0.1)
    return Workload("single_T200_C32_L40", [u], {"seed": seed})


def cfg_plain_batch(n: int = 64, t_lo: int = 500, t_hi: int = 1500, C: int = 32,
                    seed: int = 2) -> Workload:
    """n utterances, T ~ U{t_lo..t_hi}, L = round(T/5), one launch each."""
    rngs, _ = _children(seed, n)
    utts = []
    for r in rngs:
        T = int(r.integers(t_lo, t_hi + 1))
        utts.append(utterance(r, T, C, int(round(T / 5)), 0, 6.0, 1.0, 0.1))
    return Workload(f"plain{n}_T{t_lo}-{t_hi}_C{C}", utts, {"seed": seed})


def cfg_long(T: int = 90_000, C: int = 32, L: int = 15_000, seed: int = 3) -> Workload:
    """Long-form single alignment (30 min at 50 Hz): planted +4 over N(0, 1.5)."""
    rngs, _ = _children(seed, 1)
    u = utterance(rngs[0], T, C, L, 0, 4.0, 1.5, 0.1)
    return Workload(f"long_T{T}_C{C}_L{L}", [u], {"seed": seed})


def _spec_batched(r: np.random.Generator, C: int, t_lo: int, t_hi: int):
    T = _log_uniform_T(r, t_lo, t_hi)
    L = _L_quarter_sixth(r, T)
    return T, int(C), L


def _spec_serving(r: np.random.Generator, classes, t_lo: int, t_hi: int):
    T = _log_uniform_T(r, t_lo, t_hi)
    C = int(classes[int(r.integers(0, len(classes)))])
    L = _L_quarter_sixth(r, T)
    return T, C, L


def _batched_classes(top: np.random.Generator, n: int, classes):
    k = len(classes)
    cs = np.array([classes[i % k] for i in range(n)], dtype=np.int64)
    return cs[top.permutation(n)]


def cfg_batched(n: int = 4096, t_lo: int = 100, t_hi: int = 6000,
                classes=(32, 256), seed: int = 4) -> Workload:
    """n utterances, T log-uniform [t_lo, t_hi], L ~ U{ceil(T/6)..floor(T/4)},
    exactly n/len(classes) per class count by a seeded permutation, labels i.i.d."""
    rngs, top = _children(seed, n)
    cs = _batched_classes(top, n, classes)
    utts = []
    for r, C in zip(rngs, cs):
        T, C, L = _spec_batched(r, C, t_lo, t_hi)
        utts.append(utterance(r, T, C, L, 0, 6.0, 1.0, None))
    return Workload(f"batched{n}_T{t_lo}-{t_hi}_C{'/'.join(map(str, classes))}",
                    utts, {"seed": seed})


def cfg_serving(pool: int = 4096, t_lo: int = 100, t_hi: int = 30_000,
                classes=(32, 256), seed: int = 5) -> Workload:
    """Device-resident request pool with the serving distributions
    (T log-uniform [t_lo, t_hi], C uniform over `classes`)."""
    rngs, _ = _children(seed, pool)
    utts = []
    for r in rngs:
        T, C, L = _spec_serving(r, classes, t_lo, t_hi)
        utts.append(utterance(r, T, C, L, 0, 6.0, 1.0, None))
    return Workload(f"serving_pool{pool}_T{t_lo}-{t_hi}", utts, {"seed": seed})


# ---- the same workloads generated by a pool of forked workers -------------

_PAR = {}


def _par_work(i: int):
    """Worker: regenerate utterance i from its own stream into the shared
    emission buffer; return its labels."""
    g = _PAR
    r = np.random.default_rng(g["seqs"][i])
    if g["kind"] == "batched":
        T, C, L = _spec_batched(r, g["cs"][i], g["t_lo"], g["t_hi"])
    else:
        T, C, L = _spec_serving(r, g["classes"], g["t_lo"], g["t_hi"])
    u = utterance(r, T, C, L, 0, 6.0, 1.0, None)
    off = g["em_off"][i]
    g["em"][off:off + T * C] = u.emission.reshape(-1)
    return i, u.labels


def packed_parallel(kind: str, n: int, workers: int = 8, t_lo: int = 100, t_hi: int = 6000,
                    classes=(32, 256), seed: int = 4):
    """pack(cfg_batched(...).utts) (kind="batched") or pack(cfg_serving(...).utts)
    (kind="serving"), bit-identical, generated by `workers` forked processes
    writing into one anonymous shared mapping.  Call before any GPU work."""
    import mmap
    import multiprocessing as mp
    seqs = np.random.SeedSequence(seed).spawn(n + 1)
    top = np.random.default_rng(seqs[n])
    T = np.zeros(n, np.int32)
    C = np.zeros(n, np.int32)
    L = np.zeros(n, np.int32)
    cs = _batched_classes(top, n, classes) if kind == "batched" else None
    for i in range(n):       # shapes only: the first draws of each stream
        r = np.random.default_rng(seqs[i])
        if kind == "batched":
            T[i], C[i], L[i] = _spec_batched(r, cs[i], t_lo, t_hi)
        else:
            T[i], C[i], L[i] = _spec_serving(r, classes, t_lo, t_hi)
    em_off = np.zeros(n, np.int64)
    lab_off = np.zeros(n, np.int64)
    fr_off = np.zeros(n, np.int64)
    e = l = f = 0
    for i in range(n):
        em_off[i], lab_off[i], fr_off[i] = e, l, f
        e += (int(T[i]) * int(C[i]) + 63) // 64 * 64
        l += int(L[i])
        f += int(T[i])
    buf = mmap.mmap(-1, max(e, 1) * 4)
    em = np.frombuffer(buf, dtype=np.float32)
    _PAR.clear()
    _PAR.update(kind=kind, seqs=seqs, cs=cs, classes=classes, t_lo=t_lo, t_hi=t_hi,
                em_off=em_off, em=em)
    lab = np.zeros(max(l, 1), np.int32)
    ctx = mp.get_context("fork")
    with ctx.Pool(max(1, workers)) as pool:
        for i, y in pool.imap_unordered(_par_work, range(n), chunksize=4):
            lab[lab_off[i]:lab_off[i] + len(y)] = y
    _PAR.clear()
    return dict(em=em, lab=lab, em_off=em_off, lab_off=lab_off, fr_off=fr_off,
                T=T, C=C, L=L, frames=f, _buf=buf)


def poisson_arrivals(rate: float, seconds: float, pool: int, seed: int = 5):
    """(arrival times in s, pool indices) of a Poisson stream, seeded and
    independent of the pool's own streams."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xA221]))
    n = int(rng.poisson(rate * seconds))
    times = np.sort(rng.uniform(0.0, seconds, size=n))
    idx = rng.integers(0, pool, size=n)
    return times, idx


def pack(utts: List[Utterance]):
    """Concatenate a list of utterances into flat arrays plus offsets.

    Emission offsets are in elements and rounded up to a multiple of 64
    elements (256 bytes) so every utterance starts on an aligned address.
    """
    n = len(utts)
    em_off = np.zeros(n, dtype=np.int64)
    lab_off = np.zeros(n, dtype=np.int64)
    fr_off = np.zeros(n, dtype=np.int64)
    e = l = f = 0
    for i, u in enumerate(utts):
        em_off[i], lab_off[i], fr_off[i] = e, l, f
        e += (u.T * u.C + 63) // 64 * 64
        l += u.L
        f += u.T
    em = np.zeros(max(e, 1), dtype=np.float32)
    lab = np.zeros(max(l, 1), dtype=np.int32)
    for i, u in enumerate(utts):
        em[em_off[i]:em_off[i] + u.T * u.C] = u.emission.reshape(-1)
        lab[lab_off[i]:lab_off[i] + u.L] = u.labels
    T = np.array([u.T for u in utts], dtype=np.int32)
    C = np.array([u.C for u in utts], dtype=np.int32)
    L = np.array([u.L for u in utts], dtype=np.int32)
    return dict(em=em, lab=lab, em_off=em_off, lab_off=lab_off, fr_off=fr_off,
                T=T, C=C, L=L, frames=f)


# ---- CTC beam search decoding workload ---------------------------------------
#
# Stand-in for the paper's decoder benchmark (Sec. 5, "CUDA CTC decoder":
# LibriSpeech test-other through an acoustic model with a 500-token
# vocabulary, beam 10; neither the dataset nor the model is used here).
# Per-frame probabilities (softmax outputs, not logs) over V = 500 classes,
# peaky like a trained CTC model's: a planted CTC path gives each label one
# frame plus a geometric number of extra frames (mean 0.3), a blank between
# equal labels at least one frame, and spreads the remaining frames
# uniformly over the blank states, so most frames are blank; logits are
# N(0, 1) plus a boost on the planted class, drawn per frame from U(10, 16)
# (a confident frame: its class above ~0.96) with probability 0.9, else from
# U(2, 8) (an uncertain frame); softmax in float64, rounded once to float32.
# Labels are i.i.d. over the non-blank classes.  Utterances: T log-uniform in
# [50, 900] frames, L ~ U{ceil(T/8)..floor(T/4)} tokens.


def decode_states(rng: np.random.Generator, T: int, labels: np.ndarray) -> np.ndarray:
    """State index (0..2L) of a planted CTC path with short label runs."""
    L = int(labels.shape[0])
    S = 2 * L + 1
    dur = np.zeros(S, dtype=np.int64)
    dur[1::2] = 1 + rng.geometric(1.0 / 1.3, size=L) - 1
    if L > 1:
        dur[2:2 * L:2] = (labels[1:] == labels[:-1]).astype(np.int64)
    extra = T - int(dur.sum())
    if extra < 0:   # label runs too long for T: fall back to single frames
        dur[1::2] = 1
        extra = T - int(dur.sum())
    if extra < 0:
        raise ValueError(f"T={T} too short for L={L}")
    dur[0::2] += rng.multinomial(extra, np.full(L + 1, 1.0 / (L + 1)))
    return np.repeat(np.arange(S, dtype=np.int32), dur)


def decode_probs(rng: np.random.Generator, T: int, V: int, L: int, blank: int = 0,
                 confident: float = 0.9, sigma: float = 1.0):
    """(float32 probabilities [T, V], int32 planted labels [L])."""
    labels = draw_labels(rng, L, V, blank, None)
    states = decode_states(rng, T, labels)
    logits = rng.standard_normal((T, V)) * sigma
    cls = np.where(states % 2 == 0, blank,
                   labels[np.maximum(states - 1, 0) // 2] if labels.size else blank)
    sure = rng.random(T) < confident
    boost = np.where(sure, rng.uniform(10.0, 16.0, size=T), rng.uniform(2.0, 8.0, size=T))
    logits[np.arange(T), cls] += boost
    z = logits - logits.max(axis=1, keepdims=True)
    e = np.exp(z)
    return (e / e.sum(axis=1, keepdims=True)).astype(np.float32), labels


def _spec_decode(r: np.random.Generator, t_lo: int, t_hi: int):
    T = _log_uniform_T(r, t_lo, t_hi)
    L = int(r.integers(math.ceil(T / 8), T // 4 + 1))
    return T, L


_DEC = {}


def _dec_work(i: int):
    g = _DEC
    r = np.random.default_rng(g["seqs"][i])
    T, L = _spec_decode(r, g["t_lo"], g["t_hi"])
    y, _ = decode_probs(r, T, g["V"], L, 0)
    off = g["y_off"][i]
    g["y"][off:off + T * g["V"]] = y.reshape(-1)
    return i


def decode_packed(n: int = 2048, t_lo: int = 50, t_hi: int = 900, V: int = 500, seed: int = 6,
                  workers: int = 8):
    """The decoding workload packed flat: dict(y, y_off, T, V, frames), rows of
    utterance i at y[y_off[i]:...] ([T_i][V], offsets multiples of 64),
    generated by `workers` forked processes into one shared mapping (call
    before any GPU work).  Utterance i draws from SeedSequence(seed) child i."""
    import mmap
    import multiprocessing as mp
    seqs = np.random.SeedSequence(seed).spawn(n + 1)
    T = np.zeros(n, np.int32)
    for i in range(n):
        T[i], _ = _spec_decode(np.random.default_rng(seqs[i]), t_lo, t_hi)
    y_off = np.zeros(n, np.int64)
    e = 0
    for i in range(n):
        y_off[i] = e
        e += (int(T[i]) * V + 63) // 64 * 64
    buf = mmap.mmap(-1, max(e, 1) * 4)
    y = np.frombuffer(buf, dtype=np.float32)
    _DEC.clear()
    _DEC.update(seqs=seqs, t_lo=t_lo, t_hi=t_hi, V=V, y_off=y_off, y=y)
    if workers <= 1:
        for i in range(n):
            _dec_work(i)
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            for _ in pool.imap_unordered(_dec_work, range(n), chunksize=8):
                pass
    _DEC.clear()
    return dict(y=y, y_off=y_off, T=T, V=V, frames=int(T.astype(np.int64).sum()), _buf=buf)
