"""CPU oracles for CTC forced alignment and CTC prefix beam search -- test
infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library under
``paper_2310_17864_amd`` never does, and shares no code with it.

The arithmetic lives in ``viterbi.c`` (forced alignment: plain C, one float
add per state and frame, strict-greater tie rule) and ``beam.c`` (prefix
beam search with blank collapse, float32 probabilities, fixed operation
order and tie rule); this module only marshals numpy arrays into them.
Status codes: 0 ok, 1 invalid input, 2 infeasible (alignment) / no
hypothesis (beam search).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "viterbi.c"), os.path.join(_HERE, "beam.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EINFEASIBLE, ENOMEM = 0, 1, 2, 3

_lib = None


def build(force: bool = False) -> str:
    """Compile the C sources with gcc: -O2, no fast-math, no FMA contraction."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f)
                                            for f in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall",
                               "-o", tmp] + _SRCS + ["-lpthread", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        lib.oracle_align_f32.argtypes = [P, i32, i32, P, i32, i32, P, P, P]
        lib.oracle_align_f32.restype = ctypes.c_int
        lib.oracle_align_f64.argtypes = [P, i32, i32, P, i32, i32, P, P, P]
        lib.oracle_align_f64.restype = ctypes.c_int
        lib.oracle_align_batch_f32.argtypes = [i32, P, P, P, P, P, P, P, i32,
                                               P, P, P, P, P, i32]
        lib.oracle_align_batch_f32.restype = ctypes.c_int
        f32 = ctypes.c_float
        lib.oracle_blank_collapse.argtypes = [P, i32, i32, i32, f32, P]
        lib.oracle_blank_collapse.restype = ctypes.c_int
        lib.oracle_beam_decode.argtypes = [P, i32, i32, i32, i32, f32, P, P, P, P, P]
        lib.oracle_beam_decode.restype = ctypes.c_int
        lib.oracle_beam_decode_ex.argtypes = [P, i32, i32, i32, i32, f32, P, P, P, P, P, P, P]
        lib.oracle_beam_decode_ex.restype = ctypes.c_int
        lib.oracle_beam_decode_batch.argtypes = [i32, P, P, P, i32, i32, i32, f32, P, P, P, P,
                                                 P, P, P, P, P, i32]
        lib.oracle_beam_decode_batch.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def align_f32(emission: np.ndarray, labels, blank: int = 0
              ) -> Tuple[int, np.ndarray, np.ndarray, float]:
    """(status, path int32[T], scores float32[T], total float32)."""
    lib = _load()
    E = np.ascontiguousarray(emission, dtype=np.float32)
    y = np.ascontiguousarray(np.asarray(labels, dtype=np.int32).reshape(-1))
    T, C = E.shape
    path = np.empty(T, dtype=np.int32)
    scores = np.empty(T, dtype=np.float32)
    total = np.zeros(1, dtype=np.float32)
    st = lib.oracle_align_f32(_ptr(E), T, C, _ptr(y) if y.size else None, y.size,
                              blank, _ptr(path), _ptr(scores), _ptr(total))
    return st, path, scores, np.float32(total[0])


def align_f64(emission: np.ndarray, labels, blank: int = 0
              ) -> Tuple[int, np.ndarray, np.ndarray, float]:
    """(status, path int32[T], scores float64[T], total float64)."""
    lib = _load()
    E = np.ascontiguousarray(emission, dtype=np.float32)
    y = np.ascontiguousarray(np.asarray(labels, dtype=np.int32).reshape(-1))
    T, C = E.shape
    path = np.empty(T, dtype=np.int32)
    scores = np.empty(T, dtype=np.float64)
    total = np.zeros(1, dtype=np.float64)
    st = lib.oracle_align_f64(_ptr(E), T, C, _ptr(y) if y.size else None, y.size,
                              blank, _ptr(path), _ptr(scores), _ptr(total))
    return st, path, scores, np.float64(total[0])


def align_batch_f32(packed: dict, blank: int = 0, threads: int = 1):
    """Align every utterance of a packed batch (see synth.pack) on `threads`
    POSIX threads.  Returns (status[n], paths[frames], scores[frames],
    totals[n], threads_used)."""
    lib = _load()
    n = int(packed["T"].shape[0])
    frames = int(packed["frames"])
    paths = np.empty(max(frames, 1), dtype=np.int32)
    scores = np.empty(max(frames, 1), dtype=np.float32)
    totals = np.empty(n, dtype=np.float32)
    status = np.empty(n, dtype=np.int32)
    arrs = {k: np.ascontiguousarray(packed[k]) for k in
            ("em", "em_off", "T", "C", "lab", "lab_off", "L", "fr_off")}
    used = lib.oracle_align_batch_f32(
        n, _ptr(arrs["em"]), _ptr(arrs["em_off"]), _ptr(arrs["T"]), _ptr(arrs["C"]),
        _ptr(arrs["lab"]), _ptr(arrs["lab_off"]), _ptr(arrs["L"]), blank,
        _ptr(paths), _ptr(scores), _ptr(arrs["fr_off"]), _ptr(totals), _ptr(status),
        int(threads))
    return status, paths[:frames], scores[:frames], totals, used


def token_spans(path, scores, blank: int = 0):
    """Token spans of a frame-level alignment (the step after alignment in a
    forced-alignment pipeline, paper Sec. 4: frame-level alignments are
    grouped per transcript token).

    A span is a maximal run of frames carrying the same non-blank class; in
    a CTC alignment two occurrences of one class are always separated by a
    blank, so there is exactly one span per transcript token.  Returns
    (token class int32[n], start int32[n], end int32[n] exclusive,
    score float32[n] = float32 left fold of the span's per-frame scores)."""
    path = np.asarray(path)
    scores = np.asarray(scores, dtype=np.float32)
    tok, st, en, sc = [], [], [], []
    t = 0
    T = len(path)
    while t < T:
        c = int(path[t])
        if c == blank or c < 0:
            t += 1
            continue
        s0 = t
        acc = np.float32(scores[t])
        t += 1
        while t < T and int(path[t]) == c:
            acc = np.float32(acc + scores[t])
            t += 1
        tok.append(c)
        st.append(s0)
        en.append(t)
        sc.append(acc)
    return (np.array(tok, np.int32), np.array(st, np.int32), np.array(en, np.int32),
            np.array(sc, np.float32))


# ---- CTC prefix beam search with blank collapse (beam.c) -------------------


def blank_collapse(y: np.ndarray, blank: int = 0, a: float = 1.0) -> np.ndarray:
    """Indices of the frames kept after blank collapse with threshold a
    (frame t is a blank frame when y[t, blank] > a; every maximal run of blank
    frames keeps its first frame only)."""
    lib = _load()
    y = np.ascontiguousarray(y, dtype=np.float32)
    T, V = y.shape
    kept = np.empty(max(T, 1), np.int32)
    n = lib.oracle_blank_collapse(_ptr(y), T, V, blank, np.float32(a), _ptr(kept))
    return kept[:n].copy()


def beam_decode(y: np.ndarray, blank: int = 0, beam: int = 10, a: float = 1.0, raw: bool = False):
    """CTC prefix beam search over per-frame probabilities y [T, V] (float32)
    after blank collapse with threshold a.  Returns (status, hyps, logp,
    n_kept): the final beam in rank order as a list of int32 label arrays and
    a float64 array of their log-probabilities; with raw=True also the scaled
    totals (float32, relative to 2^E) and E."""
    lib = _load()
    y = np.ascontiguousarray(y, dtype=np.float32)
    T, V = y.shape
    tok = np.zeros((beam, max(T, 1)), np.int32)
    ln = np.zeros(beam, np.int32)
    lp = np.zeros(beam, np.float64)
    n_out = np.zeros(1, np.int32)
    n_kept = np.zeros(1, np.int32)
    sc = np.zeros(beam, np.float32)
    ex = np.zeros(1, np.int32)
    st = lib.oracle_beam_decode_ex(_ptr(y), T, V, blank, beam, np.float32(a), _ptr(tok), _ptr(ln),
                                   _ptr(lp), _ptr(sc), _ptr(ex), _ptr(n_out), _ptr(n_kept))
    n = int(n_out[0])
    if raw:
        return (st, [tok[k, :ln[k]].copy() for k in range(n)], lp[:n].copy(), int(n_kept[0]),
                sc[:n].copy(), int(ex[0]))
    return st, [tok[k, :ln[k]].copy() for k in range(n)], lp[:n].copy(), int(n_kept[0])


def beam_decode_batch(packed: dict, blank: int = 0, beam: int = 10, a: float = 1.0,
                      threads: int = 1, raw: bool = False):
    """beam_decode over a packed batch (keys y, y_off, T, V).  Returns
    (status[n], hyps: list of lists of label arrays, logp: list of float64
    arrays, n_kept[n], threads_used)."""
    lib = _load()
    Ts = np.ascontiguousarray(packed["T"], dtype=np.int32)
    n = int(Ts.shape[0])
    V = int(packed["V"])
    tok_off = np.zeros(n, np.int64)
    if n:
        tok_off[1:] = np.cumsum(Ts.astype(np.int64) * beam)[:-1]
    tok = np.zeros(max(int(np.sum(Ts.astype(np.int64))) * beam, 1), np.int32)
    ln = np.zeros(max(n * beam, 1), np.int32)
    lp = np.zeros(max(n * beam, 1), np.float64)
    n_out = np.zeros(max(n, 1), np.int32)
    n_kept = np.zeros(max(n, 1), np.int32)
    status = np.zeros(max(n, 1), np.int32)
    sc = np.zeros(max(n * beam, 1), np.float32)
    ex = np.zeros(max(n, 1), np.int32)
    y = np.ascontiguousarray(packed["y"], dtype=np.float32)
    y_off = np.ascontiguousarray(packed["y_off"], dtype=np.int64)
    used = lib.oracle_beam_decode_batch(n, _ptr(y), _ptr(y_off), _ptr(Ts), V, blank, beam,
                                        np.float32(a), _ptr(tok), _ptr(tok_off), _ptr(ln), _ptr(lp),
                                        _ptr(sc), _ptr(ex), _ptr(n_out), _ptr(n_kept), _ptr(status),
                                        int(threads))
    hyps, logps, scaled = [], [], []
    for i in range(n):
        base = int(tok_off[i])
        T = int(Ts[i])
        hyps.append([tok[base + k * T: base + k * T + ln[i * beam + k]].copy()
                     for k in range(int(n_out[i]))])
        logps.append(lp[i * beam: i * beam + int(n_out[i])].copy())
        scaled.append(sc[i * beam: i * beam + int(n_out[i])].copy())
    if raw:
        return status[:n].copy(), hyps, logps, n_kept[:n].copy(), used, scaled, ex[:n].copy()
    return status[:n].copy(), hyps, logps, n_kept[:n].copy(), used
