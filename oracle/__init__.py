"""CPU oracle for CTC forced alignment -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library under
``paper_2310_17864_amd`` never does, and shares no code with it.

The arithmetic lives in ``viterbi.c`` (plain C, one float add per state and
frame, strict-greater tie rule); this module only marshals numpy arrays into
it.  Status codes: 0 ok, 1 invalid labels, 2 infeasible.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "viterbi.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EINFEASIBLE, ENOMEM = 0, 1, 2, 3

_lib = None


def build(force: bool = False) -> str:
    """Compile viterbi.c with gcc: -O2, no fast-math, no FMA contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall",
                               "-o", tmp, _SRC, "-lpthread", "-lm"])
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
