"""libctcalign: CTC forced alignment on AMD MI355X (gfx950).

Python face of the C library (include/ctcalign.h).  PyTorch provides device
memory and streams; every step of the alignment runs in hand-written HIP
kernels, and there is no CPU fallback: without the built library or a GPU
these functions raise.

    path, scores, total, status = align(emission_cuda_f32[T, C], labels_cuda_i32[L])

The method is the paper's forced alignment (Sec. 4, paragraph "CTC-based
forced alignment"): the highest-scoring CTC alignment of a transcript to
per-frame log-probabilities, with per-frame label ids and scores.
"""
from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (CtcAlignError, EAGAIN, EBUSY, EDEVICE, EINFEASIBLE, EINVAL, ENOMEM, OK,
                   LibraryMissing, strerror)

__all__ = ["align", "beam_decode", "BeamResult", "align_checkpointed", "checkpointed_workspace_bytes", "align_noalloc", "token_spans", "align_many_launches", "Context", "Plan", "Server", "workspace_bytes", "strerror",
           "CtcAlignError", "LibraryMissing", "OK", "EINVAL", "EINFEASIBLE", "ENOMEM",
           "EDEVICE", "EAGAIN", "EBUSY"]

_contexts: Dict[int, "Context"] = {}

# Live library objects, closed in dependency order (servers, then plans, then
# contexts) by an exit hook that runs while the HIP runtime is still up.
# After it has run -- or once the interpreter is finalizing -- close() and
# __del__ make no library call at all.
_live = {"server": weakref.WeakSet(), "plan": weakref.WeakSet(), "context": weakref.WeakSet()}
_closed_at_exit = False


def _library_usable() -> bool:
    return not _closed_at_exit and not sys.is_finalizing()


@atexit.register
def _close_all_at_exit():
    global _closed_at_exit
    for kind in ("server", "plan", "context"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass
    _contexts.clear()
    _closed_at_exit = True


PACK_WAVES = 4   # wavefronts per work item of the batched kernel


def _torch():
    import torch
    return torch


def _stream_handle(device) -> int:
    torch = _torch()
    return int(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A library context on one device (stream, workspace arena, tuning table)."""

    def __init__(self, device: int = 0):
        lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(lib.ctcalign_ctx_create(int(device), ctypes.byref(h)), "ctx_create")
        self.handle = h
        self.device = int(device)
        _live["context"].add(self)

    def close(self):
        if getattr(self, "handle", None):
            if _library_usable():
                _lib.load().ctcalign_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, T: int, L: int, C: int) -> int:
        return int(_lib.load().ctcalign_workspace_bytes(self.handle, T, L, C))

    # geometry table (kind 0: single launches, 1: batched persistent kernel)
    def tune_set(self, kind: int, s_lo: int, s_hi: int, C: int, W: int, M: int):
        _lib.check(_lib.load().ctcalign_tune_set(self.handle, kind, s_lo, s_hi, C, W, M), "tune_set")

    def tune_clear(self, kind: int, s_lo: int, s_hi: int, C: int):
        self.tune_set(kind, s_lo, s_hi, C, 0, 0)

    def tune_get(self, kind: int, S: int, C: int):
        W, M = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.load().ctcalign_tune_get(self.handle, kind, S, C, ctypes.byref(W),
                                                 ctypes.byref(M)), "tune_get")
        return int(W.value), int(M.value)

    KNOBS = {"pack_target_m": 1, "crit_frac": 2, "crit_per_cu": 3}

    def tune_knob(self, name: str, value: Optional[float] = None) -> float:
        """Sets a scheduling knob of batched plans (ctcalign_tune_knob) and
        returns its previous value; value=None only reads it."""
        prev = ctypes.c_double()
        lib = _lib.load()
        k = self.KNOBS[name]
        if value is None:
            lib.ctcalign_tune_knob(self.handle, k, -1.0, ctypes.byref(prev))
            return float(prev.value)
        _lib.check(lib.ctcalign_tune_knob(self.handle, k, float(value), ctypes.byref(prev)),
                   "tune_knob")
        return float(prev.value)

    def tune_save(self, path: str):
        _lib.check(_lib.load().ctcalign_tune_save(self.handle, path.encode()), "tune_save")

    def tune_load(self, path: str):
        _lib.check(_lib.load().ctcalign_tune_load(self.handle, path.encode()), "tune_load")


def context(device: Optional[int] = None) -> Context:
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _contexts:
        _contexts[dev] = Context(dev)
    return _contexts[dev]


def workspace_bytes(T: int, L: int, C: int, device: Optional[int] = None) -> int:
    return context(device).workspace_bytes(T, L, C)


def _check_dev_tensor(x, dtype, name):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def align(emission, labels, blank: int = 0, out=None, workspace=None, sync: bool = True):
    """Forced alignment of one utterance on the current stream.

    emission: float32 [T, C] device tensor (log-probabilities); labels: int32
    [L] device tensor.  Returns (path int32[T], scores float32[T],
    total float32[1], status int32[1]) device tensors; with sync=True the
    call waits and raises CtcAlignError on EINVAL / EINFEASIBLE.
    """
    torch = _torch()
    _check_dev_tensor(emission, torch.float32, "emission")
    _check_dev_tensor(labels, torch.int32, "labels")
    if emission.dim() != 2:
        raise ValueError("emission must be [T, C]")
    T, C = emission.shape
    L = labels.numel()
    dev = emission.device
    ctx = context(dev.index)
    if out is None:
        path = torch.empty(T, dtype=torch.int32, device=dev)
        scores = torch.empty(T, dtype=torch.float32, device=dev)
        total = torch.empty(1, dtype=torch.float32, device=dev)
        status = torch.empty(1, dtype=torch.int32, device=dev)
    else:
        path, scores, total, status = out
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    rc = _lib.load().ctcalign_align_ex(
        ctx.handle, emission.data_ptr(), T, C, labels.data_ptr() if L else None, L, blank,
        path.data_ptr(), scores.data_ptr(), total.data_ptr(), status.data_ptr(),
        ws_ptr, ws_bytes, _stream_handle(dev))
    _lib.check(rc, "align")
    if sync:
        st = int(status.item())
        if st != OK:
            raise CtcAlignError(st, "align")
    return path, scores, total, status


def align_checkpointed(emission, labels, blank: int = 0, every: int = 0, out=None,
                       workspace=None, sync: bool = True):
    """align() with a workspace that grows like sqrt(T): column checkpoints
    every `every` frames (0: about 4.6 sqrt(T)) and backpointers for one
    stretch at a time, bitwise the same results (ctcalign_align_checkpointed)."""
    torch = _torch()
    _check_dev_tensor(emission, torch.float32, "emission")
    _check_dev_tensor(labels, torch.int32, "labels")
    if emission.dim() != 2:
        raise ValueError("emission must be [T, C]")
    T, C = emission.shape
    L = labels.numel()
    dev = emission.device
    ctx = context(dev.index)
    if out is None:
        out = (torch.empty(T, dtype=torch.int32, device=dev),
               torch.empty(T, dtype=torch.float32, device=dev),
               torch.empty(1, dtype=torch.float32, device=dev),
               torch.empty(1, dtype=torch.int32, device=dev))
    path, scores, total, status = out
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().ctcalign_align_checkpointed(
        ctx.handle, emission.data_ptr(), T, C, labels.data_ptr() if L else None, L, blank,
        path.data_ptr(), scores.data_ptr(), total.data_ptr(), status.data_ptr(), int(every),
        ws_ptr, ws_bytes, _stream_handle(dev)), "align_checkpointed")
    if sync:
        st = int(status.item())
        if st != OK:
            raise CtcAlignError(st, "align_checkpointed")
    return path, scores, total, status


def checkpointed_workspace_bytes(T: int, L: int, C: int, every: int = 0,
                                 device: Optional[int] = None) -> int:
    return int(_lib.load().ctcalign_checkpointed_workspace_bytes(context(device).handle, T, L, C,
                                                                 int(every)))


class BeamResult:
    """Device outputs of beam_decode (tensors on the probabilities' device)."""

    def __init__(self, tokens, tok_off, T, beam, lengths, logp, scaled, exp2, nhyp, nkept, status):
        self.tokens, self.tok_off, self.T, self.beam = tokens, tok_off, T, beam
        self.lengths, self.logp, self.scaled, self.exp2 = lengths, logp, scaled, exp2
        self.nhyp, self.nkept, self.status = nhyp, nkept, status

    def hypotheses(self, i: int):
        """Final beam of utterance i as (list of int32 label arrays, float32
        log-probabilities), in rank order (copies to the host)."""
        n = int(self.nhyp[i].item())
        T = int(self.T[i])
        base = int(self.tok_off[i])
        toks = self.tokens[base: base + self.beam * T].view(self.beam, T).cpu().numpy()
        lens = self.lengths[i * self.beam: i * self.beam + n].cpu().numpy()
        lp = self.logp[i * self.beam: i * self.beam + n].cpu().numpy()
        return [toks[k, :lens[k]].copy() for k in range(n)], lp


def beam_decode(probs, prob_off, T, blank: int = 0, beam: int = 10, threshold: float = 1.0,
                V: Optional[int] = None):
    """CTC prefix beam search with blank collapse (ctcalign_beam_decode) over
    N utterances whose per-frame probabilities sit in one flat float32 device
    tensor: utterance i has T[i] frames of V classes at element prob_off[i].
    Asynchronous on the current stream; returns a BeamResult."""
    torch = _torch()
    _check_dev_tensor(probs, torch.float32, "probs")
    dev = probs.device
    ctx = context(dev.index)
    Tn = np.ascontiguousarray(T, dtype=np.int32)
    off = np.ascontiguousarray(prob_off, dtype=np.int64)
    n = int(Tn.shape[0])
    if V is None:
        if probs.dim() != 2 or n != 1:
            raise ValueError("V is needed for a flat batch")
        V = int(probs.shape[1])
    tok_off = np.zeros(n, np.int64)
    if n:
        tok_off[1:] = np.cumsum(Tn.astype(np.int64) * beam)[:-1]
    tokens = torch.zeros(max(int(np.sum(Tn.astype(np.int64))) * beam, 1), dtype=torch.int32, device=dev)
    lengths = torch.zeros(max(n * beam, 1), dtype=torch.int32, device=dev)
    logp = torch.empty(max(n * beam, 1), dtype=torch.float32, device=dev)
    scaled = torch.empty(max(n * beam, 1), dtype=torch.float32, device=dev)
    exp2 = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    nhyp = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    nkept = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    status = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _lib.check(_lib.load().ctcalign_beam_decode(
        ctx.handle, n, probs.data_ptr(), ptr(off), ptr(Tn), int(V), int(blank), int(beam),
        ctypes.c_float(threshold), tokens.data_ptr(), ptr(tok_off), lengths.data_ptr(),
        logp.data_ptr(), scaled.data_ptr(), exp2.data_ptr(), nhyp.data_ptr(), nkept.data_ptr(),
        status.data_ptr(), None, 0, _stream_handle(dev)), "beam_decode")
    return BeamResult(tokens, tok_off, Tn, beam, lengths, logp, scaled, exp2, nhyp, nkept, status)


def align_noalloc(emission, labels, blank: int = 0, out=None):
    """align() through ctcalign_align_noalloc: no device allocation inside
    the library call (backpointers in the library's fixed per-device scratch
    array; calls must not overlap on one device).  Returns (path, scores,
    total, status) device tensors on the current stream, without waiting."""
    torch = _torch()
    _check_dev_tensor(emission, torch.float32, "emission")
    _check_dev_tensor(labels, torch.int32, "labels")
    if emission.dim() != 2:
        raise ValueError("emission must be [T, C]")
    T, C = emission.shape
    L = labels.numel()
    dev = emission.device
    ctx = context(dev.index)
    if out is None:
        out = (torch.empty(T, dtype=torch.int32, device=dev),
               torch.empty(T, dtype=torch.float32, device=dev),
               torch.empty(1, dtype=torch.float32, device=dev),
               torch.empty(1, dtype=torch.int32, device=dev))
    path, scores, total, status = out
    _lib.check(_lib.load().ctcalign_align_noalloc(
        ctx.handle, emission.data_ptr(), T, C, labels.data_ptr() if L else None, L, blank,
        path.data_ptr(), scores.data_ptr(), total.data_ptr(), status.data_ptr(),
        _stream_handle(dev)), "align_noalloc")
    return path, scores, total, status


def token_spans(path, scores, blank: int = 0, max_spans: Optional[int] = None):
    """Token spans of an alignment on the device: (token, start, end, score)
    int32/int32/int32/float32 device tensors, one entry per transcript token."""
    torch = _torch()
    _check_dev_tensor(path, torch.int32, "path")
    _check_dev_tensor(scores, torch.float32, "scores")
    T = path.numel()
    n = T if max_spans is None else int(max_spans)
    dev = path.device
    tok = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    st = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    en = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    sc = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    _lib.check(_lib.load().ctcalign_token_spans(
        path.data_ptr(), scores.data_ptr(), T, blank, n, tok.data_ptr(), st.data_ptr(),
        en.data_ptr(), sc.data_ptr(), cnt.data_ptr(), _stream_handle(dev)), "token_spans")
    k = min(int(cnt.item()), n)
    return tok[:k], st[:k], en[:k], sc[:k]


def align_many_launches(emissions: Sequence, labels: Sequence, blank: int = 0):
    """One kernel launch per utterance, all on the current stream (the plain
    per-utterance method).  Returns a list of (path, scores, total, status)."""
    return [align(e, l, blank, sync=False) for e, l in zip(emissions, labels)]


class Plan:
    """Batched alignment of many utterances packed in flat device buffers:
    sorted longest first into a device work queue drained by one persistent
    kernel, the whole launch captured in a HIP graph and replayed by run()."""

    def __init__(self, emissions, em_off, T, C, labels, lab_off, L, frame_off, blank: int = 0,
                 outputs=None, ctx: Optional[Context] = None):
        torch = _torch()
        _check_dev_tensor(emissions, torch.float32, "emissions")
        _check_dev_tensor(labels, torch.int32, "labels")
        dev = emissions.device
        self.ctx = ctx or context(dev.index)
        self.n = n = int(len(T))
        frames = int(np.sum(np.asarray(T, dtype=np.int64)))
        self.host = {
            "em_off": np.ascontiguousarray(em_off, dtype=np.int64),
            "T": np.ascontiguousarray(T, dtype=np.int32),
            "C": np.ascontiguousarray(C, dtype=np.int32),
            "lab_off": np.ascontiguousarray(lab_off, dtype=np.int64),
            "L": np.ascontiguousarray(L, dtype=np.int32),
            "frame_off": np.ascontiguousarray(frame_off, dtype=np.int64),
        }
        if outputs is None:
            self.paths = torch.empty(max(frames, 1), dtype=torch.int32, device=dev)
            self.scores = torch.empty(max(frames, 1), dtype=torch.float32, device=dev)
            self.totals = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
            self.status = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        else:
            self.paths, self.scores, self.totals, self.status = outputs
        self._keep = (emissions, labels)
        h = self.host
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        handle = ctypes.c_void_p()
        rc = _lib.load().ctcalign_plan_create(
            self.ctx.handle, n, emissions.data_ptr(), ptr(h["em_off"]), ptr(h["T"]), ptr(h["C"]),
            labels.data_ptr(), ptr(h["lab_off"]), ptr(h["L"]), blank,
            self.paths.data_ptr(), self.scores.data_ptr(), ptr(h["frame_off"]),
            self.totals.data_ptr(), self.status.data_ptr(), ctypes.byref(handle))
        _lib.check(rc, "plan_create")
        self.handle = handle
        _live["plan"].add(self)

    def run(self, stream=None):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.paths.device)
        _lib.check(_lib.load().ctcalign_plan_run(self.handle, int(s.cuda_stream)), "plan_run")

    def trace(self):
        """(times int64[npacks, 3] = start, end, hw id; insts int32[npacks, 4])
        of the last run; needs CTCALIGN_TRACE=1 when the plan was created."""
        n = ctypes.c_int32()
        _lib.load().ctcalign_plan_trace(self.handle, 0, None, None, ctypes.byref(n))
        times = np.zeros((n.value, 3), dtype=np.int64)
        insts = np.zeros((n.value, PACK_WAVES), dtype=np.int32)
        _lib.check(_lib.load().ctcalign_plan_trace(
            self.handle, n.value, times.ctypes.data_as(ctypes.c_void_p),
            insts.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)), "plan_trace")
        return times, insts

    def close(self):
        if getattr(self, "handle", None):
            if _library_usable():
                _lib.load().ctcalign_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching alignment server on one device.

    submit() queues a request whose tensors stay on the device (written before
    the call); the library's worker thread admits requests in arrival order
    while their backpointer memory fits `budget_bytes` and hands each admitted
    group to a resident kernel, where it runs beside the requests admitted
    before it; each request completes on its own.  wait()/poll() return
    (status, timing) with timing = (submit, admit, launch, done) on the
    monotonic clock (launch: handed to the device).
    """

    def __init__(self, budget_bytes: int, max_inflight: int = 4096, ctx: Optional[Context] = None,
                 device: Optional[int] = None):
        self.ctx = ctx or context(device)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().ctcalign_server_create(self.ctx.handle, int(budget_bytes),
                                                      int(max_inflight), ctypes.byref(h)),
                   "server_create")
        self.handle = h
        self._keep = {}
        _live["server"].add(self)

    def submit(self, emission, labels, out_path, out_scores, out_total=None, blank: int = 0) -> int:
        """Queues one alignment.  An event recorded on the current stream goes
        with the request: the server admits it only once the work queued so
        far on that stream (which writes the emission and labels) is done."""
        torch = _torch()
        T, C = emission.shape
        L = labels.numel()
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(emission.device))
        req = _lib.Request(emission.data_ptr(), T, C, labels.data_ptr() if L else None, L, blank,
                           out_path.data_ptr(), out_scores.data_ptr(),
                           out_total.data_ptr() if out_total is not None else None,
                           ev.cuda_event)
        t = ctypes.c_uint64()
        _lib.check(_lib.load().ctcalign_server_submit(self.handle, ctypes.byref(req),
                                                      ctypes.byref(t)), "server_submit")
        self._keep[t.value] = (emission, labels, out_path, out_scores, out_total, ev)
        return int(t.value)

    def _finish(self, ticket: int, block: bool):
        st = ctypes.c_int32()
        tm = _lib.Timing()
        fn = _lib.load().ctcalign_server_wait if block else _lib.load().ctcalign_server_poll
        rc = fn(self.handle, ctypes.c_uint64(ticket), ctypes.byref(st), ctypes.byref(tm))
        if rc == EBUSY:
            return None
        _lib.check(rc, "server_wait" if block else "server_poll")
        self._keep.pop(ticket, None)
        return int(st.value), (tm.submit_s, tm.admit_s, tm.launch_s, tm.done_s)

    def wait(self, ticket: int):
        return self._finish(ticket, True)

    def poll(self, ticket: int):
        return self._finish(ticket, False)

    def stats(self) -> dict:
        st = _lib.ServerStats()
        _lib.check(_lib.load().ctcalign_server_get_stats(self.handle, ctypes.byref(st)), "stats")
        return {k: getattr(st, k) for k, _ in _lib.ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            if _library_usable():
                _lib.load().ctcalign_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
