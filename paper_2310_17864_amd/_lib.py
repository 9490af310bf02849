"""ctypes view of libctcalign.so (include/ctcalign.h).

Argument marshalling only: every step of the alignment runs in the library's
gfx950 kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctcalign.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ctcalign.h")

OK, EINVAL, EINFEASIBLE, ENOMEM, EDEVICE, EAGAIN, EBUSY = range(7)

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
SZ = ctypes.c_size_t

class Request(ctypes.Structure):
    _fields_ = [("emission", P), ("T", I32), ("C", I32), ("labels", P), ("L", I32),
                ("blank", I32), ("out_path", P), ("out_scores", P), ("out_total", P),
                ("ready_event", P)]


class Timing(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("launch_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("timeouts", ctypes.c_uint64),
                ("readmitted", ctypes.c_uint64),
                ("peak_charge_bytes", SZ), ("budget_bytes", SZ), ("peak_inflight", I32),
                ("waiting", I32), ("inflight", I32), ("budget_violated", I32)]


_PROTOS = {
    "ctcalign_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ctcalign_version": (ctypes.c_int, []),
    "ctcalign_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(P)]),
    "ctcalign_ctx_destroy": (ctypes.c_int, [P]),
    "ctcalign_workspace_bytes": (SZ, [P, I32, I32, I32]),
    "ctcalign_align": (ctypes.c_int, [P, I32, I32, P, I32, I32, P, P]),
    "ctcalign_align_ex": (ctypes.c_int, [P, P, I32, I32, P, I32, I32, P, P, P, P, P, SZ, P]),
    "ctcalign_align_checkpointed": (ctypes.c_int, [P, P, I32, I32, P, I32, I32, P, P, P, P, I32,
                                                   P, SZ, P]),
    "ctcalign_checkpointed_workspace_bytes": (SZ, [P, I32, I32, I32, I32]),
    "ctcalign_beam_decode": (ctypes.c_int, [P, I32, P, P, P, I32, I32, I32, ctypes.c_float, P, P,
                                            P, P, P, P, P, P, P, P, SZ, P]),
    "ctcalign_beam_workspace_bytes": (SZ, [I32, P, I32]),
    "ctcalign_align_noalloc": (ctypes.c_int, [P, P, I32, I32, P, I32, I32, P, P, P, P, P]),
    "ctcalign_noalloc_scratch_bytes": (SZ, []),
    "ctcalign_token_spans": (ctypes.c_int, [P, P, I32, I32, I32, P, P, P, P, P, P]),
    "ctcalign_plan_create": (ctypes.c_int, [P, I32, P, P, P, P, P, P, P, I32, P, P, P, P, P,
                                            ctypes.POINTER(P)]),
    "ctcalign_plan_run": (ctypes.c_int, [P, P]),
    "ctcalign_plan_destroy": (ctypes.c_int, [P]),
    "ctcalign_plan_trace": (ctypes.c_int, [P, I32, P, P, ctypes.POINTER(I32)]),
    "ctcalign_align_batched": (ctypes.c_int, [P, I32, P, P, P, P, P, P, P, I32, P, P, P, P, P, P]),
    "ctcalign_tune_set": (ctypes.c_int, [P, I32, I32, I32, I32, I32, I32]),
    "ctcalign_tune_get": (ctypes.c_int, [P, I32, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    "ctcalign_tune_knob": (ctypes.c_int, [P, I32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "ctcalign_tune_save": (ctypes.c_int, [P, ctypes.c_char_p]),
    "ctcalign_tune_load": (ctypes.c_int, [P, ctypes.c_char_p]),
    "ctcalign_server_create": (ctypes.c_int, [P, SZ, I32, ctypes.POINTER(P)]),
    "ctcalign_server_submit": (ctypes.c_int, [P, ctypes.POINTER(Request),
                                              ctypes.POINTER(ctypes.c_uint64)]),
    "ctcalign_server_poll": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.POINTER(I32),
                                            ctypes.POINTER(Timing)]),
    "ctcalign_server_wait": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.POINTER(I32),
                                            ctypes.POINTER(Timing)]),
    "ctcalign_server_get_stats": (ctypes.c_int, [P, ctypes.POINTER(ServerStats)]),
    "ctcalign_server_destroy": (ctypes.c_int, [P]),
}

_lib = None


class LibraryMissing(ImportError):
    pass


def header_functions():
    """Names of every function include/ctcalign.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ctcalign_[a-z_0-9]+)\s*\(", txt)))


def load():
    """The loaded library with prototypes set; raises LibraryMissing if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            f"{LIB_PATH} is not built; run `python -m paper_2310_17864_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().ctcalign_strerror(int(code)).decode()


class CtcAlignError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = int(code)
        super().__init__(f"{what}: {strerror(code)} (status {code})" if what else strerror(code))


def check(code: int, what: str = ""):
    if code != OK:
        raise CtcAlignError(code, what)
