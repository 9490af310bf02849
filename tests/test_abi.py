"""The C-ABI library loads and exports every function include/ctcalign.h
declares; host-side argument checks answer before any device work (CPU)."""
import ctypes

import pytest

from paper_2310_17864_amd import _lib


def test_header_symbols_exported():
    lib = _lib.load()
    names = _lib.header_functions()
    assert "ctcalign_align" in names and "ctcalign_plan_create" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_binding_covers_header():
    # every declared function has a ctypes prototype in the binding
    assert sorted(_lib._PROTOS) == _lib.header_functions()


def test_strerror_and_version():
    lib = _lib.load()
    for code in range(7):
        assert lib.ctcalign_strerror(code)
    assert lib.ctcalign_strerror(99) == b"unknown status"
    assert lib.ctcalign_version() >= 100


@pytest.mark.parametrize("args", [
    (None, 10, 32, 1, 3, 0, 1, 1),          # null emission
    (1, 0, 32, 1, 3, 0, 1, 1),              # T < 1
    (1, 10, 0, 1, 3, 0, 1, 1),              # C < 1
    (1, 10, 257, 1, 3, 0, 1, 1),            # C above the supported maximum
    (1, 10, 32, 1, -1, 0, 1, 1),            # L < 0
    (1, 10, 32, None, 3, 0, 1, 1),          # labels missing
    (1, 10, 32, 1, 3, 32, 1, 1),            # blank out of range
    (1, 10, 32, 1, 3, -1, 1, 1),            # negative blank
    (1, 10, 32, 1, 3, 0, None, 1),          # null path
    (1, 10, 32, 1, 3, 0, 1, None),          # null scores
    (1, 10, 32, 1, 20000, 0, 1, 1),         # trellis larger than one workgroup holds
])
def test_host_argument_errors(args):
    lib = _lib.load()
    # pointers are never dereferenced: validation runs before any HIP call
    assert lib.ctcalign_align(*args) == _lib.EINVAL


def test_null_context_rejected():
    lib = _lib.load()
    assert lib.ctcalign_align_ex(None, 1, 10, 32, 1, 3, 0, 1, 1, None, None, None, 0, None) == _lib.EINVAL
    assert lib.ctcalign_plan_run(None, None) == _lib.EINVAL
    assert lib.ctcalign_plan_destroy(None) == _lib.OK
    assert lib.ctcalign_ctx_destroy(None) == _lib.OK
    assert lib.ctcalign_workspace_bytes(None, 10, 3, 32) == 0
    out = ctypes.c_void_p()
    assert lib.ctcalign_plan_create(None, 1, None, None, None, None, None, None, None, 0,
                                    None, None, None, None, None, ctypes.byref(out)) == _lib.EINVAL
