"""The pins are sharp: each plausible mistake planted into a copy of the
oracle's C source (a flipped tie, a dropped transition, a transposed operand,
an off-by-one) must fail at least one pin.  CPU only; the committed oracle is
never modified."""
import ctypes
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "viterbi.c")

MUTANTS = {
    "tie_s_vs_s1": ("if (s >= 1 && prev[s - 1] > best)", "if (s >= 1 && prev[s - 1] >= best)"),
    "tie_s2": ("prev[s - 2] > best) { best = prev[s - 2]; k = 2; }",
               "prev[s - 2] >= best) { best = prev[s - 2]; k = 2; }"),
    "skip_rule_inverted": ("s >= 3 && yprime(y, blank, s) != yprime(y, blank, s - 2)",
                           "s >= 3 && yprime(y, blank, s) == yprime(y, blank, s - 2)"),
    "no_skip": ("if (s % 2 == 1 && s >= 3", "if (0 && s % 2 == 1 && s >= 3"),
    "skip_into_blank": ("if (s % 2 == 1 && s >= 3 && yprime(y, blank, s) != yprime(y, blank, s - 2)",
                        "if (s >= 2 && (s % 2 == 0 || yprime(y, blank, s) != yprime(y, blank, s - 2))"),
    "init_one_state": ("prev[s] = (s <= 1) ? E[", "prev[s] = (s <= 0) ? E["),
    "end_tie": ("send = (prev[S - 2] > prev[S - 1])", "send = (prev[S - 2] >= prev[S - 1])"),
    "end_always_last": ("send = (prev[S - 2] > prev[S - 1]) ? S - 2 : S - 1;", "send = S - 1;"),
    "emission_transposed": ("cur[s] = Et[yprime(y, blank, s)] + best;",
                            "cur[s] = E[(int64_t)yprime(y, blank, s) * T + t] + best;"),
    "emission_prev_frame": ("cur[s] = Et[yprime(y, blank, s)] + best;",
                            "cur[s] = Et[yprime(y, blank, s) - C] + best;"),
    "scores_reversed": ("scores[t] = E[(int64_t)t * C + c];",
                        "scores[t] = E[(int64_t)(T - 1 - t) * C + c];"),
    "backtrack_off_by_one": ("if (t > 0) s -= bp[(int64_t)t * S + s];",
                             "if (t > 0) s -= bp[(int64_t)(t - 1) * S + s];"),
    "blank_parity": ("return (s % 2 == 0) ? blank : y[(s - 1) / 2];",
                     "return (s % 2 == 1) ? blank : y[s / 2];"),
    "max_not_sum": ("cur[s] = Et[yprime(y, blank, s)] + best;",
                    "cur[s] = Et[yprime(y, blank, s)] > best ? Et[yprime(y, blank, s)] : best;"),
}


def _build_variant(name, find, repl, tmp):
    src = open(SRC).read()
    assert src.count(find) >= 1, f"mutation {name}: pattern not found"
    # mutate only the float variant (the first occurrence)
    src = src.replace(find, repl, 1)
    c = os.path.join(tmp, f"{name}.c")
    so = os.path.join(tmp, f"lib{name}.so")
    open(c, "w").write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-w",
                           "-o", so, c, "-lpthread", "-lm"])
    lib = ctypes.CDLL(so)
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.oracle_align_f32.argtypes = [P, i32, i32, P, i32, i32, P, P, P]
    lib.oracle_align_f32.restype = ctypes.c_int

    def align(E, y, blank=0):
        E = np.ascontiguousarray(E, dtype=np.float32)
        y = np.ascontiguousarray(np.asarray(y, dtype=np.int32).reshape(-1))
        T, C = E.shape
        path = np.empty(T, np.int32)
        scores = np.empty(T, np.float32)
        tot = np.zeros(1, np.float32)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        st = lib.oracle_align_f32(ptr(E), T, C, ptr(y) if y.size else None, y.size, blank,
                                  ptr(path), ptr(scores), ptr(tot))
        return st, path, scores, np.float32(tot[0])
    return align


def _run_pins(name):
    """Exit status 0 when the mutant passes every pin, 1 when one fails."""
    find, repl = MUTANTS[name]
    with tempfile.TemporaryDirectory() as tmp:
        align = _build_variant(name, find, repl, tmp)
        checks = [
            lambda: pins.check_brute(align, pins.tiny_cases(1, 80)),
            lambda: pins.check_tie_rule(align, pins.tiny_cases(4, 80, integer=True)),
            lambda: pins.check_closed_forms(align),
        ]
        for chk in checks:
            if chk():
                return 1
    return 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    # a mutant may also read out of bounds and crash; run it in a child
    # process, where a crash counts as a caught mistake
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys; sys.path[:0] = [%r, %r]; import test_oracle_mutants as m; "
            "sys.exit(m._run_pins(%r))" % (here, os.path.dirname(here), name))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin\n{r.stderr[-2000:]}"
