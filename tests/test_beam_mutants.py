"""The beam-search pins are sharp: each plausible mistake planted into a copy
of oracle/beam.c (a reversed tie key, the repeat rule ignoring the blank
separation, a missing merge of equal prefixes, a blank run dropped whole, a
lost scale exponent, ...) must fail at least one pin of
tests/test_beam_oracle.py.  CPU only; the committed oracle is never
modified."""
import ctypes
import os
import subprocess
import sys
import tempfile

import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "beam.c")

MUTANTS = {
    "tie_key_reversed": ("return (a->key < b->key) ? -1 : (a->key > b->key);",
                         "return (a->key > b->key) ? -1 : (a->key < b->key);"),
    "repeat_without_blank": ("const float x = (c == last ? beam[i].pb : s) * yt[c];",
                             "const float x = s * yt[c];"),
    "stay_uses_blank_column": ("beam[j].pnb * yt[beam[j].tok[beam[j].len - 1]]",
                               "beam[j].pnb * yt[blank]"),
    "no_merge": ("if (is_extension(&beam[j], &beam[i], c)) { merged = j; break; }",
                 "if (0 && is_extension(&beam[j], &beam[i], c)) { merged = j; break; }"),
    "collapse_drops_whole_run": ("if (!(is_blank && prev_blank)) kept[n++] = t;",
                                 "if (!is_blank) kept[n++] = t;"),
    "collapse_not_strict": ("int is_blank = y[(int64_t)t * V + blank] > a;",
                            "int is_blank = y[(int64_t)t * V + blank] >= a;"),
    "scale_exponent_lost": ("        E += e;", "        E += 0;"),
    "blank_from_pb_only": ("q->pb = s * yt[blank];", "q->pb = beam[j].pb * yt[blank];"),
    "scale_off_by_one": ("next[r].pnb = scale_pow2(q->pnb, -e);",
                         "next[r].pnb = scale_pow2(q->pnb, 1 - e);"),
    "zero_totals_kept": ("if (cand[q].tot > 0.0f) cand[np++] = cand[q];",
                         "if (cand[q].tot >= 0.0f) cand[np++] = cand[q];"),
    "extension_label_wrong": ("if (ext) next[r].tok[h->len] = q->c;",
                              "if (ext) next[r].tok[h->len] = q->c > 1 ? q->c - 1 : q->c;"),
}

PINS = ["test_brute_force_full_beam", "test_ctc_loss_library_routine", "test_one_hot_frames",
        "test_exact_ties_follow_the_key", "test_repeated_label_needs_a_blank",
        "test_blank_collapse_rule", "test_blank_run_still_separates_repeats"]


def _run_pins(name):
    """Exit status 0 when the mutant passes every pin, 1 when one fails."""
    import oracle
    import test_beam_oracle as t
    find, repl = MUTANTS[name]
    with tempfile.TemporaryDirectory() as tmp:
        src = open(SRC).read()
        assert src.count(find) == 1, f"mutation {name}: pattern not found once"
        c = os.path.join(tmp, "beam.c")
        so = os.path.join(tmp, "libbeam.so")
        open(c, "w").write(src.replace(find, repl))
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-w",
                               "-ffp-contract=off", "-o", so, c, "-lpthread", "-lm"])
        lib = ctypes.CDLL(so)
        P, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
        lib.oracle_blank_collapse.argtypes = [P, i32, i32, i32, f32, P]
        lib.oracle_blank_collapse.restype = ctypes.c_int
        lib.oracle_beam_decode.argtypes = [P, i32, i32, i32, i32, f32, P, P, P, P, P]
        lib.oracle_beam_decode.restype = ctypes.c_int
        oracle._lib = lib          # the wrappers now call the mutant
        for pin in PINS:
            fn = getattr(t, pin)
            args = [[0], [1], [2], [3], [4], [5], [6], [7], [8], [9], [10], [11]] \
                if pin in ("test_brute_force_full_beam", "test_ctc_loss_library_routine") else [[]]
            for a in args:
                try:
                    fn(*a)
                except Exception:
                    return 1
    return 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_beam_pins_catch_mutant(name):
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys; sys.path[:0] = [%r, %r]; import test_beam_mutants as m; "
            "sys.exit(m._run_pins(%r))" % (here, os.path.dirname(here), name))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin\n{r.stderr[-2000:]}"
