"""Geometry invariance: every (waves, states-per-lane) layout the kernels
compile gives the same bits (checked against the oracle), for single
launches and for the batched persistent kernel."""
import numpy as np
import pytest

import oracle
from gpu_util import compare_batched, compare_one, gpu_batched
from paper_2310_17864_amd import synth

pytestmark = pytest.mark.gpu

ONE = [(W, M) for W in (1, 2, 3, 4) for M in (2, 4, 6, 8, 10, 12, 14, 16)] + \
      [(W, M) for W in range(1, 9) for M in (16, 24, 32, 40, 48, 56, 60, 64)]
PACK = [(W, M) for W in (1, 2, 4) for M in (2, 4, 6, 8, 12, 16)]


def holds(S, W, M):
    seg = 64 * M
    return W * seg >= S and (W == 1 or (W - 1) * seg + 2 <= S)


@pytest.mark.parametrize("L,C", [(3, 32), (40, 32), (100, 256), (300, 32), (700, 256), (1500, 32),
                                 (2100, 7)])
def test_single_launch_geometries(L, C):
    import paper_2310_17864_amd as ca
    ctx = ca.context(0)
    S = 2 * L + 1
    r = np.random.default_rng(L)
    u = synth.utterance(r, 2 * L + 60, C, L, 0, 6.0, 1.0, 0.1)
    errs, tried = [], 0
    for W, M in ONE:
        if not holds(S, W, M):
            continue
        ctx.tune_set(0, S, S, C, W, M)
        try:
            errs += compare_one(u.emission, u.labels, 0, f"S{S} W{W} M{M}")
            tried += 1
        finally:
            ctx.tune_clear(0, S, S, C)
    assert tried >= 2
    assert errs == []


def test_pack_geometries():
    import paper_2310_17864_amd as ca
    ctx = ca.context(0)
    wl = synth.cfg_batched(n=16, t_hi=900, seed=31)
    pk = synth.pack(wl.utts)
    ref = oracle.align_batch_f32(pk, threads=8)
    for W, M in PACK:
        Ss = [2 * u.L + 1 for u in wl.utts]
        if not all(holds(S, W, M) for S in Ss):
            continue
        for u, S in zip(wl.utts, Ss):
            ctx.tune_set(1, S, S, u.C, W, M)
        try:
            assert compare_batched(pk, gpu_batched(pk), ref, f"pack W{W} M{M}") == []
        finally:
            for u, S in zip(wl.utts, Ss):
                ctx.tune_clear(1, S, S, u.C)


def test_table_roundtrip(tmp_path):
    import paper_2310_17864_amd as ca
    ctx = ca.context(0)
    ctx.tune_set(0, 320, 511, 32, 2, 4)          # 2 waves x 256 states hold 258..512
    assert ctx.tune_get(0, 400, 32) == (2, 4)
    p = str(tmp_path / "tune.txt")
    ctx.tune_save(p)
    ctx.tune_clear(0, 320, 511, 32)
    ctx.tune_load(p)
    assert ctx.tune_get(0, 400, 32) == (2, 4)
    ctx.tune_clear(0, 320, 511, 32)
    with pytest.raises(ca.CtcAlignError):
        ctx.tune_set(0, 100, 300, 32, 1, 2)      # 128 states cannot hold S=300
    with pytest.raises(ca.CtcAlignError):
        ctx.tune_set(0, 100, 300, 32, 2, 4)      # the top wave would not hold S-2 for S < 258


def test_chooser_returns_a_layout_for_every_size():
    import paper_2310_17864_amd as ca
    ctx = ca.context(0)
    for C in (32, 256):
        for S in range(1, 4097, 2):
            W, M = ctx.tune_get(1, S, C)
            assert W in (1, 2, 4) and holds(S, W, M), (S, W, M)
        for S in list(range(1, 32768, 37)) + [32767]:
            W, M = ctx.tune_get(0, S, C)
            assert W >= 1 and holds(S, W, M), (S, W, M)


def test_batched_sizes_span_every_pack_layout():
    # L from 0 to 2047: S = 2L+1 covers every batched layout
    rng = np.random.default_rng(77)
    utts = []
    for L in list(range(0, 2048, 23)) + [1024, 1025, 1100, 1152, 1153, 1280, 2047]:
        C = 32 if L % 2 else 256
        utts.append(synth.utterance(rng, 2 * L + 5, C, L, 0, 6.0, 1.0, None))
    pk = synth.pack(utts)
    ref = oracle.align_batch_f32(pk, threads=8)
    assert compare_batched(pk, gpu_batched(pk), ref, "span") == []
