"""The CPU oracle pinned to brute force, closed forms, invariants, a second
precision and an independent library routine (all CPU-only)."""
import math

import numpy as np
import pytest

import oracle
import pins
from invariants import check_alignment
from paper_2310_17864_amd import synth


def test_brute_force_random_float():
    assert pins.check_brute(oracle.align_f32, pins.tiny_cases(1, 250)) == []


def test_brute_force_with_neg_inf():
    assert pins.check_brute(oracle.align_f32, pins.tiny_cases(2, 150, neg_inf_p=0.3)) == []


def test_brute_force_denormals():
    assert pins.check_brute(oracle.align_f32, pins.tiny_cases(3, 120, denormal=True)) == []


def test_tie_rule_integer_emissions():
    assert pins.check_tie_rule(oracle.align_f32, pins.tiny_cases(4, 250, integer=True)) == []


def test_tie_rule_signed_zeros():
    assert pins.check_tie_rule(oracle.align_f32, pins.tiny_cases(5, 200, zeros=True)) == []


def test_closed_forms():
    assert pins.check_closed_forms(oracle.align_f32) == []


def test_f64_variant_matches_brute_max():
    # the double variant's total equals the exact maximum over alignments
    # (small integer emissions: every sum is exact in double)
    for E, y, blank in pins.tiny_cases(6, 120, integer=True):
        st, path, scores, total = oracle.align_f64(E, y, blank)
        pis, sc = pins.brute.brute(E, y, blank)
        best = float(sc.max()) if len(sc) else -np.inf
        assert (st == 2) == (best == -np.inf)
        if st == 0:
            assert total == best


@pytest.mark.parametrize("make", [
    lambda: synth.cfg_single(),
    lambda: synth.cfg_plain_batch(n=6),
    lambda: synth.cfg_long(T=3000, L=500),
    lambda: synth.cfg_batched(n=12, t_hi=1500),
    lambda: synth.cfg_serving(pool=6, t_hi=3000),
], ids=["single", "plain", "long", "batched", "serving"])
def test_invariants_on_workloads(make):
    wl = make()
    for u in wl.utts:
        st, path, scores, total = oracle.align_f32(u.emission, u.labels, u.blank)
        assert st == 0
        assert check_alignment(u.emission, u.labels, u.blank, path, scores, total) == []
        # the planted path is feasible, so the optimum is at least its score
        planted_lab = np.where(u.planted % 2 == 0, u.blank,
                               u.labels[np.maximum(u.planted - 1, 0) // 2] if u.L else u.blank)
        planted_score = pins.fold32(u.emission[np.arange(u.T), planted_lab])
        assert total >= planted_score


@pytest.mark.parametrize("T,L,tol", [(1500, 300, 1e-4), (10_000, 1700, 1e-4),
                                     (20_000, 3300, 1e-3)])
def test_f32_vs_f64_total(T, L, tol):
    u = synth.utterance(np.random.default_rng(T), T, 32, L, 0, 4.0, 1.5, 0.1)
    st32, _, _, t32 = oracle.align_f32(u.emission, u.labels, 0)
    st64, _, _, t64 = oracle.align_f64(u.emission, u.labels, 0)
    assert st32 == st64 == 0
    assert abs(float(t32) - float(t64)) <= tol * abs(float(t64))


def test_ctc_loss_does_not_renormalise():
    # T=1, L=1: -ctc_loss equals the single log-probability it is given
    import torch
    lp = torch.tensor([[[-0.3, -5.0, 2.0]]], dtype=torch.float64)
    loss = torch.nn.functional.ctc_loss(lp, torch.tensor([[2]]), torch.tensor([1]),
                                        torch.tensor([1]), blank=0, reduction="sum")
    assert float(loss) == pytest.approx(-2.0, abs=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_ctc_loss_beta_limit(seed):
    r = np.random.default_rng(seed)
    T = int(r.integers(20, 120))
    L = int(r.integers(1, T // 3))
    C = int(r.integers(3, 40))
    blank = int(r.integers(0, C))
    u = synth.utterance(r, T, C, L, blank, 3.0, 1.0, 0.2)
    st, _, _, t64 = oracle.align_f64(u.emission, u.labels, blank)
    assert st == 0
    assert pins.ctc_loss_limit(u.emission, u.labels, blank, float(t64)) == []


def test_batch_entry_matches_single():
    wl = synth.cfg_batched(n=16, t_hi=800)
    pk = synth.pack(wl.utts)
    status, paths, scores, totals, used = oracle.align_batch_f32(pk, threads=4)
    assert used >= 1
    for i, u in enumerate(wl.utts):
        st, p, s, t = oracle.align_f32(u.emission, u.labels, 0)
        a, b = pk["fr_off"][i], pk["fr_off"][i] + u.T
        assert status[i] == st
        assert np.array_equal(paths[a:b], p)
        assert np.array_equal(scores[a:b].view(np.uint32), s.view(np.uint32))
        assert totals[i].view(np.uint32) == t.view(np.uint32)


def test_token_spans_closed_forms():
    # hand-checkable path: blanks around, a repeated label split by a blank
    path = np.array([0, 3, 3, 0, 0, 3, 5, 5, 5, 0], np.int32)
    scores = np.array([-1, -0.5, -0.25, -1, -1, -2, -1, -1, -0.5, -3], np.float32)
    tok, st, en, sc = oracle.token_spans(path, scores, 0)
    assert tok.tolist() == [3, 3, 5]
    assert st.tolist() == [1, 5, 6] and en.tolist() == [3, 6, 9]
    assert sc.tolist() == [-0.75, -2.0, -2.5]
    # no tokens
    tok, st, en, sc = oracle.token_spans(np.zeros(7, np.int32), np.zeros(7, np.float32), 0)
    assert len(tok) == 0


def test_token_spans_on_alignments():
    # one span per transcript token, in order, covering exactly the non-blank
    # frames; with integer scores the span sums and the blank frames add up
    # exactly to the alignment total
    for seed in range(5):
        r = np.random.default_rng(seed)
        T, C, L = int(r.integers(30, 400)), 12, int(r.integers(1, 10))
        u = synth.utterance(r, max(T, 2 * L + 2), C, L, 0, 4.0, 1.0, 0.3)
        E = np.round(u.emission * 4).astype(np.float32) / 4      # exact sums
        st, path, scores, total = oracle.align_f32(E, u.labels, 0)
        tok, s0, s1, sc = oracle.token_spans(path, scores, 0)
        assert np.array_equal(tok, u.labels)
        assert np.all(s0[1:] >= s1[:-1]) and np.all(s1 > s0)
        covered = np.zeros(len(path), bool)
        for a, b in zip(s0, s1):
            covered[a:b] = True
        assert np.array_equal(covered, path != 0)
        assert float(np.sum(sc)) + float(np.sum(scores[path == 0])) == float(total)
