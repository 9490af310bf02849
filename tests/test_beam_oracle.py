"""Pins of the CPU oracle for CTC prefix beam search with blank collapse
(oracle/beam.c), none of which re-types its recursion:

* brute force: with a beam wide enough to keep every prefix and no
  collapse, the final beam holds every label sequence with positive
  probability, ranked by it, with log-probabilities equal to the float64 sum
  over all frame labellings that collapse to the sequence;
* an independent library routine: exp(-torch ctc_loss) of each final
  hypothesis in float64;
* closed forms: one-hot frames decode to the collapse of their classes with
  log-probability 0; exact ties follow the key rule (stay before extension of
  the same hypothesis when the blank is the smaller class, smaller class
  first);
* blank collapse: threshold 1 keeps every frame, a run of blank frames
  keeps exactly its first frame (so a blank still separates repeated labels),
  and decoding with a threshold equals decoding the kept frames alone;
* the running power-of-two scale: long inputs stay finite and match the
  library routine.
"""
import numpy as np
import pytest
import torch

import oracle
from beam_brute import random_probs, sequence_probs


def _ctc_logp(y: np.ndarray, labels, blank: int) -> float:
    lp = torch.from_numpy(np.log(y.astype(np.float64))).unsqueeze(1)   # [T, 1, V]
    tgt = torch.tensor([list(labels)], dtype=torch.long)
    if len(labels) == 0:
        tgt = torch.zeros((1, 1), dtype=torch.long)
    loss = torch.nn.functional.ctc_loss(lp, tgt, torch.tensor([y.shape[0]]),
                                        torch.tensor([len(labels)]), blank=blank,
                                        reduction="sum", zero_infinity=False)
    return -float(loss)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_full_beam(seed):
    rng = np.random.default_rng(seed)
    T = int(rng.integers(1, 6))
    V = int(rng.integers(2, 4))
    blank = int(rng.integers(0, V))
    y = random_probs(rng, T, V, conc=0.8)
    ref = sequence_probs(y, blank)
    st, hyps, logp, nk = oracle.beam_decode(y, blank, beam=256, a=1.0)
    assert st == 0 and nk == T
    got = {tuple(int(x) for x in h): lp for h, lp in zip(hyps, logp)}
    assert set(got) == set(ref), (sorted(got), sorted(ref))
    for k, p in ref.items():
        assert abs(got[k] - np.log(p)) <= 2e-6 * max(1.0, abs(np.log(p))), (k, got[k], np.log(p))
    # ranked by probability
    order = [tuple(int(x) for x in h) for h in hyps]
    probs = [ref[k] for k in order]
    assert all(probs[i] >= probs[i + 1] * (1 - 1e-5) for i in range(len(probs) - 1))


@pytest.mark.parametrize("seed", range(6))
def test_ctc_loss_library_routine(seed):
    rng = np.random.default_rng(100 + seed)
    T, V = 7, 3
    blank = seed % V
    y = random_probs(rng, T, V, conc=0.6)
    st, hyps, logp, _ = oracle.beam_decode(y, blank, beam=1024, a=1.0)
    assert st == 0
    for h, lp in zip(hyps[:20], logp[:20]):
        ref = _ctc_logp(y, [int(x) for x in h], blank)
        assert abs(lp - ref) <= 2e-6 * max(1.0, abs(ref)), (h, lp, ref)


def test_one_hot_frames():
    V, blank = 6, 0
    cls = [3, 3, 0, 3, 5, 5, 0, 0, 1, 2, 2]
    y = np.zeros((len(cls), V), np.float32)
    y[np.arange(len(cls)), cls] = 1.0
    st, hyps, logp, _ = oracle.beam_decode(y, blank, beam=10, a=1.0)
    assert st == 0 and len(hyps) == 1
    assert hyps[0].tolist() == [3, 3, 5, 1, 2]
    assert abs(logp[0]) < 1e-12


def test_exact_ties_follow_the_key():
    # one frame, classes 0 (blank), 1, 2: extensions 1 and 2 tie
    y = np.array([[0.25, 0.375, 0.375]], np.float32)
    st, hyps, logp, _ = oracle.beam_decode(y, 0, beam=3, a=1.0)
    assert [h.tolist() for h in hyps] == [[1], [2], []]
    assert oracle.beam_decode(y, 0, beam=1)[1][0].tolist() == [1]
    # the empty prefix's stay (key = blank) against the extension by 1 (key 1)
    y = np.array([[0.5, 0.5, 0.0]], np.float32)
    assert [h.tolist() for h in oracle.beam_decode(y, 0, beam=2)[1]] == [[], [1]]
    y = np.array([[0.0, 0.5, 0.5]], np.float32)        # blank = 2: extension 1 first
    assert [h.tolist() for h in oracle.beam_decode(y, 2, beam=2)[1]] == [[1], []]


def test_repeated_label_needs_a_blank():
    # two frames of 'a' (0.5) / blank (0.5): "aa" needs three frames
    y = np.full((2, 2), 0.5, np.float32)
    st, hyps, logp, _ = oracle.beam_decode(y, 0, beam=8, a=1.0)
    got = {tuple(h.tolist()): lp for h, lp in zip(hyps, logp)}
    assert set(got) == {(1,), ()}
    assert abs(got[(1,)] - np.log(0.75)) < 1e-7 and abs(got[()] - np.log(0.25)) < 1e-7


def test_blank_collapse_rule():
    rng = np.random.default_rng(4)
    y = random_probs(rng, 40, 5)
    assert oracle.blank_collapse(y, 0, 1.0).tolist() == list(range(40))
    # the threshold is strict: a blank probability equal to it is no blank
    # frame, so a = 1 keeps even certain blank frames
    ones = np.zeros((6, 3), np.float32)
    ones[:, 0] = 1.0
    assert oracle.blank_collapse(ones, 0, 1.0).tolist() == list(range(6))
    half = np.full((4, 2), 0.5, np.float32)
    assert oracle.blank_collapse(half, 0, 0.5).tolist() == [0, 1, 2, 3]
    assert oracle.blank_collapse(half, 0, 0.49).tolist() == [0]
    # make frames blank frames in runs, count what survives
    mask = rng.random(40) < 0.6
    z = y.copy()
    z[mask] = 0.0025
    z[mask, 2] = 0.99
    kept = oracle.blank_collapse(z, 2, 0.95)
    runs = 0
    for t in range(40):
        if mask[t] and (t == 0 or not mask[t - 1]):
            runs += 1
    assert len(kept) == int((~mask).sum()) + runs
    assert set(np.nonzero(~mask)[0].tolist()) <= set(kept.tolist())
    for t in kept:
        if mask[t]:
            assert t == 0 or not mask[t - 1]


def test_blank_run_still_separates_repeats():
    # 'a', three confident blank frames, 'a' -> two labels survive
    y = np.array([[0.01, 0.99], [0.99, 0.01], [0.99, 0.01], [0.99, 0.01], [0.01, 0.99]], np.float32)
    kept = oracle.blank_collapse(y, 0, 0.95)
    assert kept.tolist() == [0, 1, 4]
    st, hyps, _, nk = oracle.beam_decode(y, 0, beam=4, a=0.95)
    assert st == 0 and nk == 3 and hyps[0].tolist() == [1, 1]


def test_decoding_with_threshold_is_decoding_the_kept_frames():
    rng = np.random.default_rng(8)
    for _ in range(5):
        T, V = 30, 6
        y = random_probs(rng, T, V, conc=0.3)
        blanky = rng.random(T) < 0.5
        y[blanky] *= 0.02
        y[blanky, 0] = 0.98
        a = 0.9
        kept = oracle.blank_collapse(y, 0, a)
        r1 = oracle.beam_decode(y, 0, beam=5, a=a)
        r2 = oracle.beam_decode(y[kept], 0, beam=5, a=1.0)
        assert r1[3] == len(kept)
        assert [h.tolist() for h in r1[1]] == [h.tolist() for h in r2[1]]
        assert np.array_equal(r1[2], r2[2])


def test_long_input_scale_stays_exact():
    # 400 frames: the raw probabilities would underflow float32 many times
    rng = np.random.default_rng(12)
    y = random_probs(rng, 400, 4, conc=2.0)
    st, hyps, logp, _ = oracle.beam_decode(y, 0, beam=16, a=1.0)
    assert st == 0 and np.all(np.isfinite(logp))
    assert logp[0] < -100
    ref = _ctc_logp(y, hyps[0].tolist(), 0)
    # the beam keeps a subset of each hypothesis's paths: a lower bound, and
    # tight for the best one on such a peaked input
    assert logp[0] <= ref + 1e-6 * abs(ref)


def test_batch_equals_single():
    rng = np.random.default_rng(3)
    ys = [random_probs(rng, int(rng.integers(1, 60)), 7, conc=0.4) for _ in range(9)]
    off = np.concatenate([[0], np.cumsum([y.size for y in ys])[:-1]]).astype(np.int64)
    pk = {"y": np.concatenate([y.reshape(-1) for y in ys]), "y_off": off,
          "T": np.array([y.shape[0] for y in ys], np.int32), "V": 7}
    st, hyps, logps, nk, _ = oracle.beam_decode_batch(pk, 0, 4, 0.9, threads=3)
    for i, y in enumerate(ys):
        s1, h1, l1, k1 = oracle.beam_decode(y, 0, 4, 0.9)
        assert st[i] == s1 and nk[i] == k1
        assert [h.tolist() for h in hyps[i]] == [h.tolist() for h in h1]
        assert np.array_equal(logps[i], l1)
