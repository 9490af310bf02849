"""CTC prefix beam search with blank collapse on the GPU (ctcalign_beam_decode)
against the CPU oracle (oracle/beam.c): the final beam of every utterance --
its labels, their count, the exact scaled total and power-of-two exponent of
every hypothesis, the kept-frame count and the status -- bit for bit; the
log-probabilities within float32 rounding of the double-precision log.
Covers tiny exhaustive cases, exact ties, one-hot frames, every beam width up
to 16, class counts up to 1024 (each side of every 64-class column
boundary the kernel is instantiated for), a non-zero blank, collapse thresholds from
none to aggressive, flat rows that overflow the candidate list, long inputs,
failures (no positive candidate), and the decoding workload's shapes."""
import numpy as np
import pytest

import oracle
from beam_brute import random_probs
from gpu_util import torch_dev
from paper_2310_17864_amd import synth

pytestmark = pytest.mark.gpu


def _pack(ys):
    V = ys[0].shape[1]
    off = np.zeros(len(ys), np.int64)
    tot = 0
    for i, y in enumerate(ys):
        off[i] = tot
        tot += (y.size + 63) // 64 * 64
    flat = np.zeros(max(tot, 1), np.float32)
    for i, y in enumerate(ys):
        flat[off[i]:off[i] + y.size] = y.reshape(-1)
    return {"y": flat, "y_off": off, "T": np.array([y.shape[0] for y in ys], np.int32), "V": V}


def _compare(pk, blank, beam, a, label=""):
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    probs = torch.from_numpy(pk["y"]).to(dev)
    res = ca.beam_decode(probs, pk["y_off"], pk["T"], blank, beam, a, V=pk["V"])
    torch.cuda.synchronize()
    st, hyps, logps, nkept, _, scaled, exps = oracle.beam_decode_batch(pk, blank, beam, a, threads=8,
                                                                        raw=True)
    g_st = res.status.cpu().numpy()
    g_nk = res.nkept.cpu().numpy()
    g_nh = res.nhyp.cpu().numpy()
    g_sc = res.scaled.cpu().numpy()
    g_ex = res.exp2.cpu().numpy()
    errs = []
    for i in range(len(pk["T"])):
        if g_st[i] != st[i] or g_nk[i] != nkept[i]:
            errs.append(f"{label}#{i}: status {g_st[i]}/{st[i]} kept {g_nk[i]}/{nkept[i]}")
            continue
        if g_nh[i] != len(hyps[i]):
            errs.append(f"{label}#{i}: {g_nh[i]} hypotheses vs {len(hyps[i])}")
            continue
        if st[i] != 0:
            continue
        gh, glp = res.hypotheses(i)
        for k, (h, lp) in enumerate(zip(hyps[i], logps[i])):
            if not np.array_equal(gh[k], h):
                errs.append(f"{label}#{i} hyp {k}: labels differ")
                break
            if g_sc[i * beam + k].view(np.uint32) != scaled[i][k].view(np.uint32):
                errs.append(f"{label}#{i} hyp {k}: scaled total {g_sc[i * beam + k]!r} vs {scaled[i][k]!r}")
                break
            if abs(float(glp[k]) - lp) > 2e-7 * max(1.0, abs(lp)):
                errs.append(f"{label}#{i} hyp {k}: logp {glp[k]} vs {lp}")
                break
        if g_ex[i] != exps[i]:
            errs.append(f"{label}#{i}: exponent {g_ex[i]} vs {exps[i]}")
    return errs


def test_tiny_random_cases():
    rng = np.random.default_rng(0)
    errs = []
    for rep in range(4):
        ys = [random_probs(rng, int(rng.integers(1, 7)), int(rng.integers(2, 5)), conc=0.7)
              for _ in range(24)]
        V = max(y.shape[1] for y in ys)
        ys = [y for y in ys if y.shape[1] == V] or ys[:1]
        errs += _compare(_pack(ys), rep % V, 16, 1.0, f"tiny{rep}")
    assert errs == []


@pytest.mark.parametrize("beam", [1, 2, 3, 5, 8, 10, 16])
def test_beam_widths(beam):
    rng = np.random.default_rng(beam)
    ys = [random_probs(rng, int(rng.integers(5, 120)), 29, conc=0.3) for _ in range(16)]
    assert _compare(_pack(ys), 0, beam, 1.0, f"B{beam}") == []


@pytest.mark.parametrize("V,blank", [(2, 0), (2, 1), (31, 30), (64, 63), (65, 64), (100, 3), (128, 0), (129, 128),
                                     (256, 0), (257, 1), (500, 0), (512, 511), (513, 0), (1000, 7), (1024, 1023)])
def test_class_counts(V, blank):
    rng = np.random.default_rng(V)
    ys = [random_probs(rng, int(rng.integers(3, 80)), V, conc=0.05) for _ in range(8)]
    assert _compare(_pack(ys), blank, 10, 1.0, f"V{V}") == []


def test_exact_ties_and_one_hot():
    ys = [np.array([[0.25, 0.375, 0.375]], np.float32),
          np.array([[0.5, 0.5, 0.0]], np.float32),
          np.array([[0.0, 0.5, 0.5]], np.float32),
          np.full((7, 3), 0.25, np.float32) * np.array([2, 1, 1], np.float32),
          np.full((9, 3), 1.0 / 3.0, np.float32)]
    errs = []
    for blank in (0, 2):
        for beam in (1, 2, 4):
            errs += _compare(_pack(ys[:3]), blank, beam, 1.0, f"tie b{blank} B{beam}")
    errs += _compare(_pack(ys[3:]), 0, 6, 1.0, "flat")
    cls = [3, 3, 0, 3, 5, 5, 0, 0, 1, 2, 2]
    y = np.zeros((len(cls), 6), np.float32)
    y[np.arange(len(cls)), cls] = 1.0
    errs += _compare(_pack([y]), 0, 10, 1.0, "onehot")
    assert errs == []


@pytest.mark.parametrize("a", [1.0, 0.99, 0.95, 0.8, 0.5, 0.0])
def test_blank_collapse_thresholds(a):
    pk = synth.decode_packed(n=24, t_hi=400, seed=31, workers=1)
    assert _compare(pk, 0, 10, a, f"a{a}") == []


def test_flat_rows_overflow_the_list():
    # near-uniform rows: most candidates tie at the bound and the list
    # overflows, so the fallback selection runs
    rng = np.random.default_rng(9)
    ys = [np.full((30, 600), 1.0 / 600, np.float32)]
    ys.append((np.full((25, 600), 1.0, np.float32) + rng.random((25, 600)).astype(np.float32) * 1e-3))
    ys[1] = (ys[1] / ys[1].sum(axis=1, keepdims=True)).astype(np.float32)
    assert _compare(_pack(ys), 0, 16, 1.0, "flat600") == []


def test_long_inputs_and_failures():
    rng = np.random.default_rng(21)
    ys = [random_probs(rng, 1500, 8, conc=1.5), random_probs(rng, 700, 40, conc=0.2)]
    z = random_probs(rng, 50, 5)
    z[20] = 0.0                    # every candidate of frame 20 has total 0
    ys2 = [z, random_probs(rng, 30, 5)]
    errs = _compare(_pack(ys), 0, 10, 1.0, "long")
    errs += _compare(_pack(ys2), 0, 4, 1.0, "fail")
    assert errs == []


def test_decoding_workload_sample():
    pk = synth.decode_packed(n=64, seed=6, workers=1)
    errs = _compare(pk, 0, 10, 0.95, "dec095")
    errs += _compare(pk, 0, 10, 1.0, "dec100")
    assert errs == []
