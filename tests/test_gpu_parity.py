"""HIP path vs the CPU oracle, bit for bit (paths, per-frame scores, totals,
statuses), through the C-ABI library."""
import numpy as np
import pytest

import oracle
import pins
from gpu_util import compare_batched, compare_one, gpu_batched
from paper_2310_17864_amd import synth

pytestmark = pytest.mark.gpu


def test_tiny_brute_cases():
    errs = []
    for i, (E, y, blank) in enumerate(pins.tiny_cases(1, 120) + pins.tiny_cases(2, 60, neg_inf_p=0.3)):
        errs += compare_one(E, y, blank, f"tiny{i}")
    assert errs == []


def test_tie_and_zero_cases():
    errs = []
    for i, (E, y, blank) in enumerate(pins.tiny_cases(4, 80, integer=True) +
                                      pins.tiny_cases(5, 80, zeros=True) +
                                      pins.tiny_cases(3, 40, denormal=True)):
        errs += compare_one(E, y, blank, f"tie{i}")
    assert errs == []


def test_closed_form_shapes():
    errs = []
    rng = np.random.default_rng(7)
    for y in ([1, 2, 3], [1, 1, 2], [2, 2, 2], [], [3], [1, 2, 1, 2, 2]):
        R = sum(1 for j in range(1, len(y)) if y[j] == y[j - 1])
        for T in range(max(1, len(y) + R - 1), len(y) + R + 4):
            E = np.full((T, 5), -1.5, dtype=np.float32)
            errs += compare_one(E, np.array(y, np.int32), 0, f"uniform{y}T{T}")
            E = -np.abs(rng.standard_normal((T, 5))).astype(np.float32)
            errs += compare_one(E, np.array(y, np.int32), 0, f"rand{y}T{T}")
    for y in ([0], [5], [-1], [1, 0]):
        errs += compare_one(np.zeros((4, 5), np.float32), np.array(y, np.int32), 0, f"bad{y}")
    assert errs == []


@pytest.mark.parametrize("C,blank", [(32, 0), (256, 0), (32, 31), (5, 2), (29, 0), (100, 7),
                                     (256, 255), (1, 0), (2, 1)])
def test_class_counts_and_blank(C, blank):
    errs = []
    for seed in range(3):
        r = np.random.default_rng(1000 * C + seed)
        T = int(r.integers(1, 400))
        Lmax = max(0, min(T // 2, 300)) if C > 1 else 0
        L = int(r.integers(0, Lmax + 1)) if C > 1 else 0
        u = synth.utterance(r, max(T, 2 * L + 1), C, L, blank, 5.0, 1.0, 0.2 if C > 2 else None)
        errs += compare_one(u.emission, u.labels, blank, f"C{C}b{blank}s{seed}")
    assert errs == []


@pytest.mark.parametrize("L", [0, 1, 2, 31, 32, 63, 64, 100, 255, 256, 500, 1000, 2047, 2048, 3000,
                               5000, 8191, 12000])
def test_sizes_span_geometries(L):
    # S = 2L+1 crosses every single-launch geometry (W up to 16, M up to 32)
    r = np.random.default_rng(L)
    T = max(2 * L + 40, 50) if L < 3000 else 2 * L + 7
    u = synth.utterance(r, T, 32, L, 0, 6.0, 1.0, 0.1)
    assert compare_one(u.emission, u.labels, 0, f"L{L}") == []


def test_ragged_frame_counts():
    errs = []
    r = np.random.default_rng(5)
    for T in [1, 2, 3, 4, 5, 8, 9, 31, 32, 33, 34, 63, 64, 65, 97, 128, 129, 1000, 1025]:
        L = min(T // 3, 200)
        u = synth.utterance(r, T, 32, L, 0, 6.0, 1.0, 0.1)
        errs += compare_one(u.emission, u.labels, 0, f"T{T}")
        u = synth.utterance(r, T, 256, L, 0, 6.0, 1.0, None)
        errs += compare_one(u.emission, u.labels, 0, f"T{T}C256")
    assert errs == []


def test_single_utterance_config():
    u = synth.cfg_single().utts[0]
    assert compare_one(u.emission, u.labels, 0, "T200") == []


def test_plain_batch_config():
    errs = []
    for i, u in enumerate(synth.cfg_plain_batch().utts):
        errs += compare_one(u.emission, u.labels, 0, f"plain{i}")
    assert errs == []


def test_batched_small_vs_oracle():
    wl = synth.cfg_batched(n=96, t_hi=2500)
    pk = synth.pack(wl.utts)
    ref = oracle.align_batch_f32(pk, threads=8)
    assert compare_batched(pk, gpu_batched(pk), ref, "batched96") == []


def test_batched_with_invalid_and_infeasible_members():
    rng = np.random.default_rng(3)
    utts = [synth.utterance(rng, int(rng.integers(50, 600)), int(rng.choice([32, 256, 17])),
                            int(rng.integers(0, 20)), 0, 6.0, 1.0, None) for _ in range(24)]
    utts[3].labels[0] = 0                      # label == blank -> EINVAL
    utts[5] = synth.Utterance(np.zeros((4, 32), np.float32), np.array([1, 1, 1], np.int32), 0)
    pk = synth.pack(utts)
    ref = oracle.align_batch_f32(pk, threads=8)
    assert ref[0][3] == 1 and ref[0][5] == 2
    assert compare_batched(pk, gpu_batched(pk), ref, "mixed") == []


def test_batched_repeat_deterministic():
    wl = synth.cfg_batched(n=64, t_hi=1500, seed=11)
    pk = synth.pack(wl.utts)
    outs = gpu_batched(pk, runs=5)
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(np.asarray(a).view(np.uint32), np.asarray(b).view(np.uint32))


def test_batched_order_invariant():
    wl = synth.cfg_batched(n=48, t_hi=2000, seed=12)
    pk = synth.pack(wl.utts)
    st, paths, scores, totals = gpu_batched(pk)
    perm = np.random.default_rng(0).permutation(len(wl.utts))
    pk2 = synth.pack([wl.utts[i] for i in perm])
    st2, paths2, scores2, totals2 = gpu_batched(pk2)
    for j, i in enumerate(perm):
        a, b = pk["fr_off"][i], pk["fr_off"][i] + wl.utts[i].T
        c, d = pk2["fr_off"][j], pk2["fr_off"][j] + wl.utts[i].T
        assert np.array_equal(paths[a:b], paths2[c:d])
        assert np.array_equal(scores[a:b].view(np.uint32), scores2[c:d].view(np.uint32))
        assert totals[i].view(np.uint32) == totals2[j].view(np.uint32)
        assert st[i] == st2[j]


def test_batched_with_large_trellises():
    # S > 4096 runs on the second (large-trellis) persistent kernel next to the packs
    rng = np.random.default_rng(41)
    utts = [synth.utterance(rng, 2 * L + 30, C, L, 0, 6.0, 1.0, None)
            for L, C in [(2100, 32), (3000, 256), (5000, 32), (8000, 256), (12000, 32), (16383, 32)]]
    utts += [synth.utterance(rng, int(rng.integers(50, 900)), 32, int(rng.integers(5, 40)), 0, 6.0,
                             1.0, None) for _ in range(20)]
    pk = synth.pack(utts)
    ref = oracle.align_batch_f32(pk, threads=8)
    assert compare_batched(pk, gpu_batched(pk), ref, "large") == []


def test_token_spans_match_oracle():
    import paper_2310_17864_amd as ca
    from gpu_util import torch_dev
    torch, dev = torch_dev()
    for seed, (T, L, C) in enumerate([(200, 40, 32), (3000, 600, 256), (90, 0, 32), (5000, 900, 29)]):
        u = synth.utterance(np.random.default_rng(seed), T, C, L, 0, 6.0, 1.0, 0.2)
        path, scores, total, status = ca.align(torch.from_numpy(u.emission).to(dev),
                                               torch.from_numpy(u.labels).to(dev) if L else
                                               torch.empty(0, dtype=torch.int32, device=dev), 0)
        tok, st, en, sc = ca.token_spans(path, scores, 0)
        st_o, p_o, s_o, _ = oracle.align_f32(u.emission, u.labels, 0)
        rt, rs, re, rsc = oracle.token_spans(p_o, s_o, 0)
        assert np.array_equal(tok.cpu().numpy(), rt) and np.array_equal(tok.cpu().numpy(), u.labels)
        assert np.array_equal(st.cpu().numpy(), rs) and np.array_equal(en.cpu().numpy(), re)
        assert np.array_equal(sc.cpu().numpy().view(np.uint32), rsc.view(np.uint32))


@pytest.mark.parametrize("L,T", [(2049, 4200), (2500, 5100), (4096, 8300), (7000, 14100), (9000, 18100),
                                 (12288, 24700), (16383, 32800)])
def test_multi_workgroup_layouts(L, T):
    # S > 4096 spreads over ceil(W/8) workgroups (W = ceil(S/(64 M)), M = 8):
    # cross-workgroup boundaries, a top workgroup of one to eight waves
    r = np.random.default_rng(L)
    u = synth.utterance(r, T, 32 if L % 2 else 256, L, 0, 6.0, 1.0, 0.1)
    assert compare_one(u.emission, u.labels, 0, f"multiL{L}") == []


def test_multi_workgroup_repeated_launches():
    # back-to-back asynchronous launches of multi-workgroup alignments of
    # different sizes on one stream, interleaved with a batched plan: every
    # run completes (no bounded wait runs out) and equals the oracle.  (The
    # cross-workgroup slots were once read through a stale cache line left by
    # the reset of an earlier launch.)
    import paper_2310_17864_amd as ca
    from gpu_util import torch_dev
    torch, dev = torch_dev()
    cases = []
    for seed, (L, T) in enumerate([(2500, 5100), (7000, 14100), (15000, 30200)]):
        u = synth.utterance(np.random.default_rng(100 + seed), T, 32, L, 0, 6.0, 1.0, 0.1)
        st, p, s, t = oracle.align_f32(u.emission, u.labels, 0)
        cases.append((torch.from_numpy(u.emission).to(dev), torch.from_numpy(u.labels).to(dev), st, p, s))
    wl = synth.cfg_batched(n=32, t_hi=1500, seed=9)
    pk = synth.pack(wl.utts)
    plan = ca.Plan(torch.from_numpy(pk["em"]).to(dev), pk["em_off"], pk["T"], pk["C"],
                   torch.from_numpy(pk["lab"]).to(dev), pk["lab_off"], pk["L"], pk["fr_off"], 0)
    outs = []
    for rep in range(3):
        for e, y, _, _, _ in cases:
            outs.append(ca.align(e, y, 0, sync=False))
        plan.run()
    torch.cuda.synchronize()
    for k, (path, scores, total, status) in enumerate(outs):
        _, _, st, p, s = cases[k % len(cases)]
        assert int(status.item()) == st == 0, k
        assert np.array_equal(path.cpu().numpy(), p), k
        assert np.array_equal(scores.cpu().numpy().view(np.uint32), s.view(np.uint32)), k
    plan.close()


@pytest.mark.slow
def test_long_form_full_size():
    # the long-form workload as configured: T = 90,000 frames, C = 32,
    # L = 15,000 (S = 30,001; 675 MB of 2-bit backpointers), one launch over
    # several workgroups; paths, scores and total bitwise equal to the float32
    # oracle, and the float32 total within 1e-3 relative of the float64 one
    u = synth.cfg_long().utts[0]
    assert (u.T, u.C, u.L) == (90_000, 32, 15_000)
    assert compare_one(u.emission, u.labels, 0, "long90000") == []
    st32, _, _, t32 = oracle.align_f32(u.emission, u.labels, 0)
    st64, _, _, t64 = oracle.align_f64(u.emission, u.labels, 0)
    assert st32 == st64 == 0
    assert abs(float(t32) - float(t64)) <= 1e-3 * abs(float(t64))
