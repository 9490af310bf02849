"""The continuous-batching server on the GPU: every request's result is
bit-identical to the CPU oracle whether it runs alone or mixed with others,
under a large and a tiny backpointer budget, and oversize requests are
refused."""
import time

import numpy as np
import pytest

import oracle
from gpu_util import same_bits, torch_dev
from paper_2310_17864_amd import synth

pytestmark = pytest.mark.gpu


def _pool():
    wl = synth.cfg_serving(pool=40, t_hi=14000, seed=21)
    utts = list(wl.utts)
    rng = np.random.default_rng(9)
    utts.append(synth.utterance(rng, 300, 17, 40, 0, 6.0, 1.0, None))      # padded class count
    utts.append(synth.utterance(rng, 500, 100, 90, 3, 6.0, 1.0, None))     # padded, blank 3
    bad = synth.utterance(rng, 200, 32, 30, 0, 6.0, 1.0, None)
    bad.labels[5] = 0                                                      # label == blank
    utts.append(bad)
    utts.append(synth.Utterance(np.zeros((3, 32), np.float32), np.array([4, 4], np.int32), 0))
    return utts


def _upload(utts):
    torch, dev = torch_dev()
    out = []
    for u in utts:
        out.append(dict(em=torch.from_numpy(u.emission).to(dev),
                        lab=torch.from_numpy(u.labels).to(dev) if u.L else
                        torch.empty(0, dtype=torch.int32, device=dev),
                        path=torch.full((u.T,), -7, dtype=torch.int32, device=dev),
                        sc=torch.empty(u.T, dtype=torch.float32, device=dev),
                        tot=torch.empty(1, dtype=torch.float32, device=dev)))
    torch.cuda.synchronize()
    return out


def _check(utts, bufs, results):
    errs = []
    for i, (u, b, (st, tm)) in enumerate(zip(utts, bufs, results)):
        st_o, p_o, s_o, t_o = oracle.align_f32(u.emission, u.labels, u.blank)
        if st != st_o:
            errs.append(f"req {i}: status {st} vs oracle {st_o}")
            continue
        if not same_bits(b["path"].cpu().numpy(), p_o) or not same_bits(b["sc"].cpu().numpy(), s_o):
            errs.append(f"req {i}: path/scores differ (T={u.T} L={u.L} C={u.C})")
        if st_o in (0, 2) and np.float32(b["tot"].cpu().numpy()[0]).view(np.uint32) != \
                np.float32(t_o).view(np.uint32):
            errs.append(f"req {i}: total differs")
        if not (tm[0] <= tm[1] <= tm[2] <= tm[3]):
            errs.append(f"req {i}: timestamps out of order {tm}")
    return errs


def _serve(utts, bufs, budget, stagger=False):
    import paper_2310_17864_amd as ca
    srv = ca.Server(budget)
    tickets = []
    for i, (u, b) in enumerate(zip(utts, bufs)):
        tickets.append(srv.submit(b["em"], b["lab"], b["path"], b["sc"], b["tot"], u.blank))
        if stagger and i % 5 == 4:
            time.sleep(0.002)     # later arrivals join while earlier ones run
    res = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    return res, stats


def test_server_mixed_matches_oracle():
    utts = _pool()
    bufs = _upload(utts)
    res, stats = _serve(utts, bufs, 64 << 30, stagger=True)
    assert _check(utts, bufs, res) == []
    assert stats["budget_violated"] == 0 and stats["completed"] == len(utts)


def test_server_tiny_budget_serialises_but_matches():
    utts = _pool()
    bufs = _upload(utts)
    charges = [u.T * (2 * u.L + 1) // 4 + 1 for u in utts]
    budget = int(2.2 * max(charges))           # at most ~2 big requests at once
    res, stats = _serve(utts, bufs, budget)
    assert _check(utts, bufs, res) == []
    assert stats["peak_charge_bytes"] <= budget
    assert stats["budget_violated"] == 0


def test_server_alone_equals_mixed():
    import paper_2310_17864_amd as ca
    torch, _ = torch_dev()
    utts = _pool()[:12]
    bufs = _upload(utts)
    _serve(utts, bufs, 64 << 30)
    mixed = [(b["path"].cpu().numpy().copy(), b["sc"].cpu().numpy().copy()) for b in bufs]
    srv = ca.Server(64 << 30)
    for u, b, (p, s) in zip(utts, bufs, mixed):
        b["path"].fill_(-7)
        torch.cuda.synchronize()          # requests must not race the caller's own writes
        t = srv.submit(b["em"], b["lab"], b["path"], b["sc"], b["tot"], u.blank)
        srv.wait(t)
        assert np.array_equal(b["path"].cpu().numpy(), p)
        assert np.array_equal(b["sc"].cpu().numpy().view(np.uint32), s.view(np.uint32))
    srv.close()


def test_server_refuses_oversize():
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    u = synth.utterance(np.random.default_rng(1), 4000, 32, 800, 0, 6.0, 1.0, None)
    b = _upload([u])[0]
    srv = ca.Server(1 << 16)
    with pytest.raises(ca.CtcAlignError) as ei:
        srv.submit(b["em"], b["lab"], b["path"], b["sc"], b["tot"])
    assert ei.value.code == ca.ENOMEM
    srv.close()


def test_server_top_segment_single_state():
    # trellis sizes S = 64*M*k + 1: the served layout's top wave holds S-1
    # alone and takes a(S-2) from the boundary ring of the wave below; paths
    # ending in S-2 and in S-1, a one-frame request, and the two sizes
    # (S = 14337, 15361) no layout with two states on top covers
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    utts = []
    for T, L in ((12000, 2304), (30000, 7168), (30000, 7680)):
        ends = set()
        for seed in range(40):
            u = synth.utterance(np.random.default_rng(seed), T, 32, L, 0, 6.0, 1.0, None)
            end = int(u.planted[-1]) == 2 * L     # planted path ends in S-1 (blank)
            if end not in ends:
                ends.add(end)
                utts.append(u)
            if len(ends) == 2 or T > 12000:
                break
    utts.append(synth.Utterance(np.zeros((1, 32), np.float32),
                                np.arange(1, 2305, dtype=np.int32) % 31 + 1, 0))
    bufs = _upload(utts)
    srv = ca.Server(64 << 30)
    res = [srv.wait(srv.submit(b["em"], b["lab"], b["path"], b["sc"], b["tot"], u.blank))
           for u, b in zip(utts, bufs)]
    srv.close()
    assert _check(utts, bufs, res) == []
    ends = {int(np.asarray(p)[-1]) != 0 for p in (b["path"].cpu().numpy() for b in bufs[:2])}
    assert ends == {True, False}                  # both end states taken
    assert res[-1][0] == 2                        # one frame: infeasible


def test_server_restarts_after_idle():
    # the resident kernel stops after ~20 ms without work and is started
    # again by the next request: requests separated by idle gaps (and a burst
    # right after a gap) all complete with the oracle's results
    import paper_2310_17864_amd as ca
    utts = _pool()[:9]
    bufs = _upload(utts)
    srv = ca.Server(64 << 30)
    res = [None] * len(utts)
    for i, (u, b) in enumerate(zip(utts, bufs)):
        if i in (0, 1, 2, 3):
            time.sleep(0.08)                      # longer than the idle stop
            res[i] = srv.wait(srv.submit(b["em"], b["lab"], b["path"], b["sc"], b["tot"], u.blank))
    time.sleep(0.08)
    tickets = {i: srv.submit(bufs[i]["em"], bufs[i]["lab"], bufs[i]["path"], bufs[i]["sc"],
                             bufs[i]["tot"], utts[i].blank) for i in range(4, len(utts))}
    for i, t in tickets.items():
        res[i] = srv.wait(t)
    srv.close()
    assert _check(utts, bufs, res) == []


def test_server_multi_workgroup_parts():
    # large requests run over several resident workgroups while a sync
    # region is free and on one workgroup otherwise: a burst larger than the
    # region pool takes both layouts, and a long run of one-at-a-time
    # requests takes one region through all its generations and its reset
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    big = synth.utterance(np.random.default_rng(31), 20000, 32, 4000, 0, 6.0, 1.0, None)
    st_o, p_o, s_o, _ = oracle.align_f32(big.emission, big.labels, 0)
    em = torch.from_numpy(big.emission).to(dev)
    lab = torch.from_numpy(big.labels).to(dev)
    outs = [(torch.full((big.T,), -7, dtype=torch.int32, device=dev),
             torch.empty(big.T, dtype=torch.float32, device=dev)) for _ in range(12)]
    torch.cuda.synchronize()
    srv = ca.Server(64 << 30)
    ts = [srv.submit(em, lab, p, s, None, 0) for p, s in outs]
    res = [srv.wait(t) for t in ts]
    assert all(r[0] == st_o for r in res)
    for p, s in outs:
        assert same_bits(p.cpu().numpy(), p_o) and same_bits(s.cpu().numpy(), s_o)

    small = synth.utterance(np.random.default_rng(32), 2400, 32, 2100, 0, 6.0, 1.0, None)
    st2, p2, s2, _ = oracle.align_f32(small.emission, small.labels, 0)
    em2 = torch.from_numpy(small.emission).to(dev)
    lab2 = torch.from_numpy(small.labels).to(dev)
    n = 1100                                    # > 1023 generations of one region
    paths = torch.full((n, small.T), -7, dtype=torch.int32, device=dev)
    scs = torch.empty((n, small.T), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    sts = []
    for i in range(n):                          # one at a time: region 0 each time
        sts.append(srv.wait(srv.submit(em2, lab2, paths[i], scs[i], None, 0))[0])
    assert sts == [st2] * n
    ref_p = torch.from_numpy(p2).to(dev)
    ref_s = torch.from_numpy(s2.view(np.int32)).to(dev)
    bad = int((paths != ref_p).any(dim=1).sum().item()) + \
        int((scs.view(torch.int32) != ref_s).any(dim=1).sum().item())
    srv.close()
    assert bad == 0


def test_server_padded_large_requests():
    # rows the kernels cannot stage directly (C not 32/256, or a misaligned
    # emission pointer) are padded by the workgroup that runs the request,
    # here on the one-workgroup layout of a large trellis
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    rng = np.random.default_rng(41)
    u1 = synth.utterance(rng, 12000, 100, 2500, 3, 6.0, 1.0, None)          # C = 100, blank 3
    u2 = synth.utterance(rng, 9000, 32, 1800, 0, 6.0, 1.0, None)            # misaligned rows
    flat = torch.zeros(u2.T * u2.C + 1, dtype=torch.float32, device=dev)
    flat[1:] = torch.from_numpy(u2.emission.reshape(-1)).to(dev)
    em2 = flat[1:].view(u2.T, u2.C)                                           # 4-byte offset
    outs = []
    srv = ca.Server(64 << 30)
    tickets = []
    for u, em in ((u1, torch.from_numpy(u1.emission).to(dev)), (u2, em2)):
        lab = torch.from_numpy(u.labels).to(dev)
        p = torch.full((u.T,), -7, dtype=torch.int32, device=dev)
        s = torch.empty(u.T, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        outs.append((u, em, lab, p, s))
        tickets.append(srv.submit(em, lab, p, s, None, u.blank))
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for (u, _, _, p, s), (st, _) in zip(outs, res):
        st_o, p_o, s_o, _ = oracle.align_f32(u.emission, u.labels, u.blank)
        assert st == st_o
        assert same_bits(p.cpu().numpy(), p_o) and same_bits(s.cpu().numpy(), s_o)


def test_server_on_few_workgroups(monkeypatch):
    # the resident kernel kept to 2 workgroups: requests queue for them, large
    # ones whose parts would need more workgroups take the one-workgroup
    # layout, and every result still matches the oracle
    monkeypatch.setenv("CTCALIGN_SERVE_WGS", "2")
    utts = _pool()
    bufs = _upload(utts)
    res, stats = _serve(utts, bufs, 64 << 30)
    assert _check(utts, bufs, res) == []
    assert stats["completed"] == len(utts)
