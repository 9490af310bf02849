"""Calls that share library state across HIP streams, through the C-ABI:
single alignments without a workspace of their own on two streams at once
(they share the context's backpointer arena and pad buffer), one batched
plan replayed on two streams (its workspace and queue heads), and a served
request whose inputs are still being written on another stream when it is
submitted (its ready event).  Every result is compared bit for bit with the
float32 oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import compare_batched, same_bits, torch_dev
from paper_2310_17864_amd import synth

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(77)
    shapes = [(300, 32, 60), (1200, 256, 250), (900, 17, 150), (5100, 32, 2500),
              (800, 100, 120), (2000, 32, 900), (14100, 32, 7000), (400, 256, 80)]
    return [synth.utterance(rng, T, C, L, 0, 6.0, 1.0, None) for T, C, L in shapes]


def test_single_alignments_on_two_streams():
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    utts = _cases()
    ins = [(torch.from_numpy(u.emission).to(dev), torch.from_numpy(u.labels).to(dev)) for u in utts]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for rep in range(3):
        for k, (e, y) in enumerate(ins):
            s = streams[(k + rep) % 2]
            with torch.cuda.stream(s):
                outs.append((k, ca.align(e, y, 0, sync=False)))
    torch.cuda.synchronize()
    ref = [oracle.align_f32(u.emission, u.labels, 0) for u in utts]
    for k, (path, scores, total, status) in outs:
        st, p, sc, t = ref[k]
        assert int(status.item()) == st == 0, k
        assert same_bits(path.cpu().numpy(), p), k
        assert same_bits(scores.cpu().numpy(), sc), k
        assert np.float32(total.cpu().numpy()[0]).view(np.uint32) == np.float32(t).view(np.uint32), k


def test_plan_replayed_on_two_streams():
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    wl = synth.cfg_batched(n=80, t_hi=3000, seed=31)
    pk = synth.pack(wl.utts)
    ref = oracle.align_batch_f32(pk, threads=8)
    plan = ca.Plan(torch.from_numpy(pk["em"]).to(dev), pk["em_off"], pk["T"], pk["C"],
                   torch.from_numpy(pk["lab"]).to(dev), pk["lab_off"], pk["L"], pk["fr_off"], 0)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(6):
        plan.run(streams[rep % 2])
    torch.cuda.synchronize()
    out = (plan.status.cpu().numpy()[: plan.n], plan.paths.cpu().numpy(), plan.scores.cpu().numpy(),
           plan.totals.cpu().numpy()[: plan.n])
    plan.close()
    assert compare_batched(pk, out, ref, "two-stream plan") == []


def test_served_request_waits_for_its_inputs():
    # the emission is copied in on a side stream behind a spinning kernel,
    # and submitted without a host synchronisation: the request's ready
    # event holds it back until the copy is done
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    rng = np.random.default_rng(5)
    utts = [synth.utterance(rng, T, C, L, 0, 6.0, 1.0, None)
            for T, C, L in [(1500, 32, 300), (700, 256, 130), (6000, 32, 2400)]]
    srv = ca.Server(1 << 30)
    side = torch.cuda.Stream()
    bufs, tickets = [], []
    for u in utts:
        b = dict(src=torch.from_numpy(u.emission).pin_memory(),
                 em=torch.zeros((u.T, u.C), dtype=torch.float32, device=dev),
                 lab=torch.from_numpy(u.labels).to(dev),
                 path=torch.full((u.T,), -7, dtype=torch.int32, device=dev),
                 sc=torch.empty(u.T, dtype=torch.float32, device=dev),
                 tot=torch.empty(1, dtype=torch.float32, device=dev))
        bufs.append(b)
    torch.cuda.synchronize()
    for u, b in zip(utts, bufs):
        with torch.cuda.stream(side):
            torch.cuda._sleep(20_000_000)
            b["em"].copy_(b["src"], non_blocking=True)
            tickets.append(srv.submit(b["em"], b["lab"], b["path"], b["sc"], b["tot"]))
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for u, b, (st, tm) in zip(utts, bufs, results):
        st_o, p_o, s_o, t_o = oracle.align_f32(u.emission, u.labels, 0)
        assert st == st_o == 0
        assert same_bits(b["path"].cpu().numpy(), p_o)
        assert same_bits(b["sc"].cpu().numpy(), s_o)
        assert np.float32(b["tot"].cpu().numpy()[0]).view(np.uint32) == np.float32(t_o).view(np.uint32)
