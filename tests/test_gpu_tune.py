"""The autotuner on the GPU (paper_2310_17864_amd/tune.py): per-size geometry
search for single launches and packs, the batched plan's knob search on a
workload, the table saved and loaded into a fresh context (same geometry
picks, same knob values), and a batch through a plan built from the loaded
table bit-exact against the CPU oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import compare_batched, torch_dev
from paper_2310_17864_amd import synth

pytestmark = pytest.mark.gpu


def test_tuner_round_trip_stays_exact(tmp_path):
    import paper_2310_17864_amd as ca
    from paper_2310_17864_amd import tune
    torch, dev = torch_dev()
    quiet = lambda *a: None
    ctx = ca.Context(0)
    best1 = tune.tune_single(ctx, 32, reps=1, samples=[81, 641], log=quiet)
    tune.apply(ctx, 0, 32, best1)
    best2 = tune.tune_pack(ctx, 256, batch=16, reps=1, samples=[161, 1025], log=quiet)
    tune.apply(ctx, 1, 256, best2)
    wl = synth.cfg_batched(n=64, t_hi=2000, seed=13)
    pk = synth.pack(wl.utts)
    grid = {"pack_target_m": (8, 12), "crit_frac": (0.0, 0.6), "crit_per_cu": (1.0,)}
    best, best_ms, default_ms, results = tune.tune_workload(ctx, pk, grid=grid, reps=1, log=quiet)
    assert best_ms <= default_ms and len(results) == 4
    path = str(tmp_path / "table.txt")
    ctx.tune_save(path)
    ctx2 = ca.Context(0)
    ctx2.tune_load(path)
    for S in list(best1) + [100, 300, 1000]:
        assert ctx2.tune_get(0, S, 32) == ctx.tune_get(0, S, 32)
    for S in list(best2) + [100, 700, 3000]:
        assert ctx2.tune_get(1, S, 256) == ctx.tune_get(1, S, 256)
    for k, v in best.items():
        assert ctx2.tune_knob(k) == v
    ref = oracle.align_batch_f32(pk, threads=8)
    em = torch.from_numpy(pk["em"]).to(dev)
    lab = torch.from_numpy(pk["lab"]).to(dev)
    plan = ca.Plan(em, pk["em_off"], pk["T"], pk["C"], lab, pk["lab_off"], pk["L"], pk["fr_off"], 0,
                   ctx=ctx2)
    plan.run()
    torch.cuda.synchronize()
    out = (plan.status.cpu().numpy()[: plan.n], plan.paths.cpu().numpy(), plan.scores.cpu().numpy(),
           plan.totals.cpu().numpy()[: plan.n])
    plan.close()
    assert compare_batched(pk, out, ref, "tuned") == []


def test_knob_limits():
    import paper_2310_17864_amd as ca
    ctx = ca.Context(0)
    prev = ctx.tune_knob("crit_frac", 0.5)
    assert ctx.tune_knob("crit_frac") == 0.5
    ctx.tune_knob("crit_frac", prev)
    with pytest.raises(ca.CtcAlignError):
        ctx.tune_knob("pack_target_m", 40)
    with pytest.raises(ca.CtcAlignError):
        ctx.tune_knob("crit_frac", 1.5)
