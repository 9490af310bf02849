"""Autotuner for the geometry table (waves per alignment W, states per lane M).

For each sampled trellis size S and class count C it times every geometry the
kernels compile that can hold S, on synthetic emissions, and writes the
fastest into the context's table (ctcalign_tune_set) for the S range between
the neighbouring samples; the table can be saved and later loaded through
$CTCALIGN_TUNE_CACHE.

* kind 0 (single launches): objective = latency of one alignment.
* kind 1 (batched persistent kernel): objective = time of a batch of
  `batch` alignments of that size through one plan.

    python -m paper_2310_17864_amd.tune --out tune.txt
"""
from __future__ import annotations

import argparse
import sys
import time
from typing import Dict, List, Tuple

import numpy as np

ONE = [(W, M) for W in (1, 2, 3, 4) for M in (2, 4, 6, 8, 10, 12, 14, 16)] + \
      [(W, M) for W in range(1, 9) for M in (16, 24, 32, 40, 48, 56, 60, 64)]
PACK = [(W, M) for W in (1, 2, 4) for M in (2, 4, 6, 8, 12, 16)]
S_SAMPLES_ONE = [41, 81, 161, 321, 641, 1025, 1601, 2401, 3201, 4097, 6001, 8001, 12001,
                 16001, 24001, 30001]
S_SAMPLES_PACK = [41, 81, 161, 321, 641, 1025, 1601, 2401, 3201, 4097]


def holds(S: int, W: int, M: int) -> bool:
    seg = 64 * M
    return W * seg >= S and (W == 1 or (W - 1) * seg + 2 <= S)


def _utt(S: int, C: int, frames_per_label: float, seed: int):
    from . import synth
    L = (S - 1) // 2
    T = max(int(frames_per_label * L), 2 * L + 2, 16)
    return synth.utterance(np.random.default_rng(seed), T, C, L, 0, 6.0, 1.0, None)


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def tune_single(ctx, C: int, reps: int = 5, frames_per_label: float = 5.0,
                samples=S_SAMPLES_ONE, log=print) -> Dict[int, Tuple[int, int, float]]:
    import torch

    from . import align
    dev = torch.device("cuda", ctx.device)
    best: Dict[int, Tuple[int, int, float]] = {}
    for S in samples:
        u = _utt(S, C, frames_per_label, S)
        e = torch.from_numpy(u.emission).to(dev)
        y = torch.from_numpy(u.labels).to(dev)
        out = align(e, y, 0, sync=False)
        res = []
        for W, M in ONE:
            if not holds(S, W, M):
                continue
            ctx.tune_set(0, S, S, C, W, M)
            ms = _time(lambda: align(e, y, 0, out=out, sync=False), reps)
            res.append((ms, W, M))
            ctx.tune_clear(0, S, S, C)
        ms, W, M = min(res)
        best[S] = (W, M, ms)
        log(f"single C={C} S={S}: W={W} M={M} {ms * 1e3:.1f} us ({len(res)} candidates)")
    return best


def tune_pack(ctx, C: int, batch: int = 512, reps: int = 3, frames_per_label: float = 5.0,
              samples=S_SAMPLES_PACK, log=print) -> Dict[int, Tuple[int, int, float]]:
    import torch

    from . import Plan, synth
    dev = torch.device("cuda", ctx.device)
    best: Dict[int, Tuple[int, int, float]] = {}
    for S in samples:
        utts = [_utt(S, C, frames_per_label, 1000 * S + i) for i in range(batch)]
        pk = synth.pack(utts)
        em = torch.from_numpy(pk["em"]).to(dev)
        lab = torch.from_numpy(pk["lab"]).to(dev)
        res = []
        for W, M in PACK:
            if not holds(S, W, M):
                continue
            ctx.tune_set(1, S, S, C, W, M)
            plan = Plan(em, pk["em_off"], pk["T"], pk["C"], lab, pk["lab_off"], pk["L"],
                        pk["fr_off"], 0, ctx=ctx)
            ms = _time(plan.run, reps)
            plan.close()
            res.append((ms, W, M))
            ctx.tune_clear(1, S, S, C)
        ms, W, M = min(res)
        best[S] = (W, M, ms)
        log(f"pack C={C} S={S}: W={W} M={M} {ms:.3f} ms per {batch} ({len(res)} candidates)")
    return best


def apply(ctx, kind: int, C: int, best: Dict[int, Tuple[int, int, float]]) -> List[tuple]:
    """Write each sample's winner over the S range up to the next sample
    (64-state buckets), where that geometry holds every S of the range."""
    keys = sorted(best)
    applied = []
    for i, S in enumerate(keys):
        W, M, _ = best[S]
        lo = keys[i - 1] + 1 if i else 1
        hi = keys[i + 1] - 1 if i + 1 < len(keys) else S
        # shrink to the part of [lo, hi] this geometry can hold
        seg = 64 * M
        a = max(lo, (W - 1) * seg + 2 if W > 1 else 1)
        b = min(hi, W * seg)
        a, b = max(a, lo), max(min(b, hi), a)
        # whole 64-state buckets only
        a = (a + 63) // 64 * 64 if a % 64 else a
        b = (b + 1) // 64 * 64 - 1
        if a <= S <= b or b >= a:
            try:
                ctx.tune_set(kind, a, b, C, W, M)
                applied.append((kind, C, a, b, W, M))
            except Exception:
                pass
    return applied


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="ctcalign_tune.txt")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--batch", type=int, default=256)
    args = ap.parse_args(argv)
    from . import context
    ctx = context(0)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    t0 = time.time()
    for C in (32, 256):
        apply(ctx, 0, C, tune_single(ctx, C, args.reps, log=log))
        apply(ctx, 1, C, tune_pack(ctx, C, args.batch, args.reps, log=log))
    ctx.tune_save(args.out)
    log(f"tuning table written to {args.out} in {time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
