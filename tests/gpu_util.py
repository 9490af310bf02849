"""Helpers for GPU parity tests: run the HIP path through the C-ABI binding
and compare with the CPU oracle bit for bit."""
from __future__ import annotations

import numpy as np

import oracle


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def gpu_align(E: np.ndarray, y: np.ndarray, blank: int = 0):
    """(status, path, scores, total) from the single-utterance HIP path."""
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    e = torch.from_numpy(np.ascontiguousarray(E, dtype=np.float32)).to(dev)
    yy = np.asarray(y, dtype=np.int32).reshape(-1)
    lab = torch.from_numpy(yy if yy.size else np.zeros(1, np.int32)).to(dev)[: yy.size]
    if yy.size == 0:
        lab = torch.empty(0, dtype=torch.int32, device=dev)
    path, scores, total, status = ca.align(e, lab, blank, sync=False)
    torch.cuda.synchronize()
    return (int(status.item()), path.cpu().numpy(), scores.cpu().numpy(),
            np.float32(total.cpu().numpy()[0]))


def same_bits(a, b) -> bool:
    a = np.asarray(a)
    b = np.asarray(b)
    if a.shape != b.shape:
        return False
    if a.dtype == np.float32:
        return np.array_equal(a.view(np.uint32), b.astype(np.float32).view(np.uint32))
    return np.array_equal(a, b)


def compare_one(E, y, blank=0, label=""):
    """Return a list of mismatch messages between HIP path and oracle."""
    st_o, p_o, s_o, t_o = oracle.align_f32(E, y, blank)
    st_g, p_g, s_g, t_g = gpu_align(E, y, blank)
    errs = []
    if st_o != st_g:
        errs.append(f"{label}: status gpu {st_g} oracle {st_o}")
        return errs
    if not same_bits(p_g, p_o):
        bad = np.nonzero(p_g != p_o)[0]
        errs.append(f"{label}: path differs at {len(bad)} frames, first {bad[:5]}")
    if not same_bits(s_g, s_o):
        errs.append(f"{label}: scores differ")
    if st_o in (0, 2) and np.float32(t_g).view(np.uint32) != np.float32(t_o).view(np.uint32):
        errs.append(f"{label}: total gpu {t_g!r} oracle {t_o!r}")
    if st_o == 1 and not np.isnan(t_g):
        errs.append(f"{label}: total should be NaN for invalid labels")
    return errs


def upload_packed(pk: dict):
    torch, dev = torch_dev()
    em = torch.from_numpy(pk["em"]).to(dev)
    lab = torch.from_numpy(pk["lab"]).to(dev)
    return em, lab


def gpu_batched(pk: dict, blank: int = 0, runs: int = 1):
    """Align a packed batch with one plan; returns (status, paths, scores, totals)
    after the last of `runs` graph replays."""
    import paper_2310_17864_amd as ca
    torch, dev = torch_dev()
    em, lab = upload_packed(pk)
    plan = ca.Plan(em, pk["em_off"], pk["T"], pk["C"], lab, pk["lab_off"], pk["L"],
                   pk["fr_off"], blank)
    outs = []
    for _ in range(runs):
        plan.paths.fill_(-7)
        plan.scores.fill_(float("nan"))
        plan.run()
        torch.cuda.synchronize()
        outs.append((plan.status.cpu().numpy()[: plan.n].copy(), plan.paths.cpu().numpy().copy(),
                     plan.scores.cpu().numpy().copy(), plan.totals.cpu().numpy()[: plan.n].copy()))
    plan.close()
    return outs if runs > 1 else outs[0]


def compare_batched(pk: dict, gpu_out, oracle_out, label=""):
    st_g, p_g, s_g, t_g = gpu_out
    st_o, p_o, s_o, t_o, _ = oracle_out
    n = len(pk["T"])
    F = int(pk["frames"])
    errs = []
    if not np.array_equal(st_g, st_o):
        errs.append(f"{label}: statuses differ at {np.nonzero(st_g != st_o)[0][:10]}")
    if not same_bits(p_g[:F], p_o):
        bad = np.nonzero(p_g[:F] != p_o)[0]
        utt = np.searchsorted(pk["fr_off"], bad[:5], side="right") - 1
        errs.append(f"{label}: paths differ at {len(bad)} frames (utterances {utt})")
    if not same_bits(s_g[:F], s_o):
        errs.append(f"{label}: scores differ")
    ok = st_o == 0
    if not np.array_equal(t_g[ok].view(np.uint32), t_o[ok].view(np.uint32)):
        errs.append(f"{label}: totals differ")
    return errs
