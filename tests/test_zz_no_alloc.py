"""ctcalign_align_noalloc through the C-ABI: the same bits as
ctcalign_align_ex (which allocates its workspace) and as the float32 oracle,
on two calls in a row, the second smaller than the first (the scratch array
keeps the first call's contents), including a padded class count and a
trellis above the single-wave sizes; a call that needs more scratch than the
array holds is refused with ENOMEM and launches nothing."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import same_bits, torch_dev
from paper_2310_17864_amd import synth

pytestmark = pytest.mark.gpu


def _run(lib, fn_name, ctx, e, y, blank, outs, stream):
    path, scores, total, status = outs
    T, C = e.shape
    L = y.numel()
    if fn_name == "ex":
        return lib.ctcalign_align_ex(ctx, e.data_ptr(), T, C, y.data_ptr() if L else None, L, blank,
                                     path.data_ptr(), scores.data_ptr(), total.data_ptr(),
                                     status.data_ptr(), None, 0, stream)
    return lib.ctcalign_align_noalloc(ctx, e.data_ptr(), T, C, y.data_ptr() if L else None, L, blank,
                                      path.data_ptr(), scores.data_ptr(), total.data_ptr(),
                                      status.data_ptr(), stream)


def _outs(torch, dev, T):
    return (torch.full((T,), -7, dtype=torch.int32, device=dev),
            torch.full((T,), 7.0, dtype=torch.float32, device=dev),
            torch.zeros(1, dtype=torch.float32, device=dev),
            torch.full((1,), -1, dtype=torch.int32, device=dev))


def test_noalloc_matches_align_ex_and_oracle():
    import paper_2310_17864_amd as ca
    from paper_2310_17864_amd import _lib
    torch, dev = torch_dev()
    lib = _lib.load()
    ctx = ca.context(0).handle
    assert lib.ctcalign_noalloc_scratch_bytes() == 64 << 20
    rng = np.random.default_rng(2024)
    # first the larger call (S = 10,001: one 7-wave workgroup, ~40 MB of
    # backpointers), then a smaller padded one (C = 17), then a tiny one
    cases = [synth.utterance(rng, 20_000, 32, 5000, 0, 6.0, 1.0, 0.1),
             synth.utterance(rng, 900, 17, 150, 3, 6.0, 1.0, None),
             synth.utterance(rng, 200, 256, 40, 0, 6.0, 1.0, None)]
    stream = torch.cuda.current_stream().cuda_stream
    for k, u in enumerate(cases):
        e = torch.from_numpy(u.emission).to(dev)
        y = torch.from_numpy(u.labels).to(dev)
        a, b = _outs(torch, dev, u.T), _outs(torch, dev, u.T)
        torch.cuda.synchronize()
        assert _run(lib, "noalloc", ctx, e, y, u.blank, a, stream) == 0, k
        torch.cuda.synchronize()
        assert _run(lib, "ex", ctx, e, y, u.blank, b, stream) == 0, k
        torch.cuda.synchronize()
        st, p, s, t = oracle.align_f32(u.emission, u.labels, u.blank)
        for got in (a, b):
            assert int(got[3].item()) == st == 0, k
            assert same_bits(got[0].cpu().numpy(), p), k
            assert same_bits(got[1].cpu().numpy(), s), k
            assert np.float32(got[2].cpu().numpy()[0]).view(np.uint32) == np.float32(t).view(np.uint32), k


def test_noalloc_refuses_oversize():
    import paper_2310_17864_amd as ca
    from paper_2310_17864_amd import _lib
    torch, dev = torch_dev()
    lib = _lib.load()
    ctx = ca.context(0).handle
    # T * S * 3/16 bytes of backpointers well above 64 MiB: refused, nothing written
    T, L, C = 60_000, 6000, 32
    e = torch.zeros((T, C), dtype=torch.float32, device=dev)
    y = torch.ones(L, dtype=torch.int32, device=dev)
    outs = _outs(torch, dev, T)
    torch.cuda.synchronize()
    rc = _run(lib, "noalloc", ctx, e, y, 0, outs, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == ca.ENOMEM
    assert int(outs[3].item()) == -1 and int(outs[0][0].item()) == -7
