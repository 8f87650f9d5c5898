"""The allocation-free output head (tpfnn_head_noalloc) against tpfnn_head with a
caller workspace, through the C ABI: two calls in a row, the second on a
smaller input, and a size beyond its fixed scratch array."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _inputs(torch, rng, npix, Cc):
    x = torch.from_numpy((rng.normal(size=(npix, Cc)) * 0.5).astype(np.float32)).to(torch.bfloat16).cuda()
    w = torch.from_numpy((rng.normal(size=Cc) * 0.3).astype(np.float32)).cuda()
    b = torch.tensor([0.1], dtype=torch.float32, device="cuda")
    t = torch.from_numpy(rng.uniform(size=npix).astype(np.float32)).cuda()
    return x, w, b, t


def _outputs(torch, npix, Cc):
    return (torch.full((npix,), float("nan"), dtype=torch.float32, device="cuda"),
            torch.zeros(npix * Cc, dtype=torch.bfloat16, device="cuda"),
            torch.zeros(Cc, dtype=torch.float32, device="cuda"),
            torch.zeros(1, dtype=torch.float32, device="cuda"),
            torch.zeros(1, dtype=torch.float64, device="cuda"))


def test_head_noalloc_matches_head_with_workspace():
    import torch
    from paper_2311_05091_amd.surrogate import nnlib
    lib = nnlib()
    p = lambda t: C.c_void_p(t.data_ptr())
    rng = np.random.default_rng(5)
    for npix, Cc in ((200_000, 32), (4096, 32)):   # second call on a smaller input
        _say("head_noalloc", npix, Cc)
        x, w, b, t = _inputs(torch, rng, npix, Cc)
        ref = _outputs(torch, npix, Cc)
        got = _outputs(torch, npix, Cc)
        ws = lib.tpfnn_head_workspace(npix, Cc)
        work = torch.empty(int(ws), dtype=torch.uint8, device="cuda")
        assert lib.tpfnn_head(p(x), npix, Cc, p(w), p(b), p(ref[0]), p(t), p(ref[1]), p(ref[2]), p(ref[3]),
                              p(ref[4]), p(work), work.numel(), None) == 0
        assert lib.tpfnn_head_noalloc(p(x), npix, Cc, p(w), p(b), p(got[0]), p(t), p(got[1]), p(got[2]),
                                      p(got[3]), p(got[4]), None) == 0
        torch.cuda.synchronize()
        for a, r in zip(got, ref):
            assert torch.equal(a, r)
        assert torch.isfinite(got[0]).all() and got[4].item() > 0
        # inference form (no target): predictions only
        pred = torch.full((npix,), float("nan"), dtype=torch.float32, device="cuda")
        assert lib.tpfnn_head_noalloc(p(x), npix, Cc, p(w), p(b), p(pred), None, None, None, None, None,
                                      None) == 0
        torch.cuda.synchronize()
        assert torch.equal(pred, ref[0])


def test_head_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    from paper_2311_05091_amd.surrogate import nnlib
    lib = nnlib()
    p = lambda t: C.c_void_p(t.data_ptr())
    _say("head_noalloc too large")
    small = torch.zeros(64, dtype=torch.float32, device="cuda")
    limit = 4 << 20
    npix = 1
    while lib.tpfnn_head_workspace(npix, 32) <= limit:
        npix *= 2
    # the size check comes before any launch, so the small buffers are never read
    assert lib.tpfnn_head_noalloc(p(small), npix, 32, p(small), p(small), p(small), p(small), p(small), p(small),
                                  p(small), p(small), None) == -1
