"""phgrms_denoise_noalloc: the pass loop with the library's fixed device
scratch as workspace, no allocation.  Checked against phgrms_denoise_async
(the same path with a caller workspace) bit for bit -- image, iteration
count and per-pass counts -- on two calls in a row, the second with a
smaller image (the scratch keeps the first call's contents), through the C
ABI; captured into a graph and replayed; and a workspace above the
scratch's size is refused before any work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1306_5390_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _lib():
    from paper_1306_5390_amd import _api
    lib = _api.load_library()
    lib.phgrms_denoise_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _api.Params,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.phgrms_denoise_noalloc.restype = ctypes.c_int
    return _api, lib


def _noalloc(api, lib, img, alpha, beta, k, stream):
    rows, cols = img.shape
    out = torch.empty_like(img)
    ch = torch.full((max(k, 1),), -1, dtype=torch.int64, device=DEV)
    it = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    rc = lib.phgrms_denoise_noalloc(img.data_ptr(), out.data_ptr(),
                                    api.Params(rows, cols, alpha, beta, k), ch.data_ptr(),
                                    it.data_ptr(), stream.cuda_stream)
    assert rc == 0, lib.phgrms_last_error()
    return out, ch, it


@pytest.mark.parametrize("shape_kind", ["tuned", "skipping"])
def test_noalloc_matches_workspace_path(shape_kind):
    api, lib = _lib()
    cases = [((1500, 2100, 0.4, 31), 20, 2, 24), ((300, 517, 0.2, 32), 10, 1, 9)]
    skip = [s for s in range(len(api.shapes())) if api.shape_skips_unchanged(s)]
    old = {(b, c): api.get_tuning_class(b, c) for b in (1, 2) for c in range(3)}
    try:
        if shape_kind == "skipping":
            for b in (1, 2):
                api.set_tuning(b, skip[0])
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        for (h, w, rho, seed), alpha, beta, k in cases:
            img = torch.from_numpy(synth.noisy_image(h, w, rho, seed)).to(DEV)
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                out, ch, it = _noalloc(api, lib, img, alpha, beta, k, s)
                ref, rch, rit = api.denoise_async(img, alpha, beta, k, stream=s)
            torch.cuda.synchronize()
            n = int(rit.item())
            assert int(it.item()) == n
            assert torch.equal(out, ref), ((h, w), alpha, beta, k)
            assert ch[:n].cpu().tolist() == rch[:n].cpu().tolist()
    finally:
        for (b, c), v in old.items():
            api.set_tuning_class(b, c, v)


def test_noalloc_captured_in_a_graph():
    # the callers it is for: code under graph capture.  One eager call first
    # (it looks the scratch address up), then the call is captured, and the
    # graph's replays, with the outputs overwritten and a workspace-path run
    # between them, equal the workspace path's result.
    api, lib = _lib()
    img = torch.from_numpy(synth.noisy_image(700, 900, 0.3, 33)).to(DEV)
    ref, rit, rch = api.denoise(img, 20, 2, 10)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        _noalloc(api, lib, img, 20, 2, 10, s)
    torch.cuda.synchronize()
    out = torch.empty_like(img)
    ch = torch.zeros(10, dtype=torch.int64, device=DEV)
    it = torch.zeros(1, dtype=torch.int32, device=DEV)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rc = lib.phgrms_denoise_noalloc(img.data_ptr(), out.data_ptr(),
                                        api.Params(700, 900, 20, 2, 10), ch.data_ptr(),
                                        it.data_ptr(), s.cuda_stream)
    assert rc == 0, lib.phgrms_last_error()
    other = torch.from_numpy(synth.noisy_image(200, 200, 0.5, 34)).to(DEV)
    for rep in range(3):
        print("noalloc graph replay", rep, flush=True)
        out.fill_(0)
        ch.fill_(-1)
        it.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(it.item()) == rit
        assert ch[:rit].cpu().tolist() == rch
        assert torch.equal(out, ref), rep
        api.denoise(other, 20, 1, 4)
        torch.cuda.synchronize()


def test_noalloc_refuses_what_does_not_fit():
    api, lib = _lib()
    big = api.Params(16384, 16384, 20, 2, 32)
    assert api.workspace_bytes(16384, 16384, 20, 2, 32) > (96 << 20)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: the size check comes first
    assert lib.phgrms_denoise_noalloc(fake, fake, big, None, None, None) == -2
    assert b"scratch" in lib.phgrms_last_error()
