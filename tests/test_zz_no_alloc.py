"""The allocation-free forward pass of the warm-start network
(swr_mlp_forward_noalloc) against swr_mlp_forward, through the C ABI: the
same kernels on the library's own scratch array instead of a caller
workspace, so the outputs agree bit for bit.  Two calls in a row, the
second with a smaller batch (the array keeps the first call's contents),
and a batch whose activations exceed the array is refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_forward_matches_workspace_forward():
    import torch
    from paper_1710_02401_amd import swr as S
    lib = S.load_library()
    d = S.swr_mlp_desc(552, 256, 3, 16384)
    n = ctypes.c_int64()
    assert lib.swr_mlp_param_count(ctypes.byref(d), ctypes.byref(n)) == 0
    g = torch.Generator().manual_seed(7)
    params = (torch.rand(n.value, generator=g, dtype=torch.float32) - 0.5).mul_(0.1).cuda()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for batch in (96, 17):
        print(f"[gpu] no-alloc forward, batch {batch}", flush=True)
        x = torch.rand(batch, 552, generator=g, dtype=torch.float32).cuda()
        ws_bytes = ctypes.c_uint64()
        assert lib.swr_mlp_workspace_bytes(ctypes.byref(d), batch, ctypes.byref(ws_bytes)) == 0
        ws = torch.empty(ws_bytes.value, dtype=torch.uint8, device="cuda")
        y_ref = torch.empty(batch, 16384, dtype=torch.float32, device="cuda")
        y = torch.full((batch, 16384), float("nan"), dtype=torch.float32, device="cuda")
        assert lib.swr_mlp_forward(ctypes.byref(d), S._vp(params), S._vp(x), batch, S._vp(y_ref),
                                   S._vp(ws), ws_bytes, stream) == 0
        assert lib.swr_mlp_forward_noalloc(ctypes.byref(d), S._vp(params), S._vp(x), batch,
                                           S._vp(y), stream) == 0
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        assert bool(torch.isfinite(y).all())
    # activations beyond the 64 MiB array: refused on the host, nothing runs
    big = 1024
    x = torch.zeros(1, 552, dtype=torch.float32, device="cuda")
    y = torch.zeros(1, 16384, dtype=torch.float32, device="cuda")
    assert lib.swr_mlp_forward_noalloc(ctypes.byref(d), S._vp(params), S._vp(x), big, S._vp(y),
                                       stream) == S.SWR_E_SIZE
