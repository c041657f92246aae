"""GPU: the allocation-free entry point (epic_interp_noalloc) through the C
ABI gives, bitwise, what epic_interp gives: on the 1024 x 436 scene and then
on a smaller one in the next call (the library's device array keeps the
last call's contents; each call clears what it needs).  Sizes beyond its
64 MiB array are refused on the host."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from scenes import config_scene, random_case


def _noalloc(lib, cost, m, K, a, mode, flow):
    import torch
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    H, W = cost.shape
    return lib.epic_interp_noalloc(cost.data_ptr(), H, W, m.data_ptr(), m.shape[0], int(K), float(a),
                                   int(mode), flow.data_ptr(), stream)


@pytest.mark.gpu
def test_noalloc_equals_interp_twice():
    import torch
    import paper_1501_02565_amd as epic
    from paper_1501_02565_amd import _lib
    lib = _lib.load()
    cases = [config_scene(2), random_case(96, 128, 300, seed=71, K=32)]   # the second is smaller
    with epic.Context(0, epic.workspace_bytes(436, 1024, 8000, 100)) as ctx:
        for sc in cases:
            print(f"[case] noalloc {sc.name}", flush=True)
            c = torch.from_numpy(sc.cost).cuda()
            m = torch.from_numpy(sc.matches).cuda()
            f0 = torch.full((sc.H, sc.W, 2), float("nan"), device="cuda")
            assert _noalloc(lib, c, m, sc.K, sc.a, sc.mode, f0) == 0
            f1 = ctx.interp(c, m, sc.K, sc.a, sc.mode)
            torch.cuda.synchronize()
            assert ctx.stats(0)["status"] == 0
            assert torch.equal(f0, f1)


def test_noalloc_refuses_oversize():
    """Host-side check, before any device call."""
    from paper_1501_02565_amd import _lib
    lib = _lib.load()
    P = ctypes.c_void_p(0x1000)
    assert lib.epic_interp_noalloc(P, 4096, 4096, P, 100000, 100, 1.0, 1, P, None) == _lib.ERR_WORKSPACE
    assert lib.epic_interp_noalloc(P, 10, 20, P, 5, 3, -1.0, 1, P, None) == _lib.ERR_ARG
