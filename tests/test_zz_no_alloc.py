"""mc_apply_H_direct_noalloc (the table-free apply with its staged constants
in a library-owned device array, for callers that cannot allocate) against
mc_apply_H_direct with a caller workspace: bitwise equal on consecutive
calls, each smaller than the one before, through the C ABI."""

import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import rel_inf

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_noalloc_apply_matches_workspace_apply(mc, oracle_native):
    from paper_2005_13679_amd import _lib as L
    lib = L.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    need = ctypes.c_size_t(0)
    assert lib.mc_workspace_size(14, 8, L.MC_OP_APPLY, ctypes.byref(need)) == 0
    assert need.value <= lib_scratch_bytes()
    # dims 324,632, then 116,280 (M = 8, the largest constants), then 220
    for N, M, seed in [(30, 6, 1), (14, 8, 2), (9, 4, 3)]:
        C, h, g = W.random_instance(N, M, seed)
        Cd, hd, gd = (torch.from_numpy(x).cuda() for x in (C, h, g))
        out = torch.full_like(Cd, float("nan"))
        print(f"[no-alloc] N={N} M={M} dim={C.size}", flush=True)
        st = lib.mc_apply_H_direct_noalloc(N, M, _p(hd), _p(gd), _p(Cd), _p(out), stream)
        assert st == 0, lib.mc_strerror(st)
        ref = mc.apply_H_direct(hd, gd, Cd, N, M)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        if C.size <= 400_000:
            assert rel_inf(out.cpu().numpy(), oracle_native.apply_h(N, M, h, g, C)) <= 1e-12
    # sizes the table-free apply rejects are rejected here too
    z = torch.zeros(mc.dim(2, 9), dtype=torch.complex128, device="cuda")
    hz = torch.zeros(81, dtype=torch.complex128, device="cuda")
    gz = torch.zeros(9 ** 4, dtype=torch.complex128, device="cuda")
    assert lib.mc_apply_H_direct_noalloc(2, 9, _p(hz), _p(gz), _p(z), _p(z.clone()), stream) != 0


def lib_scratch_bytes():
    import re
    import os
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mc.h")
    with open(hdr) as f:
        return int(re.search(r"#define MC_NOALLOC_SCRATCH_BYTES (\d+)", f.read()).group(1))
