"""The allocation-free solve (stm_st_solve_noalloc) against stm_st_solve.

Both run the same solver kernels; the allocation-free call carves its team
synchronisation, task table, statistics and workspaces from the library's
fixed per-device array.  Two calls in a row, the second with fewer samples,
so the second starts from the array as the first left it.
"""

import ctypes

import numpy as np
import pytest

import oracle.api as oapi
import stinputs

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_noalloc_solve_matches_allocating_solve_on_two_calls():
    import torch
    from paper_1911_06066_amd import Context
    dev = torch.device("cuda:0")
    wl = stinputs.workload("small_mc_2d", steps=[32])
    basis = oapi.kl_basis(wl)
    modes = torch.from_numpy(oapi.kl_modes(wl, 0, basis)).to(dev)
    xi = torch.from_numpy(stinputs.xi("small_mc_2d", 0, 24, wl["n_modes"])).to(dev)
    with Context(wl) as ctx:
        sig = ctx.kl_synthesize(0, modes, xi)
        for S in (24, 7):
            s = sig[:S].contiguous()
            ref, st_ref = ctx.st_solve(0, s)
            out = torch.full_like(ref, float("nan"))
            u, st = ctx.st_solve(0, s, out=out, noalloc=True)
            torch.cuda.synchronize()
            assert u.data_ptr() == out.data_ptr()
            assert all(x["status"] == 0 for x in st) and all(x["status"] == 0 for x in st_ref)
            assert _rel(u.cpu().numpy(), ref.cpu().numpy()) < 1e-9
            assert all(x["newton_iters"] > 0 for x in st)


def test_noalloc_solve_rejects_a_workspace_beyond_the_array():
    """A 129 x 129 x 33 float64 level needs more than the fixed array for one
    lane: refused before any work, with the message saying so."""
    import torch
    from paper_1911_06066_amd import Context
    from paper_1911_06066_amd import _lib
    wl = stinputs.workload("mlmc5_3d", precision="fp64")
    with Context(wl, precision="fp64") as ctx:
        dummy = torch.zeros(4, dtype=torch.float64, device="cuda:0")
        st = ctx.lib.stm_st_solve_noalloc(ctx.h, 4, ctypes.c_void_p(dummy.data_ptr()), None, 1,
                                          ctypes.c_void_p(dummy.data_ptr()), None)
        assert _lib.STATUS[st] == "STM_E_INVALID"
        assert b"stm_st_solve_noalloc needs" in ctx.lib.stm_last_error(ctx.h)
