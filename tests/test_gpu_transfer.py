"""GPU parity of the space-time prolongation (Sec. 3.4) and its use as the
first Newton iterate of the fine member of a pair."""

import numpy as np
import pytest

import oracle.api as oapi
import stinputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("case", ["2d", "2d_ratio3", "3d", "cube"])
def test_prolongation_matches_oracle(torch_dev, case):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    if case == "2d":
        wl = stinputs.workload("small_mc_2d", levels=[(9, 7), (17, 13), (33, 25)], steps=[5, 10, 20],
                               lengths=(1.0, 0.75))
    elif case == "2d_ratio3":
        wl = stinputs.workload("small_mc_2d", levels=[(9, 9), (17, 17)], steps=[4, 12])
    elif case == "3d":
        wl = stinputs.workload("slab3d", levels=[(9, 9, 3), (17, 17, 5)], steps=[6, 12], precision="fp64")
    else:
        wl = stinputs.workload("cube4_3d", levels=[(6, 6, 6), (11, 11, 11)], steps=[24, 48])
    ctx = Context(wl)
    L = len(wl["levels"])
    rng = np.random.default_rng(7)
    for l in range(1, L):
        nc, _, mc = ctx.sizes[l - 1]
        Uc = rng.uniform(-0.2, 1.2, (3, mc, nc))
        Uf = ctx.prolong_st(l, torch.from_numpy(Uc).to(dev)).cpu().numpy()
        ref = oapi.prolong_st(wl, l, Uc)
        assert np.abs(Uf - ref).max() <= 1e-14


@pytest.mark.parametrize("workload", ["mlmc3_2d", "cube4_3d"])
def test_prolonged_coarse_solution_as_first_iterate(torch_dev, workload):
    """The fine solve from the prolonged coarse solution reaches the same
    solution as from its default first iterate."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    if workload == "mlmc3_2d":
        wl = stinputs.workload("mlmc3_2d", levels=[(17, 17), (33, 33)], steps=[16, 32], kl_grid=(17, 17))
    else:
        wl = stinputs.workload("cube4_3d", levels=[(6, 6, 6), (11, 11, 11)], steps=[24, 48], kl_grid=(11, 11, 11))
    basis = oapi.kl_basis(wl)
    modes = [torch.from_numpy(oapi.kl_modes(wl, l, basis)).to(dev) for l in range(2)]
    y = torch.from_numpy(stinputs.xi(wl["name"], 1, 3, wl["n_modes"])).to(dev)
    ctx = Context(wl, max_lanes=3)
    sc = ctx.kl_synthesize(0, modes[0], y)
    sf = ctx.kl_synthesize(1, modes[1], y)
    uc, _ = ctx.st_solve(0, sc)
    guess = ctx.prolong_st(1, uc)
    u1, st1 = ctx.st_solve(1, sf)
    u2, st2 = ctx.st_solve(1, sf, u0_guess=guess)
    assert all(s["status"] == 0 for s in st1 + st2)
    assert _rel(u2.cpu().numpy(), u1.cpu().numpy()) < 1e-9


def test_prolongation_rejects_bad_arguments(torch_dev):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context, StmError
    wl = stinputs.workload("small_mc_2d", levels=[(9, 9), (17, 17)], steps=[4, 8])
    ctx = Context(wl)
    nc, _, mc = ctx.sizes[0]
    u = torch.zeros((2, mc, nc), dtype=torch.float64, device=dev)
    out = torch.empty((2, 8, ctx.sizes[1][0]), dtype=torch.float64, device=dev)
    for level in (0, 2):
        st = ctx.lib.stm_prolong_st(ctx.h, level, u.data_ptr(), 2, out.data_ptr())
        assert st == -1
    assert ctx.lib.stm_prolong_st(ctx.h, 1, None, 2, out.data_ptr()) == -1
    assert ctx.lib.stm_prolong_st(ctx.h, 1, u.data_ptr(), 0, out.data_ptr()) == 0


@pytest.mark.parametrize("case", ["2d", "strip", "strip_split"])
def test_space_time_qoi_mlmc_matches_oracle(torch_dev, case):
    """E[u] on the finest space-time grid (Sec. 4.1): mean, variance, level
    fields and V_l in the L^2(0, T; L^2(D)) sense against the oracle."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    if case == "2d":
        wl = stinputs.workload("small_mc_2d", levels=[(9, 9), (17, 17), (33, 33)], steps=[6, 12, 24],
                               n_modes=8, kl_grid=(17, 17), ic_radius=0.25, sigma_f0=4e-3, qoi="spacetime")
        N = [8, 4, 3]
    else:
        wl = stinputs.workload("cable1d", levels=[(32, 2), (63, 2), (125, 2)], steps=[4, 8, 16],
                               kl_grid=(125, 2))
        N = [16, 8, 4] if case == "strip" else [16, 8, 9]  # 9 finest pairs: the split group path
    basis = oapi.kl_basis(wl)
    modes = [oapi.kl_modes(wl, l, basis) for l in range(3)]
    xi = [stinputs.xi(wl["name"], l, N[l], wl["n_modes"]) for l in range(3)]
    ctx = Context(wl)
    out = ctx.mlmc_estimate(N, [torch.from_numpy(m).to(dev) for m in modes],
                            [torch.from_numpy(x).to(dev) for x in xi])
    ref = oapi.mlmc_estimate(wl, N, xi, modes, solve_mode="timestep")
    mean = out["mean"].cpu().numpy()
    assert mean.shape == ref["mean"].shape == (wl["steps"][-1] * ctx.sizes[-1][0],)
    assert np.abs(mean - ref["mean"]).max() <= 1e-9 * np.abs(ref["mean"]).max()
    rv = ref["var"]
    assert np.abs(out["var"].cpu().numpy() - rv).max() <= 1e-9 * np.abs(rv).max()
    # V_l = (|D| T)^-1 int int s^2(Y_l): with both solutions within ~1e-10 of
    # the exact discrete ones (Newton tolerance on u = O(1)), Y_l moves by at
    # most ~2e-10 and V_l by ~4e-10 sqrt(V_l) -- which matters for the tiny
    # level corrections of the linear 1D problem
    V, Vr = np.asarray(out["V"]), np.asarray(ref["V"])
    assert np.all(np.abs(V - Vr) <= 4e-10 * np.sqrt(Vr) + 1e-8 * Vr + 1e-20), (V, Vr)
    lm = out["level_mean"].cpu().numpy()
    for l in range(3):
        assert np.abs(lm[l] - ref["level_mean"][l]).max() <= 1e-9 * np.abs(ref["mean"]).max()
    assert out["worst_status"] == 0
