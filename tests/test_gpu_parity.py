"""GPU parity: the HIP path through the C interface vs the CPU oracle.

Sizes are chosen so the oracle finishes in seconds while the grids still span
several workgroup sweeps, multigrid levels and ragged tails.  Tolerances:
float64 path 1e-9 relative in u and in the activation map; mixed path
1e-6 T in activation time and 1e-4 relative in the MLMC variance.
"""

import numpy as np
import pytest

import oracle.api as oapi
from oracle import mlmc as omlmc
import stinputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _wl(**kw):
    base = dict(levels=[(17, 17)], steps=[16], n_modes=8, kl_grid=(17, 17), ic_radius=0.25, sigma_f0=4e-3)
    base.update(kw)
    return stinputs.workload("small_mc_2d", **base)


def _inputs(wl, S, seed_level=0):
    basis = oapi.kl_basis(wl)
    modes = [oapi.kl_modes(wl, l, basis) for l in range(len(wl["levels"]))]
    xi = stinputs.xi(wl["name"], seed_level, S, wl["n_modes"])
    return modes, xi


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# ---------------------------------------------------------------------------
# KL synthesis
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("S,shape,M", [(1, (5, 5), 3), (37, (33, 33), 16), (130, (17, 21), 64), (16, (9, 9), 128)])
def test_kl_synthesize_fp64(torch_dev, S, shape, M):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[shape], n_modes=M, kl_grid=(13, 13))
    modes, _ = _inputs(wl, 1)
    xi = stinputs.normal_field((S, M), seed=S + M)
    ctx = Context(wl)
    sig = ctx.kl_synthesize(0, torch.from_numpy(modes[0]).to(dev), torch.from_numpy(xi).to(dev))
    ref = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    assert _rel(sig.cpu().numpy(), ref) < 1e-14


@pytest.mark.parametrize("S,shape,M", [(37, (33, 33), 16), (130, (17, 21), 64), (5, (9, 9), 128)])
def test_kl_synthesize_split_fp16(torch_dev, S, shape, M):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[shape], n_modes=M, kl_grid=(13, 13))
    modes, _ = _inputs(wl, 1)
    xi = stinputs.normal_field((S, M), seed=S + 2 * M)
    ctx = Context(wl, precision="mixed")
    sig = ctx.kl_synthesize(0, torch.from_numpy(modes[0]).to(dev), torch.from_numpy(xi).to(dev))
    ref = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    err = np.abs(np.log(sig.cpu().numpy() / ref)).max()
    assert err < 1e-6, err


# ---------------------------------------------------------------------------
# space-time solve + activation map, float64
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,m,S", [((17, 17), 16, 3), ((33, 33), 24, 2), ((21, 13), 10, 2), ((5, 5), 4, 1)])
def test_st_solve_fp64_matches_oracle(torch_dev, shape, m, S):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[shape], steps=[m])
    modes, xi = _inputs(wl, S)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    ctx = Context(wl)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    U_ref, _ = oapi.st_solve(wl, 0, sig)
    assert all(s["status"] == 0 for s in stats), stats
    assert _rel(u.cpu().numpy(), U_ref) < 1e-9
    t, cen = ctx.activation_map(0, u)
    t_ref, cen_ref = oapi.activation_map(wl, 0, U_ref)
    assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-9 * wl["T"]
    assert list(cen) == list(cen_ref)


@pytest.mark.parametrize("sweeps", [1, 7, 9])
def test_odd_and_single_sweep_counts_match_oracle(torch_dev, sweeps):
    """The smoother's buffers alternate per sweep; any count leaves the
    preconditioned vector where GMRES reads it."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[(33, 33)], steps=[24])
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    ctx = Context(wl, level_tuning=[(sweeps, 10.0)])
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    assert all(s["status"] == 0 for s in stats), stats
    U_ref, _ = oapi.st_solve(wl, 0, sig, mode="timestep")
    assert _rel(u.cpu().numpy(), U_ref) < 1e-9


@pytest.mark.parametrize("precision,sweeps", [("fp64", 1), ("fp64", 2), ("fp64", 14), ("mixed", 9)])
def test_resident_smoother_matches_oracle(torch_dev, precision, sweeps):
    """One workgroup per sample on a grid that fits one tile: every sweep of
    the smoother runs in LDS within one pass."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[(33, 33)], steps=[24], precision=precision)
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    ctx = Context(wl, level_tuning=[(sweeps, 10.0)], team_size=1)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    assert all(s["status"] == 0 for s in stats), stats
    assert ctx.timings()["solve_blocks"] == 2
    U_ref, _ = oapi.st_solve(wl, 0, sig, mode="timestep")
    if precision == "fp64":
        assert _rel(u.cpu().numpy(), U_ref) < 1e-9
    else:
        t, _ = ctx.activation_map(0, u)
        t_ref, _ = oapi.activation_map(wl, 0, U_ref)
        assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-6 * wl["T"]


@pytest.mark.parametrize("precision,G", [("fp64", 1), ("fp64", 3), ("mixed", 1), ("mixed", 3)])
def test_fused_sweep_pairs_on_small_tiles_match_oracle(torch_dev, precision, G):
    """In 2D the smoother runs its sweeps in fused pairs, each tile with a
    two-row halo.  A 32 KiB staging budget cuts 33 rows into many tiles with a
    ragged last one, and teams of 3 put halo rows in the neighbouring bands."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[(33, 33)], steps=[24], precision=precision)
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    ctx = Context(wl, level_tuning=[(9, 10.0)], lds_kb=32, team_size=G)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    assert all(s["status"] == 0 for s in stats), stats
    U_ref, _ = oapi.st_solve(wl, 0, sig, mode="timestep")
    if precision == "fp64":
        assert _rel(u.cpu().numpy(), U_ref) < 1e-9
    else:
        t, _ = ctx.activation_map(0, u)
        t_ref, _ = oapi.activation_map(wl, 0, U_ref)
        assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-6 * wl["T"]


def test_st_solve_small_mc_workload_grid(torch_dev):
    """The 33^2 x 64-step grid of the single-level workload, 2 samples."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = stinputs.workload("small_mc_2d", kl_grid=(21, 21))
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    ctx = Context(wl)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    U_ref, _ = oapi.st_solve(wl, 0, sig, mode="timestep")
    assert _rel(u.cpu().numpy(), U_ref) < 1e-9
    t, cen = ctx.activation_map(0, u)
    t_ref, cen_ref = oapi.activation_map(wl, 0, U_ref)
    assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-9 * wl["T"]


def test_warm_start_and_explicit_guess_reach_same_solution(torch_dev):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl()
    modes, xi = _inputs(wl, 6)
    sig = torch.from_numpy(oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])).to(dev)
    a, _ = Context(wl, max_lanes=6).st_solve(0, sig)          # one sample per lane
    b, sb = Context(wl, max_lanes=2).st_solve(0, sig)         # lanes reuse previous samples
    c, _ = Context(wl, max_lanes=6).st_solve(0, sig, u0_guess=a.flip(0).contiguous())
    assert _rel(b.cpu().numpy(), a.cpu().numpy()) < 1e-10
    assert _rel(c.cpu().numpy(), a.cpu().numpy()) < 1e-10


@pytest.mark.parametrize("dim,G", [(2, 2), (2, 4), (2, 8), (2, 11), (3, 2), (3, 4), (3, 5)])
def test_multi_workgroup_teams_match_oracle(torch_dev, dim, G):
    """Samples split over G workgroups (row bands, team barriers, rank-ordered
    reductions) reach the oracle solution; G = 11 on 33 rows and G = 5 on 17
    rows give the narrowest bands allowed, 3 rows per member."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    if dim == 2:
        wl = _wl(levels=[(33, 33)], steps=[24])
    else:
        wl = stinputs.workload("slab3d", levels=[(17, 17, 5)], steps=[6], n_modes=8, kl_grid=(9, 9, 3),
                               precision="fp64", ic_radius=0.3, sigma_f0=4e-3)
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    ctx = Context(wl, team_size=G)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    assert all(s["status"] == 0 for s in stats), stats
    assert ctx.timings()["solve_blocks"] == G * ctx.timings()["solve_teams"]
    U_ref, _ = oapi.st_solve(wl, 0, sig)
    assert _rel(u.cpu().numpy(), U_ref) < 1e-9


def test_nonconvergence_is_reported_not_hidden(torch_dev):
    """One backward-Euler step over the whole horizon (dt = T) makes the slab
    operator indefinite; the solver stops at its Newton limit and says so."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context, StmError
    wl = _wl(levels=[(17, 17)], steps=[1])
    modes, xi = _inputs(wl, 1)
    sig = torch.from_numpy(oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])).to(dev)
    ctx = Context(wl, newton_max=5)
    with pytest.raises(StmError) as e:
        ctx.st_solve(0, sig)
    assert e.value.code == "STM_E_NOT_CONVERGED"


@pytest.mark.parametrize("shape,m,precision", [((17, 17), 8, "fp64"), ((17, 17), 4, "fp64"), ((33, 33), 8, "fp64"),
                                               ((33, 33), 8, "mixed"), ((17, 17), 4, "mixed")])
def test_large_time_steps_converge_like_the_oracle(torch_dev, shape, m, precision):
    """dt = T/8 and T/4: the slab Newton takes large steps from the previous
    slab (halved while the residual grows, as the oracle's) and reaches the
    oracle's solution, which converges there."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[shape], steps=[m], precision=precision)
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    U_ref, st_ref = oapi.st_solve(wl, 0, sig, mode="timestep")
    assert all(s.converged for s in st_ref)
    ctx = Context(wl)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    assert all(s["status"] == 0 for s in stats), stats
    t, _ = ctx.activation_map(0, u)
    t_ref, _ = oapi.activation_map(wl, 0, U_ref)
    if precision == "fp64":
        assert _rel(u.cpu().numpy(), U_ref) < 1e-9
        assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-9 * wl["T"]
    else:
        assert _rel(u.cpu().numpy(), U_ref) < 1e-8
        assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-6 * wl["T"]


def test_activation_map_kernel_vs_oracle_on_synthetic_series(torch_dev):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[(9, 7)], steps=[12])
    n, m = 63, 12
    rng = np.random.default_rng(4)
    U = np.cumsum(rng.uniform(-0.05, 0.12, (3, m, n)), axis=1)
    ctx = Context(wl)
    t, cen = ctx.activation_map(0, torch.from_numpy(U).to(dev))
    t_ref, cen_ref = oapi.activation_map(wl, 0, U)
    assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-12
    assert list(cen) == list(cen_ref)


# ---------------------------------------------------------------------------
# 3D
# ---------------------------------------------------------------------------

def test_st_solve_3d_fp64_matches_oracle(torch_dev):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = stinputs.workload("slab3d", levels=[(9, 9, 5)], steps=[8], n_modes=8, kl_grid=(9, 9, 3),
                           precision="fp64", ic_radius=0.3, sigma_f0=4e-3)
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    ctx = Context(wl)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    U_ref, _ = oapi.st_solve(wl, 0, sig)
    assert _rel(u.cpu().numpy(), U_ref) < 1e-9
    t, cen = ctx.activation_map(0, u)
    t_ref, _ = oapi.activation_map(wl, 0, U_ref)
    assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-9 * wl["T"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_theta_not_a_power_of_two_3d_matches_oracle(torch_dev, precision):
    """theta = 0.75: the 3D passes fold the stiffness scale (theta, 1 - theta)
    into the element factors instead of scaling the vertex values, which is
    exact only for powers of two; any other theta must still give the
    theta-scheme's discrete solution (a team of 3 by planes, rot3d fibres)."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = stinputs.workload("slab3d", levels=[(9, 9, 17)], steps=[6], n_modes=8, kl_grid=(9, 9, 3),
                           precision=precision, ic_radius=0.3, sigma_f0=4e-3, theta=0.75)
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    with Context(wl, team_size=3) as ctx:
        u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
        assert all(s["status"] == 0 for s in stats), stats
    U_ref, _ = oapi.st_solve(wl, 0, sig, mode="timestep")
    assert _rel(u.cpu().numpy(), U_ref) < (1e-9 if precision == "fp64" else 1e-8)
    U_be, _ = oapi.st_solve(dict(wl, theta=1.0), 0, sig, mode="timestep")
    assert _rel(U_be, U_ref) > 1e-6  # theta matters at this size


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_plane_group_teams_match_oracle(torch_dev, precision):
    """A team of 3 on 9 x 9 x 17 nodes splits its members by planes (three
    groups of 5-6 planes over all 9 rows, each pass starting with a step on
    the layer below the group): members read their neighbours' halo planes,
    and every z-march starts away from plane 0 (rot3d fibre rows per layer)."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = stinputs.workload("slab3d", levels=[(9, 9, 17)], steps=[6], n_modes=8, kl_grid=(9, 9, 3),
                           precision=precision, ic_radius=0.3, sigma_f0=4e-3)
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    with Context(wl, team_size=3) as ctx:
        u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
        assert all(s["status"] == 0 for s in stats), stats
        assert ctx.timings()["solve_blocks"] == 3 * ctx.timings()["solve_teams"]
        U_ref, _ = oapi.st_solve(wl, 0, sig, mode="timestep")
        assert _rel(u.cpu().numpy(), U_ref) < (1e-9 if precision == "fp64" else 1e-8)


@pytest.mark.parametrize("shape,precision,G", [((9, 9, 9), "fp64", 1), ((9, 9, 9), "mixed", 3),
                                               ((17, 17, 9), "fp64", 1), ((17, 17, 9), "fp64", 3),
                                               ((17, 17, 9), "mixed", 1), ((17, 17, 9), "mixed", 3)])
def test_rot3d_fibres_on_many_tiles_match_oracle(torch_dev, shape, precision, G):
    """The fibre angle changes with every element layer (rot3d), and a 3D pass
    reads the layer's fibre row at every plane it marches through.  A 16 KiB
    staging budget cuts the rows into several tiles (each marching through all
    planes from its own prologue), for every staged pass (2, 3 and 4 fields);
    teams of 3 add row bands."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = stinputs.workload("slab3d", levels=[shape], steps=[6], n_modes=8, kl_grid=(9, 9, 3),
                           precision=precision, ic_radius=0.3, sigma_f0=4e-3)
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    ctx = Context(wl, lds_kb=16, team_size=G)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    assert all(s["status"] == 0 for s in stats), stats
    assert ctx.timings()["solve_blocks"] == G * ctx.timings()["solve_teams"]
    U_ref, _ = oapi.st_solve(wl, 0, sig, mode="timestep")
    t, _ = ctx.activation_map(0, u)
    t_ref, _ = oapi.activation_map(wl, 0, U_ref)
    if precision == "fp64":
        assert _rel(u.cpu().numpy(), U_ref) < 1e-9
        assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-9 * wl["T"]
    else:
        assert _rel(u.cpu().numpy(), U_ref) < 1e-8
        assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-6 * wl["T"]
    # the law matters at this size: fibres along x give a different solution
    U_x, _ = oapi.st_solve(dict(wl, fiber_law="x"), 0, sig, mode="timestep")
    assert _rel(U_x, U_ref) > 1e-6


# ---------------------------------------------------------------------------
# Crank-Nicolson (the paper's time scheme)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim,precision,G", [(2, "fp64", 1), (2, "fp64", 3), (3, "fp64", 1), (2, "mixed", 1)])
def test_crank_nicolson_matches_oracle(torch_dev, dim, precision, G):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    if dim == 2:
        wl = _wl(levels=[(33, 33)], steps=[24], theta=0.5, precision=precision)
    else:
        wl = stinputs.workload("slab3d", levels=[(9, 9, 5)], steps=[8], n_modes=8, kl_grid=(9, 9, 3),
                               precision=precision, ic_radius=0.3, sigma_f0=4e-3, theta=0.5)
    modes, xi = _inputs(wl, 2)
    sig = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    ctx = Context(wl, team_size=G)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    assert all(s["status"] == 0 for s in stats), stats
    U_ref, _ = oapi.st_solve(wl, 0, sig, mode="timestep")
    t, _ = ctx.activation_map(0, u)
    t_ref, _ = oapi.activation_map(wl, 0, U_ref)
    if precision == "fp64":
        assert _rel(u.cpu().numpy(), U_ref) < 1e-9
        assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-9 * wl["T"]
    else:
        assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-6 * wl["T"]
    # the scheme matters: backward Euler gives a measurably different solution
    U_be, _ = oapi.st_solve(dict(wl, theta=1.0), 0, sig, mode="timestep")
    assert _rel(U_be, U_ref) > 1e-6


def test_crank_nicolson_mlmc_matches_oracle(torch_dev):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl, N, modes, xi = _mlmc_case("fp64")
    wl = dict(wl, theta=0.5)
    ctx = Context(wl)
    out = ctx.mlmc_estimate(N, [torch.from_numpy(m).to(dev) for m in modes],
                            [torch.from_numpy(x).to(dev) for x in xi])
    ref = oapi.mlmc_estimate(wl, N, xi, modes, solve_mode="timestep")
    assert np.abs(out["mean"].cpu().numpy() - ref["mean"]).max() <= 1e-9 * wl["T"]
    np.testing.assert_allclose(out["V"], ref["V"], rtol=1e-8, atol=1e-15)


# ---------------------------------------------------------------------------
# mixed precision
# ---------------------------------------------------------------------------

def test_st_solve_mixed_activation_within_tolerance(torch_dev):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[(33, 33)], steps=[32])
    modes, xi = _inputs(wl, 3)
    ctx = Context(wl, precision="mixed")
    sig = ctx.kl_synthesize(0, torch.from_numpy(modes[0]).to(dev), torch.from_numpy(xi).to(dev))
    u, stats = ctx.st_solve(0, sig)
    t, cen = ctx.activation_map(0, u)
    sig_ref = oapi.kl_synthesize(modes[0], xi, wl["sigma_f0"])
    U_ref, _ = oapi.st_solve(wl, 0, sig_ref, mode="timestep")
    t_ref, _ = oapi.activation_map(wl, 0, U_ref)
    assert np.abs(t.cpu().numpy() - t_ref).max() <= 1e-6 * wl["T"]


# ---------------------------------------------------------------------------
# MLMC estimator
# ---------------------------------------------------------------------------

def _mlmc_case(precision):
    wl = stinputs.workload("mlmc3_2d", levels=[(9, 9), (17, 17), (33, 33)], steps=[8, 16, 32], n_modes=8,
                           kl_grid=(17, 17), ic_radius=0.25, sigma_f0=4e-3, precision=precision)
    N = [12, 6, 3]
    basis = oapi.kl_basis(wl)
    modes = [oapi.kl_modes(wl, l, basis) for l in range(3)]
    xi = [stinputs.xi("mlmc3_2d", l, N[l], wl["n_modes"]) for l in range(3)]
    return wl, N, modes, xi


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mlmc_estimate_matches_oracle(torch_dev, precision):
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl, N, modes, xi = _mlmc_case(precision)
    ctx = Context(wl)
    out = ctx.mlmc_estimate(N, [torch.from_numpy(m).to(dev) for m in modes],
                            [torch.from_numpy(x).to(dev) for x in xi])
    ref = oapi.mlmc_estimate(wl, N, xi, modes, solve_mode="timestep")
    T = wl["T"]
    mean = out["mean"].cpu().numpy()
    var = out["var"].cpu().numpy()
    if precision == "fp64":
        assert np.abs(mean - ref["mean"]).max() <= 1e-9 * T
        assert np.abs(var - ref["var"]).max() <= 1e-9 * max(np.abs(ref["var"]).max(), 1e-12)
        np.testing.assert_allclose(out["V"], ref["V"], rtol=1e-8, atol=1e-15)
    else:
        assert np.abs(mean - ref["mean"]).max() <= 1e-6 * T
        scale = np.linalg.norm(ref["var"])
        assert np.linalg.norm(var - ref["var"]) <= 1e-4 * scale
    assert out["N"] == N
    # level fields
    lm = out["level_mean"].cpu().numpy()
    for l in range(3):
        assert np.abs(lm[l] - ref["level_mean"][l]).max() <= (1e-9 if precision == "fp64" else 1e-6) * T


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mlmc_with_split_finest_group_matches_oracle(torch_dev, precision):
    """With at least 8 pairs on the finest level, its fine members are split
    by predicted cost into two groups solved through a sample order list;
    the estimate still matches the oracle's statistics sample by sample."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = _wl(levels=[(9, 9), (17, 17)], steps=[8, 16], n_modes=8, precision=precision)
    N = [10, 12]
    basis = oapi.kl_basis(wl)
    modes = [oapi.kl_modes(wl, l, basis) for l in range(2)]
    xi = [stinputs.xi(wl["name"], l, N[l], wl["n_modes"]) for l in range(2)]
    ctx = Context(wl)
    for _ in range(2):  # the second call prices the hard part from the first call's measurement
        out = ctx.mlmc_estimate(N, [torch.from_numpy(m).to(dev) for m in modes],
                                [torch.from_numpy(x).to(dev) for x in xi])
    ref = oapi.mlmc_estimate(wl, N, xi, modes, solve_mode="timestep")
    T = wl["T"]
    if precision == "fp64":
        assert np.abs(out["mean"].cpu().numpy() - ref["mean"]).max() <= 1e-9 * T
        assert np.abs(out["var"].cpu().numpy() - ref["var"]).max() <= 1e-9 * max(np.abs(ref["var"]).max(), 1e-12)
        np.testing.assert_allclose(out["V"], ref["V"], rtol=1e-8, atol=1e-15)
    else:
        assert np.abs(out["mean"].cpu().numpy() - ref["mean"]).max() <= 1e-6 * T
        assert np.linalg.norm(out["var"].cpu().numpy() - ref["var"]) <= 1e-4 * np.linalg.norm(ref["var"])
    assert out["N"] == N and out["worst_status"] == 0
