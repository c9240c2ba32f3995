"""GPU checks at the workloads' full sizes.

The full-size space-time solves are too long for the oracle (about 80 s for
one 129^2 x 256-step sample on one core), so these tests compare what the
oracle can compute:

* causal prefixes: slabs 1..k of a space-time solution depend only on the
  slabs before them, so the oracle solves the first k steps (same dt) and the
  HIP path's full-horizon solution must agree there slab for slab;
* the fused MLMC launch against the statistics the oracle computes from the
  same samples solved one call at a time;
* the mixed path against the float64 path at full size;
* invariants that hold at any size (the adaptive sample counts against the
  oracle's allocation rule, activation times in [0, T]).

Launch configuration as in the benchmark: default block size, the committed
per-level smoother tuning, teams for the finest level.
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


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _tuning(wl):
    from paper_1911_06066_amd import autotune
    return autotune.level_tuning(wl, wl["precision"])


def _prefix_workload(wl, level, k):
    """The same problem on the first k steps of `level` (same dt)."""
    wp = dict(wl)
    wp["steps"] = list(wl["steps"])
    wp["T"] = wl["T"] * k / wl["steps"][level]
    wp["steps"][level] = k
    return wp


def _check_prefix(torch, dev, ctx, wl, level, k, xi, modes, tol_t=1e-9):
    sig_ref = oapi.kl_synthesize(modes, xi, wl["sigma_f0"])
    sig = ctx.kl_synthesize(level, torch.from_numpy(modes).to(dev), torch.from_numpy(xi).to(dev))
    assert _rel(sig.cpu().numpy(), sig_ref) < 1e-14
    u, stats = ctx.st_solve(level, sig)
    assert all(s["status"] == 0 for s in stats), stats
    solve_timings = ctx.timings()
    wp = _prefix_workload(wl, level, k)
    U_ref, _ = oapi.st_solve(wp, level, sig_ref, mode="timestep")
    up = u.cpu().numpy()[:, :k]
    assert _rel(up, U_ref) < 1e-9
    # activation times inside the prefix horizon agree; nodes the prefix leaves
    # censored activate at or after it
    t, _ = ctx.activation_map(level, u)
    t_ref, _ = oapi.activation_map(wp, level, U_ref)
    t = t.cpu().numpy()
    inside = t_ref < wp["T"]
    assert np.abs(t[inside] - t_ref[inside]).max() <= tol_t * wl["T"]
    assert np.all(t[~inside] >= wp["T"] - 1e-12)
    return u, solve_timings


@pytest.mark.parametrize("level,k,G", [(0, 64, 1), (1, 48, 1), (2, 32, 3)])
def test_mlmc3_2d_full_size_prefix_matches_oracle(torch_dev, level, k, G):
    """Each level of the benchmark workload at full size (33^2 x 64,
    65^2 x 128, 129^2 x 256 with a team of 3 workgroups), the first k slabs."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = stinputs.workload("mlmc3_2d")
    basis = oapi.kl_basis(wl)
    modes = oapi.kl_modes(wl, level, basis)
    xi = stinputs.xi("mlmc3_2d", level, 1, wl["n_modes"])
    ctx = Context(wl, level_tuning=_tuning(wl), team_size=G)
    _, tm = _check_prefix(torch, dev, ctx, wl, level, k, xi, modes)
    assert tm["solve_blocks"] == G


def test_mlmc3_2d_full_estimate_equals_statistics_of_solved_samples(torch_dev):
    """The benchmark's fused MLMC launch (all 672 pairs, teams, in-launch KL)
    against the oracle's statistics of the same samples solved level by level
    through the separate calls."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context, klmodes
    wl = stinputs.workload("mlmc3_2d")
    N = list(wl["samples"])
    M = wl["n_modes"]
    modes = [torch.from_numpy(m).to(dev) for m in klmodes.workload_modes(wl)]
    xi = [torch.from_numpy(stinputs.xi(wl["name"], l, N[l], M)).to(dev) for l in range(3)]
    ctx = Context(wl, level_tuning=_tuning(wl))
    out = ctx.mlmc_estimate(N, modes, xi)
    assert out["worst_status"] == 0 and out["N"] == N
    # the same samples through kl_synthesize / st_solve / activation_map
    grids = [oapi.level_grid(wl, l) for l in range(3)]
    fine_q, coarse_q = [], []
    for l in range(3):
        qs = []
        for lv in ([l, l - 1] if l > 0 else [l]):
            t_all = []
            for s0 in range(0, N[l], 128):
                sig = ctx.kl_synthesize(lv, modes[lv], xi[l][s0:s0 + 128].contiguous())
                u, st = ctx.st_solve(lv, sig, stats=False)
                t, _ = ctx.activation_map(lv, u)
                t_all.append(t.cpu().numpy())
                del u
            t_all = np.concatenate(t_all)
            qs.append(np.array([omlmc.interpolate(grids[lv], ti, grids[2]) for ti in t_all]))
        fine_q.append(qs[0])
        coarse_q.append(qs[1] if l > 0 else None)
    ref = omlmc.mlmc_combine(fine_q, coarse_q, grids[2].lumped_weights())
    T = wl["T"]
    assert np.abs(out["mean"].cpu().numpy() - ref["mean"]).max() <= 1e-9 * T
    var = out["var"].cpu().numpy()
    assert np.abs(var - ref["var"]).max() <= 1e-8 * np.abs(ref["var"]).max()
    np.testing.assert_allclose(out["V"], ref["V"], rtol=1e-7)


def test_mlmc4_2d_mixed_finest_level_full_size(torch_dev):
    """257^2 x 512 steps (the finest level of the four-level mixed workload):
    the mixed path within 1e-6 T of the float64 path on two samples; the
    float64 path matches the oracle on the first 4 slabs of the first."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = stinputs.workload("mlmc4_2d_mixed")
    level = 3
    basis = oapi.kl_basis(wl)
    modes = oapi.kl_modes(wl, level, basis)
    xi = stinputs.xi(wl["name"], level, 2, wl["n_modes"])
    mt, xt = torch.from_numpy(modes).to(dev), torch.from_numpy(xi).to(dev)
    c64 = Context(wl, precision="fp64")
    _check_prefix(torch, dev, c64, dict(wl, precision="fp64"), level, 4, xi[:1], modes)
    u64, st = c64.st_solve(level, c64.kl_synthesize(level, mt, xt))
    assert all(s["status"] == 0 for s in st)
    t64, _ = c64.activation_map(level, u64)
    del u64
    cmx = Context(wl, precision="mixed")
    sig = cmx.kl_synthesize(level, mt, xt)
    umx, st = cmx.st_solve(level, sig)
    assert all(s["status"] == 0 for s in st)
    tmx, _ = cmx.activation_map(level, umx)
    assert np.abs(tmx.cpu().numpy() - t64.cpu().numpy()).max() <= 1e-6 * wl["T"]
    tt = tmx.cpu().numpy()
    assert tt.min() >= 0.0 and tt.max() <= wl["T"]


def test_slab3d_full_size_mixed_matches_fp64(torch_dev):
    """The 3D slab at full size (65 x 65 x 17 nodes, 256 steps, 64 modes): the
    mixed path within 1e-6 T of the float64 path over the whole horizon.  (The
    oracle's sparse LU needs minutes per slab at this size; 3D parity with the
    oracle is checked at smaller sizes.)"""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = stinputs.workload("slab3d")
    basis = oapi.kl_basis(wl)
    modes = oapi.kl_modes(wl, 0, basis)
    xi = stinputs.xi(wl["name"], 0, 2, wl["n_modes"])
    mt, xt = torch.from_numpy(modes).to(dev), torch.from_numpy(xi).to(dev)
    c64 = Context(wl, precision="fp64")
    u64, st = c64.st_solve(0, c64.kl_synthesize(0, mt, xt))
    assert all(s["status"] == 0 for s in st)
    t64, cen = c64.activation_map(0, u64)
    del u64
    t = t64.cpu().numpy()
    assert t.min() >= 0.0 and t.max() <= wl["T"]
    g = oapi.level_grid(wl, 0)
    x = g.nodes() - np.asarray(wl["ic_center"])
    in_ball = (x * x).sum(axis=1) <= wl["ic_radius"] ** 2
    assert np.all(t[:, in_ball] == 0.0) and np.all(t[:, ~in_ball] > 0.0)
    cmx = Context(wl, precision="mixed")
    umx, st = cmx.st_solve(0, cmx.kl_synthesize(0, mt, xt))
    assert all(s["status"] == 0 for s in st)
    tmx, _ = cmx.activation_map(0, umx)
    assert np.abs(tmx.cpu().numpy() - t64.cpu().numpy()).max() <= 1e-6 * wl["T"]


def test_adaptive_sample_counts_follow_the_allocation_rule(torch_dev):
    """Adaptive MLMC (pilot, then rounds of the optimal allocation) on a
    reduced 3D hierarchy: at exit every level has at least the oracle's
    allocation for the final variances and costs (or its capacity), so the
    estimator variance sum V_l / N_l is within half the squared target."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context, klmodes
    wl = stinputs.workload("mlmc5_3d", levels=[(9, 9, 3), (17, 17, 5), (33, 33, 9)], steps=[8, 16, 32],
                           n_modes=16, kl_grid=(9, 9, 3))
    cap = [400, 200, 100]
    M = wl["n_modes"]
    modes = [torch.from_numpy(m).to(dev) for m in klmodes.workload_modes(wl)]
    xi = [torch.from_numpy(stinputs.xi(wl["name"], l, cap[l], M)).to(dev) for l in range(3)]
    ctx = Context(wl)
    eps = 4e-3 * wl["T"]
    out = ctx.mlmc_estimate(None, modes, xi, capacity=cap, target_rmse=eps, pilot=16)
    assert out["worst_status"] == 0
    assert out["rounds"] >= 1
    N, V, C = np.array(out["N"]), np.array(out["V"]), np.array(out["cost"])
    assert np.all(N >= 16) and np.all(V >= 0) and np.all(C > 0)
    want = omlmc.giles_allocation(V, C, eps)
    assert np.all((N >= want) | (N == np.array(cap))), (N, want)
    if np.all(N < np.array(cap)):
        assert np.sum(V / N) <= 0.5 * eps ** 2 * (1 + 1e-12)
    assert np.isfinite(out["bias_estimate"])
    # the level-0 mean averages interpolated activation times (in [0, T]); each
    # correction averages differences of two of them (in [-T, T]); the MLMC
    # mean is their sum (not a convex combination: it may leave [0, T])
    lm = out["level_mean"].cpu().numpy()
    T = wl["T"]
    assert lm[0].min() >= 0.0 and lm[0].max() <= T
    assert np.abs(lm[1:]).max() <= T
    assert np.abs(out["mean"].cpu().numpy() - lm.sum(axis=0)).max() <= 1e-12 * T


@pytest.mark.skip(reason="written for the earlier multi-grid kernel variant (coarse grids read from global "
                         "memory, the solver state in scratch memory), which faulted the GPU once (memory aperture "
                         "violation) with no cause shown; that variant was removed, and the V-cycle rebuilt on the "
                         "staged LDS passes is covered by tests/test_gpu_multigrid.py")
@pytest.mark.parametrize("dim", [2, 3])
def test_multigrid_vcycle_matches_oracle(torch_dev, dim):
    """The multigrid preconditioner (restriction, coarse operators from
    averaged tensors, prolongation, weighted-Jacobi and coarse sweeps): a
    deep V-cycle reaches the oracle solution."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    if dim == 2:
        wl = stinputs.workload("small_mc_2d", levels=[(33, 33)], steps=[24], n_modes=8, kl_grid=(17, 17),
                               ic_radius=0.25, sigma_f0=4e-3)
    else:
        wl = stinputs.workload("slab3d", levels=[(17, 17, 9)], steps=[8], n_modes=8, kl_grid=(9, 9, 3),
                               precision="fp64", ic_radius=0.3, sigma_f0=4e-3)
    basis = oapi.kl_basis(wl)
    modes = oapi.kl_modes(wl, 0, basis)
    xi = stinputs.xi(wl["name"], 0, 2, wl["n_modes"])
    sig = oapi.kl_synthesize(modes, xi, wl["sigma_f0"])
    ctx = Context(wl, mg_levels=-1, smoother=(0 if dim == 2 else 1), smooth_steps=2, coarse_sweeps=16)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    assert all(s["status"] == 0 for s in stats), stats
    U_ref, _ = oapi.st_solve(wl, 0, sig, mode="timestep")
    assert _rel(u.cpu().numpy(), U_ref) < 1e-9


def _read_prefix_golden(path):
    norms, sums, nodes, vals = {}, {}, [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            p = line.split()
            if p[0] == "norm2":
                norms[int(p[1])] = float(p[2])
            elif p[0] == "sum":
                sums[int(p[1])] = float(p[2])
            elif p[0] == "node":
                nodes.append(int(p[1]))
                vals.append([float(v) for v in p[2:]])
    return norms, sums, np.array(nodes), np.array(vals)


@pytest.mark.parametrize("precision,G", [("fp64", 16), ("mixed", 1), ("mixed", 16)])
def test_slab3d_full_size_prefix_matches_stored_oracle(torch_dev, precision, G):
    """The full 65 x 65 x 17 slab, 256 steps, rotating fibres: its first two
    slabs against the oracle's (tests/golden/slab3d_prefix2.txt, written by
    make_slab3d_prefix.py from the oracle alone; minutes of sparse LU per slab):
    the 2-norm and sum over all nodes and the values at 1.3k nodes around the
    stimulus and 300 others.  The solve takes the conductivity stored with
    them: the covariance's degenerate eigenpairs make modes computed on another
    machine a different, equally valid basis.  One workgroup per sample as in
    the slab workload, and a team of 16 as for the finest 3D MLMC levels."""
    import os
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    norms, sums, nodes, vals = _read_prefix_golden(os.path.join(gdir, "slab3d_prefix2.txt"))
    sig = np.load(os.path.join(gdir, "slab3d_prefix2_sigma.npy"))[None]
    wl = stinputs.workload("slab3d", precision=precision)
    ctx = Context(wl, level_tuning=_tuning(wl), team_size=G)
    u, stats = ctx.st_solve(0, torch.from_numpy(sig).to(dev))
    assert all(s["status"] == 0 for s in stats), stats
    assert ctx.timings()["solve_blocks"] == G
    up = u[0, :2].cpu().numpy()
    ctx.close()
    tol = 1e-9 if precision == "fp64" else 1e-8
    for k in (1, 2):
        assert abs(np.linalg.norm(up[k - 1]) - norms[k]) <= tol * norms[k]
        # the sum adds 71825 nodal errors of either sign: ten times the bound
        assert abs(up[k - 1].sum() - sums[k]) <= 10 * tol * abs(sums[k])
    assert _rel(up[:, nodes].T, vals) < tol


def test_slab3d_full_size_kl_synthesis_matches_oracle(torch_dev):
    """The float64 KL GEMM at the slab's full size (65536 elements, 64 modes)
    against the oracle's synthesis from the same modes."""
    torch, dev = torch_dev
    from paper_1911_06066_amd import Context
    wl = stinputs.workload("slab3d", precision="fp64")
    basis = oapi.kl_basis(wl)
    modes = oapi.kl_modes(wl, 0, basis)
    xi = stinputs.xi("slab3d", 0, 4, wl["n_modes"])
    with Context(wl) as ctx:
        sig = ctx.kl_synthesize(0, torch.from_numpy(modes).to(dev), torch.from_numpy(xi).to(dev))
    assert _rel(sig.cpu().numpy(), oapi.kl_synthesize(modes, xi, wl["sigma_f0"])) < 1e-14
