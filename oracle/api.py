"""The four boundary calls, written plainly on top of the oracle modules.

Same names as the library boundary: kl_synthesize, st_solve, activation_map,
mlmc_estimate.  A workload is a plain dict (see the seeded-input module for the
keys); ``level`` indexes its list of grids.

Test infrastructure only (see the package docstring).
"""

import numpy as np

from . import kl, mlmc, qoi, spacetime
from .grid import Grid


def level_grid(wl, level):
    return Grid(wl["levels"][level], wl["lengths"])


def initial_state(wl, grid):
    """u0 = 1 inside the closed ball |x - c| <= r, else 0 (ic_kind 'ball'); or the
    Gaussian bump u0 = exp(-|x - c|^2 / r^2) (ic_kind 'gauss': the paper's
    stimulus shape of Sec. 4, in units of u_peak, taken as the initial state)."""
    x = grid.nodes()
    c = np.asarray(wl["ic_center"], dtype=np.float64)[: grid.dim]
    r = wl["ic_radius"]
    d2 = ((x - c) ** 2).sum(axis=1)
    if wl.get("ic_kind", "ball") == "gauss":
        return np.exp(-d2 / (r * r))
    return (d2 <= r * r).astype(np.float64)


def level_problem(wl, level, **kw):
    g = level_grid(wl, level)
    args = dict(
        grid=g, m=wl["steps"][level], T=wl["T"], u0=initial_state(wl, g),
        k_react=wl["k_react"], a_react=wl["a_react"], sigma_f0=wl["sigma_f0"],
        transverse_ratio=wl["transverse_ratio"], fiber_law=wl["fiber_law"], theta=wl.get("theta", 1.0),
        tau_relative=bool(wl.get("tau_relative", 0)),
    )
    args.update(kw)
    return spacetime.STProblem(**args)


def kl_basis(wl):
    """KL eigenpairs of the workload's covariance: Nystrom on its KL grid for
    the exponential kernel; for the Gaussian kernel, the rank-M pivoted
    Cholesky factor on the nodes of the KL grid (the finest mesh)."""
    g = Grid(wl["kl_grid"], wl["lengths"])
    if wl.get("kernel", "exp") == "gauss":
        return kl.PivotedCholeskyKL(g.nodes(), wl["sig_kl"], wl["n_modes"])
    return kl.NystromKL(g, wl["ell"], wl["s2"], wl["n_modes"])


def kl_damping(wl, basis):
    """The additive field's factor s (1 for the lognormal field)."""
    if wl.get("field", "lognormal") != "additive":
        return 1.0
    return kl.damping(basis.modes(basis.pts), wl["kl_s"], wl["kl_delta"])


def kl_modes(wl, level, basis=None):
    """modes[e, k] = sqrt(lambda_k) phi_k(x_e) at the level's element centroids
    (times the damping s for the additive field)."""
    basis = kl_basis(wl) if basis is None else basis
    return basis.modes(level_grid(wl, level).centroids()) * kl_damping(wl, basis)


def kl_synthesize(modes, xi, sigma_f0, field="lognormal"):
    if field == "additive":
        return kl.synthesize_additive(modes, xi, sigma_f0)
    return kl.synthesize_sigma(modes, xi, sigma_f0)


def st_solve(wl, level, sigma, u0_guess=None, mode="block", **kw):
    """Solve every sample; returns (U (S, m, n), list of NewtonStats)."""
    prob = level_problem(wl, level, **kw)
    sigma = np.atleast_2d(sigma)
    out = np.empty((sigma.shape[0], prob.m, prob.grid.n))
    stats = []
    for s in range(sigma.shape[0]):
        guess = None if u0_guess is None else u0_guess[s]
        out[s], st = spacetime.newton(prob, sigma[s], guess, mode=mode)
        stats.append(st)
    return out, stats


def activation_map(wl, level, U):
    """(t_act (S, n), n_censored per sample)."""
    prob = level_problem(wl, level)
    U = np.asarray(U)
    if U.ndim == 2:
        U = U[None]
    t = np.empty((U.shape[0], prob.grid.n))
    cens = []
    for s in range(U.shape[0]):
        t[s], c = qoi.activation_map(prob.u0, U[s], prob.dt, wl["threshold"])
        cens.append(c)
    return t, cens


def prolong_st(wl, level, U_coarse):
    """Space-time prolongation P_t (x) P_h of level-1 solutions to `level`
    (Sec. 3.4: tensor product of the spatial and the temporal transfer).

    Space: Q1 interpolation of the nested coarse grid at the fine nodes.  Time:
    the fine level at t = k dt_l is the linear interpolant, at that t, of the
    coarse levels at j dt_{l-1} and (j + 1) dt_{l-1} that bracket it; the
    coarse level at t = 0 is the fine grid's initial state.
    """
    gc, gf = level_grid(wl, level - 1), level_grid(wl, level)
    mc, mf = wl["steps"][level - 1], wl["steps"][level]
    T = wl["T"]
    U_coarse = np.atleast_3d(U_coarse)
    u0 = initial_state(wl, gf)
    out = np.empty((U_coarse.shape[0], mf, gf.n))
    for s in range(U_coarse.shape[0]):
        levels = [u0] + [mlmc.interpolate(gc, U_coarse[s, j], gf) for j in range(mc)]
        tc = np.arange(mc + 1) * (T / mc)
        for k in range(1, mf + 1):
            t = k * (T / mf)
            j = min(int(np.searchsorted(tc, t, side="right")) - 1, mc - 1)
            w = (t - tc[j]) / (tc[j + 1] - tc[j])
            if abs(w - 1.0) < 1e-12:  # t on the coarse level j + 1
                j, w = j + 1, 0.0
            if abs(w) < 1e-12:
                w = 0.0
            out[s, k - 1] = levels[j] if w == 0.0 else (1.0 - w) * levels[j] + w * levels[j + 1]
    return out


def space_time_sample(wl, level, U, finest_level):
    """A level's space-time solution U (m_l, n_l) on the finest space-time grid:
    at finest time level k (t = k dt_L, k = 1 .. m_L) the linear interpolant in
    t of the level's own time levels (level 0 its initial state), each
    interpolated in space (nested Q1) to the finest nodes; flattened [k][i]."""
    g, gL = level_grid(wl, level), level_grid(wl, finest_level)
    m, mL, T = wl["steps"][level], wl["steps"][finest_level], wl["T"]
    rows = [initial_state(wl, g)] + list(U)
    out = np.empty((mL, gL.n))
    for k in range(1, mL + 1):
        pos = k * m / mL  # in steps of the level
        j = int(np.floor(pos + 1e-12))
        w = pos - j
        if w < 1e-12:
            out[k - 1] = mlmc.interpolate(g, rows[j], gL)
        else:
            out[k - 1] = (1 - w) * mlmc.interpolate(g, rows[j], gL) + w * mlmc.interpolate(g, rows[j + 1], gL)
    return out.ravel()


def space_time_weights(wl, finest_level):
    """Quadrature of L^2(0, T; L^2(D)) on the finest time levels 1 .. m_L:
    lumped weights in space times the trapezoid rule in time (the t = 0
    level, the deterministic initial state, carries no variance)."""
    gL = level_grid(wl, finest_level)
    mL = wl["steps"][finest_level]
    dt = wl["T"] / mL
    wt = np.full(mL, dt)
    wt[-1] = 0.5 * dt
    return (wt[:, None] * gL.lumped_weights()[None, :]).ravel()


def mlmc_estimate(wl, N, xi_levels, modes_levels, solve_mode="block"):
    """MLMC mean/variance on the finest grid of the workload's QoI: the
    activation map (qoi 'activation', the default) or the space-time
    solution u on the finest space-time grid (qoi 'spacetime', the paper's
    E[u] of Sec. 4.1, with V_l in the L^2(0, T; L^2(D)) sense).

    N[l] samples on level l; xi_levels[l] (N[l], M) are the inputs shared by
    the fine (level l) and coarse (level l-1) member of each pair;
    modes_levels[l] the KL modes at level l's element centroids.
    """
    L1 = len(N)
    finest = level_grid(wl, L1 - 1)
    spacetime = wl.get("qoi", "activation") == "spacetime"
    weights = space_time_weights(wl, L1 - 1) if spacetime else finest.lumped_weights()
    vol = finest.volume() * wl["T"] if spacetime else None
    fine_q, coarse_q = [], []

    def level_qoi(lv, xi):
        sig = kl_synthesize(modes_levels[lv], xi, wl["sigma_f0"], wl.get("field", "lognormal"))
        U, _ = st_solve(wl, lv, sig, mode=solve_mode)
        if spacetime:
            return np.array([space_time_sample(wl, lv, Us, L1 - 1) for Us in U])
        t, _ = activation_map(wl, lv, U)
        g = level_grid(wl, lv)
        return np.array([mlmc.interpolate(g, ti, finest) for ti in t])

    for l in range(L1):
        xi = np.asarray(xi_levels[l])[: N[l]]
        fine_q.append(level_qoi(l, xi))
        coarse_q.append(level_qoi(l - 1, xi) if l > 0 else None)
    out = mlmc.mlmc_combine(fine_q, coarse_q, weights, vol)
    out["fine_q"] = fine_q
    out["coarse_q"] = coarse_q
    return out
