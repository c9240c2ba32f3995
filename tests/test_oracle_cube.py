"""Pins of the oracle's version of the paper's own experiment (Sec. 4): the
isotropic additive field from a Gaussian-kernel pivoted Cholesky factor,
uniform coefficients, the Gaussian stimulus as initial state, and the FHN
current in units of u_peak.

Expected values come from the dense covariance matrix (exact reconstruction
at full rank, Weyl's bound on the truncated spectrum), brute-force enumeration
of the corners of [-1, 1]^M, the closed-form isotropic tensor, Green's formula
for the stiffness of a linear field, and the paper's printed parameters.
"""

import itertools

import numpy as np
import pytest

import stinputs
from oracle import api, fem, kl
from oracle.grid import Grid


def _points(n, seed, dim=3):
    return stinputs.uniform_field(n * dim, seed).reshape(n, dim)


# ---------------------------------------------------------------------------
# Pivoted Cholesky KL of the Gaussian kernel exp(-d^2 / sigma_KL)
# ---------------------------------------------------------------------------

def test_pivoted_cholesky_full_rank_reconstructs_covariance():
    """At rank N the factor reproduces the dense covariance matrix, and the
    rotated modes reproduce it as sum_k mode_k(x_i) mode_k(x_j)."""
    pts = _points(18, 5)
    b = kl.PivotedCholeskyKL(pts, 0.25, 18)
    C = np.exp(-((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1) / 0.25)
    np.testing.assert_allclose(b.L @ b.L.T, C, rtol=0, atol=1e-10)
    m = b.modes(pts)
    np.testing.assert_allclose(m @ m.T, C, rtol=0, atol=1e-9)
    assert abs(b.trace_error) < 1e-9
    # the eigenvalues of the full-rank factor are those of C
    np.testing.assert_allclose(b.lambdas, np.sort(np.linalg.eigvalsh(C))[::-1], rtol=1e-9, atol=1e-10)


def test_pivoted_cholesky_truncation_obeys_weyl_bound():
    """C - L L^T is positive semi-definite, so every eigenvalue of the rank-M
    approximation lies within trace(C - L L^T) of the matching eigenvalue of
    C; the trace error never grows with M."""
    g = Grid((6, 6, 6), (1.0, 1.0, 1.0))
    pts = g.nodes()
    C = np.exp(-((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1) / 0.25)
    ev = np.sort(np.linalg.eigvalsh(C))[::-1]
    prev = np.inf
    for M in (8, 20, 40, 66):
        b = kl.PivotedCholeskyKL(pts, 0.25, M)
        R = C - b.L @ b.L.T
        assert np.linalg.eigvalsh(R).min() > -1e-9
        np.testing.assert_allclose(b.trace_error, np.trace(R), rtol=1e-9)
        assert np.all(np.abs(ev[:M] - b.lambdas) <= b.trace_error + 1e-9)
        assert b.trace_error <= prev + 1e-12
        prev = b.trace_error


def test_mode_extension_reproduces_pivot_columns():
    """Away from the mesh, the low-rank covariance between a point and the
    pivots equals the kernel itself (the extension interpolates the pivot
    columns), and at the mesh points the extension equals the factor."""
    g = Grid((5, 5, 5), (1.0, 1.0, 1.0))
    b = kl.PivotedCholeskyKL(g.nodes(), 0.25, 30)
    x = _points(7, 9)
    mx = b.modes(x)
    mp = b.modes(b.pts[b.piv])
    kx = np.exp(-((x[:, None, :] - b.pts[b.piv][None, :, :]) ** 2).sum(-1) / 0.25)
    np.testing.assert_allclose(mx @ mp.T, kx, rtol=0, atol=1e-10)
    np.testing.assert_allclose(b.modes(b.pts), b.L @ b.Q, rtol=0, atol=1e-10)


def test_damping_keeps_every_corner_within_delta():
    """Brute force over all 2^M corners of [-1, 1]^M: the largest |g(x)| is
    s sum_k |mode_k(x)| and stays within delta; s is lowered only when the
    paper's s would break the bound."""
    g = Grid((3, 3, 3), (1.0, 1.0, 1.0))
    b = kl.PivotedCholeskyKL(g.nodes(), 0.25, 6)
    m = b.modes(b.pts)
    s = kl.damping(m, 0.3, 0.5)
    corners = np.array(list(itertools.product((-1.0, 1.0), repeat=6)))
    worst = np.abs(corners @ (s * m).T).max()
    assert worst <= 0.5 + 1e-12
    bound = np.abs(m).sum(axis=1).max()
    if 0.3 * bound > 0.5:
        np.testing.assert_allclose(worst, 0.5, rtol=1e-12)
    else:
        assert s == 0.3
    G = kl.synthesize_additive(s * m, corners, 2.0)
    assert G.min() >= 2.0 * (1 - 0.5) - 1e-12 and G.max() <= 2.0 * (1 + 0.5) + 1e-12


def test_additive_synthesis_is_affine_in_y():
    m = _points(4, 3, dim=5)
    y = _points(3, 4, dim=5) * 2 - 1
    G = kl.synthesize_additive(m, y, 0.7)
    for s in range(3):
        np.testing.assert_allclose(G[s], 0.7 * (1 + sum(m[:, k] * y[s, k] for k in range(5))), rtol=1e-14)


# ---------------------------------------------------------------------------
# Isotropic conductivity, Gaussian initial state, FHN scaling, inputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_relative_transverse_conductivity_gives_isotropic_tensor(dim):
    rng = np.random.default_rng(2)
    sigma = rng.uniform(0.5, 2.0, 7)
    theta = rng.uniform(-1.5, 1.5, 7)
    D = fem.diffusion_tensors(sigma, theta, 0.0, dim, tau_rel=1.0)
    np.testing.assert_allclose(D, sigma[:, None, None] * np.eye(dim)[None], rtol=0, atol=1e-15)
    # ratio r: along the fibre sigma, across it r sigma
    D = fem.diffusion_tensors(sigma, theta, 0.0, dim, tau_rel=0.25)
    a = fem.fiber_directions(theta, dim)
    np.testing.assert_allclose(np.einsum("eij,ej->ei", D, a), sigma[:, None] * a, rtol=1e-14)


def test_isotropic_stiffness_of_linear_field_is_boundary_flux():
    """Green's formula with D = sigma I: (K u)_i = int psi_i sigma grad u . n."""
    g = Grid((5, 4, 4), (1.0, 0.8, 0.6))
    sigma = 0.9
    D = fem.diffusion_tensors(np.full(g.n_el, sigma), np.zeros(g.n_el), 0.0, 3, tau_rel=1.0)
    K = fem.assemble_stiffness(g, D)
    p = np.array([0.4, -0.7, 0.25])
    u = g.nodes() @ p
    flux = sigma * p
    expect = np.zeros(g.n)
    nx, ny, nz = g.shape
    hx, hy, hz = g.h
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                idx = (k * ny + j) * nx + i
                w = [hx if 0 < i < nx - 1 else 0.5 * hx, hy if 0 < j < ny - 1 else 0.5 * hy,
                     hz if 0 < k < nz - 1 else 0.5 * hz]
                for ax, (ii, n_ax) in enumerate(((i, nx), (j, ny), (k, nz))):
                    face = np.prod([w[b] for b in range(3) if b != ax])
                    if ii == 0:
                        expect[idx] -= flux[ax] * face
                    if ii == n_ax - 1:
                        expect[idx] += flux[ax] * face
    np.testing.assert_allclose(K @ u, expect, rtol=0, atol=1e-13)


def test_gaussian_initial_state():
    wl = stinputs.workload("cube4_3d")
    g = api.level_grid(wl, 1)
    u0 = api.initial_state(wl, g)
    x = g.nodes()
    np.testing.assert_allclose(u0, np.exp(-(x ** 2).sum(1) / 0.25), rtol=1e-15)
    assert u0[0] == 1.0 and 0 < u0.min() < 1e-5


def test_fhn_current_in_units_of_u_peak():
    """-I_ion(u) / u_peak with u = u_peak v equals k v (v - a)(1 - v) for the
    paper's alpha = 1.4e-3, u_rest = 0, u_th = 28, u_peak = 115 (Sec. 4)."""
    wl = stinputs.workload("cube4_3d")
    v = np.linspace(-0.2, 1.2, 15)
    u = 115.0 * v
    i_ion = 1.4e-3 * (u - 0.0) * (u - 28.0) * (u - 115.0)
    from oracle.spacetime import reaction
    np.testing.assert_allclose(reaction(v, wl["k_react"], wl["a_react"]), -i_ion / 115.0, rtol=1e-13, atol=1e-13)


def test_cube_workload_is_the_papers_hierarchy():
    """Table 2: h = 0.2 ... 0.025, dt = 0.04 ... 0.005; sigma_KL 0.25, M = 66."""
    wl = stinputs.workload("cube4_3d")
    for l, (shape, m) in enumerate(zip(wl["levels"], wl["steps"])):
        g = api.level_grid(wl, l)
        np.testing.assert_allclose(g.h, [0.2 / 2 ** l] * 3, rtol=1e-15)
        np.testing.assert_allclose(wl["T"] / m, 0.04 / 2 ** l, rtol=1e-15)
    assert wl["n_modes"] == 66 and wl["sig_kl"] == 0.25


def test_uniform_coefficients_are_prefix_stable():
    a = stinputs.xi("cube4_3d", 2, 40, 66)
    b = stinputs.xi("cube4_3d", 2, 10, 66, start=30)
    np.testing.assert_array_equal(a[30:], b)
    assert a.min() >= -1.0 and a.max() <= 1.0 and abs(a.mean()) < 0.05


def test_cube_level0_sample_is_solved_and_activates_at_the_stimulus():
    """One coarse cube sample: Newton converges; nodes where the stimulus is
    at least the threshold activate at t = 0; the far corner stays at rest."""
    wl = stinputs.workload("cube4_3d")
    b = api.kl_basis(dict(wl, kl_grid=(11, 11, 11)))
    m0 = api.kl_modes(dict(wl, kl_grid=(11, 11, 11)), 0, b)
    y = stinputs.xi("cube4_3d", 0, 1, 66)
    sig = api.kl_synthesize(m0, y, wl["sigma_f0"], "additive")
    assert sig.min() > 0.5 * wl["sigma_f0"] and sig.max() < 1.5 * wl["sigma_f0"]
    U, st = api.st_solve(wl, 0, sig)
    assert st[0].converged
    t, cens = api.activation_map(wl, 0, U)
    g = api.level_grid(wl, 0)
    u0 = api.initial_state(wl, g)
    assert np.all(t[0][u0 >= 0.5] == 0.0)
    assert t[0][-1] == wl["T"] and abs(U[0, -1, -1]) < 1e-3


# ---------------------------------------------------------------------------
# The library's own mode construction (host input preparation) against the
# oracle's, written separately
# ---------------------------------------------------------------------------

def test_product_gaussian_modes_match_oracle_covariance():
    """Both rank-M factors approximate the same covariance matrix from below,
    so their low-rank covariances differ by at most the sum of the two trace
    errors (spectral norm, hence entrywise)."""
    from paper_1911_06066_amd import klmodes
    wl = stinputs.workload("cube4_3d", kl_grid=(7, 7, 7), n_modes=40, levels=[(7, 7, 7)], steps=[24])
    pb = klmodes.GaussLowRankBasis(wl["kl_grid"], wl["lengths"], wl["sig_kl"], wl["n_modes"])
    ob = api.kl_basis(wl)
    pts = ob.pts
    mp = pb.modes_at(pts)
    mo = ob.modes(pts)
    tol = pb.residual_trace + ob.trace_error
    assert np.abs(mp @ mp.T - mo @ mo.T).max() <= tol + 1e-9
    # centroids of the level: same damped modes
    mpl = klmodes.workload_modes(wl)[0]
    mol = api.kl_modes(wl, 0, ob)
    assert np.abs(mpl @ mpl.T - mol @ mol.T).max() <= 0.1 * tol + 1e-9


def test_product_exponential_modes_match_oracle():
    """Same Nystrom discretisation on both sides.  The square has degenerate
    eigenvalue pairs, whose eigenvectors are fixed only up to a rotation, so
    the truncated covariance sum_k mode_k(x) mode_k(y) is compared (8 modes
    end at a spectral gap)."""
    from paper_1911_06066_amd import klmodes
    wl = stinputs.workload("small_mc_2d", kl_grid=(17, 17), n_modes=8, levels=[(9, 9)], steps=[8])
    lam = api.kl_basis(wl).all_lambdas
    assert lam[7] - lam[8] > 1e-3 * lam[0]
    mp = klmodes.workload_modes(wl)[0]
    mo = api.kl_modes(wl, 0)
    np.testing.assert_allclose(mp @ mp.T, mo @ mo.T, rtol=0, atol=1e-10)


# ---------------------------------------------------------------------------
# Space-time prolongation (Sec. 3.4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_space_time_prolongation_is_exact_on_multilinear_fields(dim):
    """P_t (x) P_h reproduces fields that are multilinear in space and linear
    in time (the interpolants of such fields are exact); its t = 0 end is the
    fine initial state, which the test sets to the same field."""
    if dim == 2:
        wl = stinputs.workload("small_mc_2d", levels=[(5, 4), (9, 7)], steps=[3, 6], lengths=(1.0, 0.6))
    else:
        wl = stinputs.workload("slab3d", levels=[(3, 3, 3), (5, 5, 5)], steps=[4, 12])
    f = lambda x, t: 0.3 + 0.7 * x[:, 0] - 1.1 * x[:, 1] + 0.4 * x[:, 0] * x[:, 1] + t * (0.5 - 0.2 * x[:, 0]) \
        + (0.25 * x[:, -1] * x[:, 0] if dim == 3 else 0.0)
    gc, gf = api.level_grid(wl, 0), api.level_grid(wl, 1)
    mc, mf = wl["steps"]
    T = wl["T"]
    Uc = np.stack([f(gc.nodes(), (j + 1) * T / mc) for j in range(mc)])[None]
    import oracle.api as oa
    saved = oa.initial_state
    oa.initial_state = lambda w, g: f(g.nodes(), 0.0)
    try:
        Uf = oa.prolong_st(wl, 1, Uc)
    finally:
        oa.initial_state = saved
    expect = np.stack([f(gf.nodes(), (k + 1) * T / mf) for k in range(mf)])
    np.testing.assert_allclose(Uf[0], expect, rtol=0, atol=1e-13)


def test_space_time_prolongation_time_weights():
    """A field constant in space: fine level k is the linear interpolant in t
    of the coarse levels, with the initial state at t = 0 (ratio 2 and 3)."""
    for mc, mf in ((4, 8), (2, 6)):
        wl = stinputs.workload("small_mc_2d", levels=[(3, 3), (5, 5)], steps=[mc, mf], ic_radius=10.0)
        Uc = np.repeat(np.arange(1, mc + 1, dtype=float)[:, None] * 2.0, 9, axis=1)[None]
        Uf = api.prolong_st(wl, 1, Uc)[0]
        t = np.arange(1, mf + 1) * mc / mf  # fine times in coarse steps
        expect = np.interp(t, np.arange(mc + 1), np.concatenate([[1.0], 2.0 * np.arange(1, mc + 1)]))
        np.testing.assert_allclose(Uf[:, 0], expect, rtol=0, atol=1e-14)
        np.testing.assert_allclose(Uf, Uf[:, :1].repeat(25, axis=1), rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# Space-time QoI and the 1D+1 strip (Sec. 4.1)
# ---------------------------------------------------------------------------

def test_space_time_sample_is_exact_on_multilinear_fields():
    """A level's solution sampled from f(x, t) = (multilinear in x) + t (linear
    in x), with the level's initial state f(x, 0), maps onto the finest
    space-time grid as f itself."""
    wl = stinputs.workload("small_mc_2d", levels=[(5, 4), (9, 7), (17, 13)], steps=[3, 6, 12], lengths=(1.0, 0.6))
    f = lambda x, t: 0.3 + 0.7 * x[:, 0] - 1.1 * x[:, 1] + 0.4 * x[:, 0] * x[:, 1] + t * (0.5 - 0.2 * x[:, 0])
    T = wl["T"]
    import oracle.api as oa
    saved = oa.initial_state
    oa.initial_state = lambda w, g: f(g.nodes(), 0.0)
    try:
        gL = api.level_grid(wl, 2)
        expect = np.concatenate([f(gL.nodes(), (k + 1) * T / 12) for k in range(12)])
        for l in range(3):
            g = api.level_grid(wl, l)
            m = wl["steps"][l]
            U = np.stack([f(g.nodes(), (j + 1) * T / m) for j in range(m)])
            np.testing.assert_allclose(oa.space_time_sample(wl, l, U, 2), expect, rtol=0, atol=1e-13)
    finally:
        oa.initial_state = saved


def test_space_time_weights_integrate_in_time_and_space():
    wl = stinputs.workload("cable1d")
    w = api.space_time_weights(wl, 3)
    g = api.level_grid(wl, 3)
    dt = wl["T"] / wl["steps"][3]
    np.testing.assert_allclose(w.sum(), g.volume() * (wl["T"] - 0.5 * dt), rtol=1e-13)
    # linear in t over the time levels 1 .. m: trapezoid with the t = 0 value 0 is exact
    t = np.repeat(np.arange(1, wl["steps"][3] + 1) * dt, g.n)
    np.testing.assert_allclose(w @ t, g.volume() * wl["T"] ** 2 / 2, rtol=1e-13)


def test_strip_of_one_element_row_is_the_1d_problem():
    """On y-constant vectors the strip's Q1 mass and isotropic stiffness are
    (l_y / 2) times the 1D Q1 matrices (h/6 [2 1; 1 2], sigma/h [1 -1; -1 1])
    at each of the two node rows, so the strip solves the 1D equations."""
    wl = stinputs.workload("cable1d")
    g = api.level_grid(wl, 0)
    nx = g.shape[0]
    hx, ly = g.h[0], wl["lengths"][1]
    rng = np.random.default_rng(11)
    sigma = rng.uniform(0.5, 1.5, nx - 1)
    D = fem.diffusion_tensors(sigma, np.zeros(nx - 1), 0.0, 2, tau_rel=1.0)
    M = fem.assemble_mass(g).toarray()
    K = fem.assemble_stiffness(g, D).toarray()
    M1, K1 = np.zeros((nx, nx)), np.zeros((nx, nx))
    for e in range(nx - 1):
        M1[e:e + 2, e:e + 2] += hx / 6 * np.array([[2, 1], [1, 2]])
        K1[e:e + 2, e:e + 2] += sigma[e] / hx * np.array([[1, -1], [-1, 1]])
    v = rng.uniform(-1, 1, nx)
    vv = np.concatenate([v, v])
    for A, A1 in ((M, M1), (K, K1)):
        r = A @ vv
        ref = 0.5 * ly * (A1 @ v)
        tol = 1e-11 * np.abs(ref).max()  # rounding of sums with cancellation
        np.testing.assert_allclose(r[:nx], ref, rtol=0, atol=tol)
        np.testing.assert_allclose(r[nx:], r[:nx], rtol=0, atol=tol)


def test_strip_solution_does_not_depend_on_y():
    wl = stinputs.workload("cable1d")
    b = api.kl_basis(wl)
    m = api.kl_modes(wl, 1, b)
    sig = api.kl_synthesize(m, stinputs.xi("cable1d", 1, 1, 16), wl["sigma_f0"], "additive")
    U, st = api.st_solve(wl, 1, sig, mode="timestep")
    nx = wl["levels"][1][0]
    np.testing.assert_allclose(U[0][:, nx:], U[0][:, :nx], rtol=0, atol=1e-12)
    assert st[0].converged
