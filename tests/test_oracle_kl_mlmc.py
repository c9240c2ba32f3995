"""Pins of the oracle's KL expansion, estimators and work model.

Expected values come from the closed-form eigenpairs of the 1D exponential
covariance, exact identities of the discretised covariance operator, the exact
MLMC telescoping sum, a mock solver with closed-form moments, and the numbers
printed in the paper (Table 2 Dof counts, Sec. 4.2.2 work forms).
"""

import os

import numpy as np
import pytest

from oracle import kl, mlmc, api
from oracle.grid import Grid, cube_hierarchy_level, space_time_dofs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# KL
# ---------------------------------------------------------------------------

def test_exp_kernel_1d_closed_form_golden():
    """Closed-form eigenvalues vs the stored values (computed from the same
    transcendental equations to 8 digits; ell 0.2, variance 0.1)."""
    lam, _ = kl.exp_kernel_1d_eigenpairs(0.2, 0.1, 8)
    gold = np.loadtxt(os.path.join(GOLDEN, "kl_exp1d_ell0.2_s0.1.txt"))
    np.testing.assert_allclose(lam, gold, rtol=2e-7)


def test_exp_kernel_closed_form_satisfies_integral_equation():
    """int C(x, y) phi(y) dy = lambda phi(x), checked by fine quadrature."""
    lam, funcs = kl.exp_kernel_1d_eigenpairs(0.2, 0.1, 5)
    y = np.linspace(0, 1, 20001)
    w = np.full(y.size, y[1] - y[0])
    w[0] = w[-1] = 0.5 * w[0]
    x = np.array([0.0, 0.13, 0.5, 0.77, 1.0])
    C = kl.exp_kernel(x[:, None], y[:, None], 0.2, 0.1)
    lhs = (C * w) @ funcs(y)
    np.testing.assert_allclose(lhs, funcs(x) * lam[None, :], atol=2e-8)
    # orthonormality of the closed-form functions
    G = funcs(y).T @ (w[:, None] * funcs(y))
    np.testing.assert_allclose(G, np.eye(5), atol=1e-8)


def test_nystrom_converges_second_order_to_closed_form():
    lam_exact, funcs = kl.exp_kernel_1d_eigenpairs(0.2, 0.1, 8)
    errs = []
    for n in (129, 513):
        b = kl.NystromKL(Grid((n,), (1.0,)), 0.2, 0.1, 8)
        errs.append(np.max(np.abs(b.lambdas / lam_exact - 1)))
        # eigenfunctions up to sign (1D eigenvalues are simple)
        x = np.linspace(0, 1, 101)[:, None]
        got = b.eigenfunctions(x)
        ref = funcs(x[:, 0])
        for k in range(4):
            s = np.sign(got[:, k] @ ref[:, k])
            assert np.max(np.abs(s * got[:, k] - ref[:, k])) < 5e-2 if n == 129 else 5e-3
    assert errs[1] < 2.5e-4, errs
    rate = np.log2(errs[0] / errs[1]) / 2  # grid spacing shrinks 4x
    assert 1.7 < rate < 2.3, (errs, rate)


def test_nystrom_invariants_2d():
    g = Grid((17, 13), (1.0, 0.7))
    b = kl.NystromKL(g, 0.2, 0.1, 30)
    # trace of the discrete operator = s2 |D| exactly (trapezoid weights)
    assert abs(b.all_lambdas.sum() - 0.1 * 0.7) < 1e-12
    # W-orthonormal eigenvectors
    G = b.psi_nodes.T @ (b.w[:, None] * b.psi_nodes)
    np.testing.assert_allclose(G, np.eye(30), atol=1e-12)
    # truncated pointwise variance below s2
    var = (b.psi_nodes ** 2 * b.lambdas[None, :]).sum(axis=1)
    assert np.all(var <= 0.1 + 1e-12)
    # Nystrom extension reproduces the nodal values at the nodes
    np.testing.assert_allclose(b.eigenfunctions(b.pts), b.psi_nodes, atol=1e-10)
    # eigenvalues descending and positive
    assert np.all(np.diff(b.lambdas) <= 1e-15) and b.lambdas[-1] > 0


def test_synthesized_field_log_variance():
    """Var[log(sigma / sigma_f0)] = sum lambda_k phi_k(x)^2 for xi ~ N(0, I)."""
    g = Grid((9, 9), (1.0, 1.0))
    b = kl.NystromKL(g, 0.2, 0.1, 10)
    pts = np.array([[0.1, 0.2], [0.5, 0.5], [0.9, 0.3]])
    modes = b.modes(pts)
    rng = np.random.default_rng(0)
    xi = rng.standard_normal((200000, 10))
    s = kl.synthesize_sigma(modes, xi, 2.0)
    emp = np.log(s / 2.0).var(axis=0)
    np.testing.assert_allclose(emp, (modes ** 2).sum(1), rtol=2e-2)


# ---------------------------------------------------------------------------
# Estimators
# ---------------------------------------------------------------------------

def test_welford_equals_two_pass_and_chan_merge_is_order_free():
    rng = np.random.default_rng(1)
    x = rng.normal(3.0, 2.0, (57, 11))
    w = mlmc.Welford(11)
    for row in x:
        w.push(row)
    mean, var = mlmc.two_pass(x)
    np.testing.assert_allclose(w.mean, mean, rtol=1e-13)
    np.testing.assert_allclose(w.variance(), var, rtol=1e-12)
    parts = [x[:13], x[13:40], x[40:]]
    states = []
    for p in parts:
        s = mlmc.Welford(11)
        for row in p:
            s.push(row)
        states.append(s)
    a = mlmc.Welford.merge(mlmc.Welford.merge(states[0], states[1]), states[2])
    b = mlmc.Welford.merge(states[2], mlmc.Welford.merge(states[1], states[0]))
    for s in (a, b):
        np.testing.assert_allclose(s.mean, mean, rtol=1e-13)
        np.testing.assert_allclose(s.variance(), var, rtol=1e-12)


def test_mlmc_telescopes_to_mc_on_finest_level():
    """Equal sample counts and shared inputs on every level: the MLMC mean and
    variance equal the plain MC mean and variance of the finest level."""
    rng = np.random.default_rng(4)
    N, n = 40, 25
    q = [rng.normal(size=(N, n)) * (l + 1) + l for l in range(4)]
    fine = q
    coarse = [None] + q[:-1]
    out = mlmc.mlmc_combine(fine, coarse, np.ones(n))
    mean, var = mlmc.two_pass(q[-1])
    np.testing.assert_allclose(out["mean"], mean, rtol=0, atol=1e-13)
    np.testing.assert_allclose(out["var"], var, rtol=0, atol=1e-12)


def test_mock_solver_mlmc_is_unbiased():
    """Q_l(xi) = c.xi + 2^-l d.(xi^2): E[Q_L] = 2^-L sum d."""
    rng = np.random.default_rng(8)
    M, L, n = 6, 3, 1
    c = rng.normal(size=M)
    d = rng.uniform(0.2, 1.0, size=M)
    N = [40000, 10000, 4000, 4000]

    def Q(l, xi):
        return (xi @ c + 2.0 ** -l * (xi ** 2) @ d)[:, None]

    fine, coarse = [], []
    for l in range(L + 1):
        xi = rng.standard_normal((N[l], M))
        fine.append(Q(l, xi))
        coarse.append(Q(l - 1, xi) if l > 0 else None)
    out = mlmc.mlmc_combine(fine, coarse, np.ones(n))
    exact = 2.0 ** -L * d.sum()
    var_l = [c @ c + 2 * d @ d] + [2 * d @ d * (2.0 ** -l - 2.0 ** -(l - 1)) ** 2
                                   for l in range(1, L + 1)]
    se = np.sqrt(sum(v / nl for v, nl in zip(var_l, N)))
    assert abs(out["mean"][0] - exact) < 4.5 * se
    for l in range(1, L + 1):  # per-level variance of Y_l, a closed form here
        assert abs(out["V"][l] / var_l[l] - 1) < 0.3


def test_interpolation_is_exact_for_multilinear_fields():
    coarse = Grid((5, 3), (1.0, 0.5))
    fine = Grid((17, 9), (1.0, 0.5))
    f = lambda p: 1.0 + 2 * p[:, 0] - 3 * p[:, 1] + 0.7 * p[:, 0] * p[:, 1]  # noqa: E731
    got = mlmc.interpolate(coarse, f(coarse.nodes()), fine)
    np.testing.assert_allclose(got, f(fine.nodes()), atol=1e-14)
    # injection at shared nodes
    g2 = Grid((9, 5), (1.0, 0.5))
    v = np.random.default_rng(0).normal(size=g2.n)
    out = mlmc.interpolate(g2, v, fine).reshape(9, 17)
    np.testing.assert_allclose(out[::2, ::2], v.reshape(5, 9), atol=1e-15)


def test_giles_allocation_meets_variance_budget():
    V = np.array([4.0, 1.0, 0.25, 0.06])
    C = np.array([1.0, 8.0, 64.0, 512.0])
    eps = 0.05
    N = mlmc.giles_allocation(V, C, eps)
    assert np.sum(V / N) <= eps ** 2 / 2 * (1 + 1e-12)
    # optimality: N_l proportional to sqrt(V_l / C_l)
    r = N / np.sqrt(V / C)
    assert np.max(r) / np.min(r) < 1.01


def test_small_mlmc_estimate_end_to_end_telescopes():
    """The oracle's full MLMC path with equal counts and shared inputs equals
    plain MC on the finest level (two tiny levels)."""
    wl = dict(dim=2, lengths=(1.0, 1.0), T=1.0, k_react=8.0, a_react=0.1, sigma_f0=1e-2,
              transverse_ratio=0.1, fiber_law="diag2d", ic_center=(0.0, 0.0), ic_radius=0.3,
              threshold=0.5, ell=0.2, s2=0.1, kl_grid=(9, 9), n_modes=4,
              levels=[(5, 5), (9, 9)], steps=[4, 8])
    b = api.kl_basis(wl)
    modes = [api.kl_modes(wl, l, b) for l in range(2)]
    rng = np.random.default_rng(2)
    xi = rng.standard_normal((5, 4))
    out = api.mlmc_estimate(wl, [5, 5], [xi, xi], modes)
    mean, var = mlmc.two_pass(out["fine_q"][1])
    np.testing.assert_allclose(out["mean"], mean, atol=1e-13)
    np.testing.assert_allclose(out["var"], var, atol=1e-13)


# ---------------------------------------------------------------------------
# Numbers printed in the paper
# ---------------------------------------------------------------------------

def test_cube_hierarchy_dofs_match_table_2():
    """Table 2 (cube): Dof's 5400 / 65'219 / 898'317 / 13'301'753, h 0.2 ... 0.025,
    dt 0.04 ... 0.005."""
    expect = [5400, 65219, 898317, 13301753]
    for l, e in enumerate(expect):
        g, m = cube_hierarchy_level(l)
        assert space_time_dofs(g, m) == e
        assert abs(g.h[0] - 0.2 / 2 ** l) < 1e-15
        assert abs(0.96 / m - 0.04 / 2 ** l) < 1e-15


def test_work_model_closed_forms():
    """Sec. 4.2.2: W_MC = 2^{(gd+4)L}; the MLMC sum equals the printed closed
    form when taken over the L coarse-to-fine terms l = 0..L-1 (the printed
    sum says l = 0..L, which would add one more 2^{gd L} term)."""
    for L in range(1, 6):
        # gd = 4 (cube): printed L 2^{4L}
        s = sum(2.0 ** (4 * l) * 2.0 ** (4 * (L - l)) for l in range(L))
        assert s == L * 2.0 ** (4 * L)
        assert mlmc.work_asymptotic_sum(4, L) == (L + 1) * 2.0 ** (4 * L)
        # gd = 2 (ventricle): closed form (2^{gd L} - 2^{4L}) / (2^{gd-4} - 1)
        s2 = sum(2.0 ** (2 * l) * 2.0 ** (4 * (L - l)) for l in range(L))
        closed = (2.0 ** (2 * L) - 2.0 ** (4 * L)) / (2.0 ** -2 - 1)
        assert abs(s2 - closed) < 1e-9 * closed
        # which is 4/3 (2^{4L} - 2^{2L}); the printed 3/4 factor is a slip
        assert abs(closed - 4.0 / 3.0 * (2.0 ** (4 * L) - 2.0 ** (2 * L))) < 1e-9 * closed
    # fixed-setting work of eq. work
    Wmc, Wml = mlmc.work_fixed_setting([1.0, 16.0, 256.0], [256, 16, 1])
    assert Wmc == 256.0 and Wml == 1.0 * 256 + 17.0 * 16 + 272.0 * 1
