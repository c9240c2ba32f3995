"""Pins of the oracle's discretisation against closed forms and brute force.

None of these compares the oracle with itself: each expected value comes from
mathematics the paper fixes (exact discrete eigenvectors of the Q1 operators,
the scalar ODE the PDE reduces to, the Nagumo travelling-wave speed,
manufactured solutions, tensor-product and symmetry reductions, independent
brute-force assembly and root finding).
"""

import numpy as np
import pytest
import scipy.optimize

from oracle import fem, qoi, spacetime
from oracle.grid import Grid
from oracle.spacetime import STProblem

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def _prob(grid, m, T, u0, **kw):
    return STProblem(grid=grid, m=m, T=T, u0=u0, **kw)


# ---------------------------------------------------------------------------
# Linear operator + backward Euler: Neumann cosine modes are exact discrete
# eigenvectors of the Q1 pencil (K, M) with eigenvalue per axis
# (6 D / h^2)(1 - cos(pi h)) / (2 + cos(pi h)).
# ---------------------------------------------------------------------------

def _lam1d(D, h, L=1.0):
    c = np.cos(np.pi * h / L)
    return 6.0 * D / h ** 2 * (1.0 - c) / (2.0 + c)


@pytest.mark.parametrize("shape,lengths", [((17, 9), (1.0, 1.0)), ((9, 7, 5), (1.0, 1.0, 1.0))])
def test_cosine_mode_decays_exactly(shape, lengths):
    g = Grid(shape, lengths)
    x = g.nodes()
    u0 = np.prod(np.cos(np.pi * x / np.array(lengths)), axis=1)
    sigma_f0, ratio = 2e-2, 0.1
    prob = _prob(g, 8, 0.5, u0, k_react=0.0, sigma_f0=sigma_f0, transverse_ratio=ratio,
                 fiber_law="x")
    sigma = np.full(g.n_el, sigma_f0)
    U, st = spacetime.newton(prob, sigma)
    assert st.converged
    D = [sigma_f0] + [ratio * sigma_f0] * (g.dim - 1)  # fibres along x
    # axis a of length L_a: the mode cos(pi x / L_a) has angle pi h_a / L_a
    lam = sum(_lam1d(D[a], g.h[a], lengths[a]) for a in range(g.dim))
    for k in range(prob.m):
        expect = u0 * (1.0 + prob.dt * lam) ** (-(k + 1))
        np.testing.assert_allclose(U[k], expect, rtol=0, atol=1e-13)


# Crank-Nicolson (Sec. 3.2, eq. st-system: A = M + dt/2 K, B = -M + dt/2 K):
# on a cosine mode each step multiplies by (1 - dt lam / 2) / (1 + dt lam / 2).
@pytest.mark.parametrize("shape,lengths", [((17, 9), (1.0, 1.0)), ((9, 7, 5), (1.0, 1.0, 1.0))])
def test_crank_nicolson_cosine_mode_amplification(shape, lengths):
    g = Grid(shape, lengths)
    x = g.nodes()
    u0 = np.prod(np.cos(np.pi * x / np.array(lengths)), axis=1)
    sigma_f0, ratio = 2e-2, 0.1
    prob = _prob(g, 8, 0.5, u0, k_react=0.0, sigma_f0=sigma_f0, transverse_ratio=ratio, fiber_law="x", theta=0.5)
    sigma = np.full(g.n_el, sigma_f0)
    U, st = spacetime.newton(prob, sigma)
    assert st.converged
    D = [sigma_f0] + [ratio * sigma_f0] * (g.dim - 1)
    lam = sum(_lam1d(D[a], g.h[a], lengths[a]) for a in range(g.dim))
    amp = (1.0 - 0.5 * prob.dt * lam) / (1.0 + 0.5 * prob.dt * lam)
    for k in range(prob.m):
        np.testing.assert_allclose(U[k], u0 * amp ** (k + 1), rtol=0, atol=1e-13)


def test_crank_nicolson_is_second_order_in_time():
    """Against the semi-discrete solution exp(-lam t) u0 of a cosine mode: the
    time error falls by 4 per halving of dt (2 for backward Euler)."""
    g = Grid((17, 17), (1.0, 1.0))
    x = g.nodes()
    u0 = np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
    sigma_f0 = 5e-2
    lam = _lam1d(sigma_f0, g.h[0]) + _lam1d(0.1 * sigma_f0, g.h[1])
    T = 1.0
    errs = {}
    for th in (0.5, 1.0):
        errs[th] = []
        for m in (8, 16, 32):
            prob = _prob(g, m, T, u0, k_react=0.0, sigma_f0=sigma_f0, fiber_law="x", theta=th)
            U, _ = spacetime.newton(prob, np.full(g.n_el, sigma_f0))
            errs[th].append(np.abs(U[-1] - np.exp(-lam * T) * u0).max())
    r_cn = [errs[0.5][i] / errs[0.5][i + 1] for i in range(2)]
    r_be = [errs[1.0][i] / errs[1.0][i + 1] for i in range(2)]
    assert all(3.8 < r < 4.2 for r in r_cn), r_cn
    assert all(1.8 < r < 2.2 for r in r_be), r_be


# ---------------------------------------------------------------------------
# Stiffness on a linear field: (K u)_i equals the boundary flux integral
# int_{dD} psi_i (D grad u) . n ds (Green's formula, D constant).  Pins the
# full tensor including the off-diagonal entry and its sign.
# ---------------------------------------------------------------------------

def test_stiffness_of_linear_field_is_boundary_flux():
    g = Grid((6, 5), (1.0, 0.8))
    theta = 0.7
    sigma, tau = 1.3, 0.4
    D = fem.diffusion_tensors(np.full(g.n_el, sigma), np.full(g.n_el, theta), tau, 2)
    K = fem.assemble_stiffness(g, D)
    p = np.array([0.9, -0.35])
    u = g.nodes() @ p
    flux = D[0] @ p
    expect = np.zeros(g.n)
    nx, ny = g.shape
    hx, hy = g.h
    for j in range(ny):
        for i in range(nx):
            idx = j * nx + i
            wy = hy if 0 < j < ny - 1 else 0.5 * hy  # int of the hat along the edge
            wx = hx if 0 < i < nx - 1 else 0.5 * hx
            if i == 0:
                expect[idx] += -flux[0] * wy
            if i == nx - 1:
                expect[idx] += flux[0] * wy
            if j == 0:
                expect[idx] += -flux[1] * wx
            if j == ny - 1:
                expect[idx] += flux[1] * wx
    np.testing.assert_allclose(K @ u, expect, rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# Brute-force assembly: global hat functions integrated element by element
# with 5-point Gauss rules, written without the oracle's local-vertex tables.
# ---------------------------------------------------------------------------

def _hat(x, xi, h):
    return np.maximum(0.0, 1.0 - np.abs(x - xi) / h)


def _dhat(x, xi, h):
    inside = np.abs(x - xi) < h
    return np.where(inside, -np.sign(x - xi) / h, 0.0)


def _brute_force(g, D):
    d = g.dim
    xq, wq = np.polynomial.legendre.leggauss(5)
    nodes = g.nodes()
    M = np.zeros((g.n, g.n))
    K = np.zeros((g.n, g.n))
    cent = g.centroids()
    for e in range(g.n_el):
        lo = cent[e] - 0.5 * np.array(g.h)
        grids = np.meshgrid(*[lo[a] + 0.5 * g.h[a] * (xq + 1) for a in range(d)], indexing="ij")
        wts = np.ones_like(grids[0])
        for a in range(d):
            shape = [1] * d
            shape[a] = -1
            wts = wts * (0.5 * g.h[a] * wq).reshape(shape)
        pts = [gg.ravel() for gg in grids]
        w = wts.ravel()
        near = np.where(np.all(np.abs(nodes - cent[e]) < np.array(g.h) * 0.51 + 1e-12, axis=1))[0]
        phis, grads = {}, {}
        for i in near:
            vals = [_hat(pts[a], nodes[i, a], g.h[a]) for a in range(d)]
            ders = [_dhat(pts[a], nodes[i, a], g.h[a]) for a in range(d)]
            phis[i] = np.prod(vals, axis=0)
            grads[i] = np.array([np.prod([ders[b] if b == a else vals[b] for b in range(d)], axis=0)
                                 for a in range(d)])
        for i in near:
            for j in near:
                M[i, j] += np.sum(w * phis[i] * phis[j])
                K[i, j] += np.sum(w * np.einsum("aq,ab,bq->q", grads[i], D[e], grads[j]))
    return M, K


# ---------------------------------------------------------------------------
# Fibre laws.  For linear fields u = x_p, v = x_q the Q1 stiffness gives
# v^T K u = sum_e |e| (D_e)_qp exactly (their gradients are constant), and
# D_xx, D_yy, D_xy are (s + t)/2 +- (s - t)/2 cos 2 theta and (s - t)/2 sin 2 theta.
# With theta linear in one coordinate, the sum over element layers of
# h cos(a + b z_c) at the layer midpoints z_c equals the exact integral of
# cos(a + b z) divided by sinc(b h / 2) (the midpoint rule on a sinusoid),
# which fixes the law, the axis it varies along and the evaluation point
# (centroids, not nodes) in closed form.
# ---------------------------------------------------------------------------
def _layer_sums(a, b, length, h):
    """(sum h cos(a + b z_c), sum h sin(a + b z_c)) over the layers of [0, length]."""
    sinc = np.sin(b * h / 2) / (b * h / 2)
    c = (np.sin(a + b * length) - np.sin(a)) / b / sinc
    s = (np.cos(a) - np.cos(a + b * length)) / b / sinc
    return c, s


@pytest.mark.parametrize("law", ["diag2d", "rot3d", "x", "diag"])
def test_fiber_laws_pinned_by_linear_field_energies(law):
    dim = 2 if law == "diag2d" else 3
    if dim == 2:
        g = Grid((7, 5), (1.0, 0.8))
    else:
        g = Grid((5, 4, 7), (1.0, 0.9, 0.25))
    sigma, tau = 1.7, 0.3
    D = fem.diffusion_tensors(np.full(g.n_el, sigma), fem.fiber_angles(g, law), tau, dim)
    K = fem.assemble_stiffness(g, D)
    x = g.nodes()
    E = np.array([[x[:, q] @ (K @ x[:, p]) for p in range(dim)] for q in range(dim)])
    vol = float(np.prod(g.lengths))
    if law == "diag2d":  # 2 theta = pi/2 + y
        c, s = _layer_sums(np.pi / 2, 1.0, g.lengths[1], g.h[1])
        c, s = g.lengths[0] * c, g.lengths[0] * s
    elif law == "rot3d":  # 2 theta = -2 pi/3 + (4 pi/3) z / l_z
        c, s = _layer_sums(-2 * np.pi / 3, 4 * np.pi / (3 * g.lengths[2]), g.lengths[2], g.h[2])
        c, s = g.lengths[0] * g.lengths[1] * c, g.lengths[0] * g.lengths[1] * s
    elif law == "x":
        c, s = vol, 0.0
    else:  # theta = pi/4: cos 2 theta = 0, sin 2 theta = 1
        c, s = 0.0, vol
    want = np.zeros((dim, dim))
    want[0, 0] = 0.5 * (sigma + tau) * vol + 0.5 * (sigma - tau) * c
    want[1, 1] = 0.5 * (sigma + tau) * vol - 0.5 * (sigma - tau) * c
    want[0, 1] = want[1, 0] = 0.5 * (sigma - tau) * s
    if dim == 3:
        want[2, 2] = tau * vol
    np.testing.assert_allclose(E, want, rtol=0, atol=1e-12 * sigma * vol)


@pytest.mark.parametrize("shape", [(3, 3), (4, 3), (3, 3, 3)])
def test_assembly_matches_brute_force(shape):
    g = Grid(shape, (1.0, 0.7, 0.5)[: len(shape)])
    rng = np.random.default_rng(3)
    sigma = rng.uniform(0.5, 2.0, g.n_el)
    theta = rng.uniform(-1.5, 1.5, g.n_el)
    D = fem.diffusion_tensors(sigma, theta, 0.15, g.dim)
    Mb, Kb = _brute_force(g, D)
    np.testing.assert_allclose(fem.assemble_mass(g).toarray(), Mb, rtol=0, atol=1e-14)
    np.testing.assert_allclose(fem.assemble_stiffness(g, D).toarray(), Kb, rtol=0, atol=1e-13)


@pytest.mark.parametrize("scheme", ["backward_euler", "crank_nicolson"])
def test_newton_matches_generic_root_finder(scheme):
    """Full space-time Newton vs scipy.optimize.root on 36 unknowns, with the
    residual written from brute-force dense matrices: backward Euler, and the
    paper's Crank-Nicolson blocks A = M + dt/2 K, B = -M + dt/2 K with the
    reaction dt M I_ion(u) at the new level."""
    g = Grid((3, 3), (1.0, 1.0))
    rng = np.random.default_rng(5)
    sigma = rng.uniform(0.02, 0.2, g.n_el)
    u0 = rng.uniform(0.0, 1.0, g.n)
    cn = scheme == "crank_nicolson"
    prob = _prob(g, 4, 0.2, u0, fiber_law="diag2d", theta=0.5 if cn else 1.0)
    theta = fem.fiber_angles(g, "diag2d")
    Mb, Kb = _brute_force(g, fem.diffusion_tensors(sigma, theta, prob.tau, 2))
    dt = prob.dt
    A, B = Mb + 0.5 * dt * Kb, -Mb + 0.5 * dt * Kb

    def F(x):
        U = x.reshape(4, g.n)
        out = []
        prev = u0
        for k in range(4):
            f = 8.0 * U[k] * (U[k] - 0.1) * (1.0 - U[k])
            if cn:
                out.append(A @ U[k] + B @ prev - dt * Mb @ f)
            else:
                out.append(Mb @ (U[k] - prev) / dt + Kb @ U[k] - Mb @ f)
            prev = U[k]
        return np.concatenate(out)

    sol = scipy.optimize.root(F, np.tile(u0, 4), method="hybr", tol=1e-14)
    U, st = spacetime.newton(prob, sigma, mode="monolithic")
    assert st.converged
    np.testing.assert_allclose(U.ravel(), sol.x, rtol=0, atol=1e-12)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_three_solve_modes_agree(theta):
    g = Grid((9, 9), (1.0, 1.0))
    rng = np.random.default_rng(11)
    sigma = 1e-3 * np.exp(0.3 * rng.standard_normal(g.n_el))
    x = g.nodes()
    u0 = ((x ** 2).sum(1) <= 0.3 ** 2).astype(float)
    prob = _prob(g, 8, 1.0, u0, sigma_f0=1e-3, theta=theta)
    out = [spacetime.newton(prob, sigma, mode=mode)[0] for mode in ("monolithic", "block", "timestep")]
    np.testing.assert_allclose(out[0], out[1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(out[0], out[2], rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Spatially uniform state: K 1 = 0 and the nodal reaction keeps a constant
# state constant, so each step is the scalar backward-Euler equation
# (u_k - u_{k-1}) / dt = f(u_k).  Continuous crossing time of the logistic-type
# cubic by partial fractions.
# ---------------------------------------------------------------------------

def _be_scalar(prev, dt, k=8.0, a=0.1):
    g = lambda u: (u - prev) / dt - k * u * (u - a) * (1 - u)  # noqa: E731
    # bisection on a bracket around prev (g is increasing there for small dt)
    lo, hi = prev - 0.5, prev + 0.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def _t_cross(u, c0, k=8.0, a=0.1):
    return (1 / k) * (-(1 / a) * np.log(u / c0) + (1 / (a * (1 - a))) * np.log((u - a) / (c0 - a))
                      - (1 / (1 - a)) * np.log((1 - u) / (1 - c0)))


def test_uniform_state_is_scalar_ode():
    g = Grid((5, 4), (1.0, 1.0))
    c0 = 0.3
    m = 16
    prob = _prob(g, m, 1.0, np.full(g.n, c0))
    sigma = 1e-3 * np.exp(np.random.default_rng(2).standard_normal(g.n_el))
    U, st = spacetime.newton(prob, sigma)
    prev = c0
    for k in range(m):
        uk = _be_scalar(prev, prob.dt)
        np.testing.assert_allclose(U[k], uk, rtol=0, atol=1e-13)
        prev = uk


def test_uniform_state_crossing_time_converges_first_order():
    assert abs(_t_cross(0.5, 0.3) - 0.3709046428) < 1e-9
    errs = []
    for m in (32, 64, 128):
        g = Grid((3, 3), (1.0, 1.0))
        prob = _prob(g, m, 1.0, np.full(g.n, 0.3))
        U, _ = spacetime.newton(prob, np.full(g.n_el, 1e-3), mode="timestep")
        t, cens = qoi.activation_map(prob.u0, U, prob.dt)
        assert cens == 0
        errs.append(abs(t[0] - _t_cross(0.5, 0.3)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 0.85) and np.all(rates < 1.2), (errs, rates)


# ---------------------------------------------------------------------------
# Travelling front on a 1D cable: the Nagumo equation u_t = D u_xx + k u(u-a)(1-u)
# has fronts of speed c = sqrt(2 k D)(1/2 - a).
# ---------------------------------------------------------------------------

def _front_speed(cells, dt):
    g = Grid((cells + 1,), (1.0,))
    x = g.nodes()[:, 0]
    u0 = (x <= 0.1).astype(float)
    T = 8.0
    prob = _prob(g, int(round(T / dt)), T, u0, fiber_law="x", sigma_f0=1e-3)
    U, st = spacetime.newton(prob, np.full(g.n_el, 1e-3), mode="timestep")
    assert st.converged
    t, _ = qoi.activation_map(u0, U, prob.dt)
    sel = (x > 0.2) & (x < 0.45)
    slope = np.polyfit(x[sel], t[sel], 1)[0]
    return 1.0 / slope


@pytest.mark.slow
def test_cable_front_speed_first_order():
    c = np.sqrt(2 * 8.0 * 1e-3) * (0.5 - 0.1)
    e1 = abs(_front_speed(256, 1 / 64) / c - 1)
    e2 = abs(_front_speed(512, 1 / 128) / c - 1)
    assert e1 < 1.5e-2, e1
    assert 1.6 < e1 / e2 < 2.6, (e1, e2)


# ---------------------------------------------------------------------------
# Tensor-product reduction and symmetry.
# ---------------------------------------------------------------------------

def test_2d_with_fibres_along_x_equals_1d():
    nx = 33
    g1 = Grid((nx,), (1.0,))
    g2 = Grid((nx, 6), (1.0, 0.4))
    x1 = g1.nodes()[:, 0]
    u01 = (x1 <= 0.1).astype(float)
    u02 = np.tile(u01, 6)
    p1 = _prob(g1, 16, 1.0, u01, fiber_law="x", sigma_f0=3e-3)
    p2 = _prob(g2, 16, 1.0, u02, fiber_law="x", sigma_f0=3e-3)
    U1, _ = spacetime.newton(p1, np.full(g1.n_el, 3e-3))
    U2, _ = spacetime.newton(p2, np.full(g2.n_el, 3e-3))
    for j in range(6):
        np.testing.assert_allclose(U2[:, j * nx:(j + 1) * nx], U1, rtol=0, atol=1e-12)


def test_diagonal_fibres_give_transpose_symmetric_solution():
    n = 17
    g = Grid((n, n), (1.0, 1.0))
    x = g.nodes()
    u0 = ((x ** 2).sum(1) <= 0.3 ** 2).astype(float)
    prob = _prob(g, 12, 1.0, u0, fiber_law="diag", sigma_f0=4e-3)
    U, _ = spacetime.newton(prob, np.full(g.n_el, 4e-3))
    for k in range(prob.m):
        Z = U[k].reshape(n, n)
        np.testing.assert_allclose(Z, Z.T, rtol=0, atol=1e-12)
    t, _ = qoi.activation_map(u0, U, prob.dt)
    np.testing.assert_allclose(t.reshape(n, n), t.reshape(n, n).T, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Manufactured solutions: second order in h, first order in dt.
# ---------------------------------------------------------------------------

def _mms_error(n, m, spatial):
    g = Grid((n, n), (1.0, 1.0))
    x = g.nodes()
    Dxx, Dyy = 0.05, 0.005  # fibres along x, sigma = 0.05, transverse 0.1 sigma

    if spatial:  # linear in t: backward Euler has no time error
        def ustar(p, t):
            return 0.5 + 0.3 * np.cos(np.pi * p[:, 0]) * np.cos(np.pi * p[:, 1]) * (1 + t)

        def ut(p, t):
            return 0.3 * np.cos(np.pi * p[:, 0]) * np.cos(np.pi * p[:, 1])

        def lap(p, t):  # div(D grad u*)
            return -(Dxx + Dyy) * np.pi ** 2 * (ustar(p, t) - 0.5)
    else:  # constant in space: Q1 has no space error
        def ustar(p, t):
            return 0.5 + 0.25 * np.sin(2 * t) + 0.0 * p[:, 0]

        def ut(p, t):
            return 0.5 * np.cos(2 * t) + 0.0 * p[:, 0]

        def lap(p, t):
            return 0.0 * p[:, 0]

    def src(p, t):
        u = ustar(p, t)
        return ut(p, t) - lap(p, t) - 8.0 * u * (u - 0.1) * (1 - u)

    prob = _prob(g, m, 1.0, ustar(x, 0.0), fiber_law="x", sigma_f0=Dxx, source=src)
    U, st = spacetime.newton(prob, np.full(g.n_el, Dxx), mode="timestep")
    M = prob.mass()
    errs = [np.sqrt((U[k] - ustar(x, (k + 1) * prob.dt)) @ (M @ (U[k] - ustar(x, (k + 1) * prob.dt))))
            for k in range(m)]
    return max(errs)


@pytest.mark.slow
def test_mms_second_order_in_space():
    e = [_mms_error(n, 4, True) for n in (9, 17, 33)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(rates > 1.85) and np.all(rates < 2.2), (e, rates)


def test_mms_first_order_in_time():
    e = [_mms_error(5, m, False) for m in (16, 32, 64)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(rates > 0.9) and np.all(rates < 1.1), (e, rates)


# ---------------------------------------------------------------------------
# Activation map vs bisection of the piecewise-linear time interpolant.
# ---------------------------------------------------------------------------

def test_activation_map_matches_bisection():
    rng = np.random.default_rng(9)
    m, n, dt = 12, 40, 0.1
    u0 = rng.uniform(0, 0.6, n)
    U = np.cumsum(rng.uniform(-0.05, 0.12, (m, n)), axis=0) + u0
    t, cens = qoi.activation_map(u0, U, dt)
    series = np.vstack([u0, U])
    times = np.arange(m + 1) * dt
    count = 0
    for i in range(n):
        f = lambda s: np.interp(s, times, series[:, i]) - 0.5  # noqa: E731
        if series[0, i] >= 0.5:
            assert t[i] == 0.0
            continue
        first = np.argmax(series[:, i] >= 0.5) if np.any(series[:, i] >= 0.5) else None
        if first is None:
            assert t[i] == m * dt
            count += 1
            continue
        lo, hi = times[first - 1], times[first]
        for _ in range(100):
            mid = 0.5 * (lo + hi)
            if f(mid) >= 0:
                hi = mid
            else:
                lo = mid
        assert abs(t[i] - hi) < 1e-12
    assert cens == count
