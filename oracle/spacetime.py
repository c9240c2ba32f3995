"""Nonlinear space-time system of the monodomain equation and Newton (oracle).

The paper discretises the monodomain equation (Sec. 2.1, eq. monodomain with
the cubic FitzHugh-Nagumo ionic current of eq. ionic_term) by Q1 in space and
a one-step scheme in time, and assembles all time steps into one block
lower-bidiagonal space-time system C u = f (Sec. 3.2, eq. system_C).  The
paper's scheme is Crank-Nicolson for the diffusion, diagonal blocks
A = M + dt/2 K and sub-diagonal blocks B = -M + dt/2 K (Sec. 3.2,
eq. st-system); the reaction enters as r(u) = dt (I (x) M_h) I_ion(u) with
nodal evaluation of the ionic current at the block row's own time level
(Sec. 3.3, eq. mono_disc), and the Jacobian is
J = C + dt (I_m (x) M_h) diag(I_ion'(u)).  With the reaction written as a
source f(u) = -I_ion(u) = k u (u - a)(1 - u), a weight theta of the new time
level in the diffusion term (theta = 1/2: the paper's Crank-Nicolson;
theta = 1: backward Euler, the workloads' default), and every block row
divided by dt, for k = 1..m

    R_k(U) = M (u_k - u_{k-1}) / dt + K (theta u_k + (1 - theta) u_{k-1})
             - M f(u_k) - b_k = 0,

with u_0 the initial state and b_k = theta l(t_k) + (1 - theta) l(t_{k-1})
the weighted load vector of an optional external source s(x, t) (used only
by manufactured-solution tests).  The Jacobian has diagonal blocks
A_k = M / dt + theta K - M diag f'(u_k) and sub-diagonal blocks
-M / dt + (1 - theta) K.  Newton's method (Sec. 3.5) solves the system; each linear solve is
done by sparse LU -- of the assembled space-time matrix, or block by block in
forward substitution (the same exact solve of a block lower-bidiagonal
matrix).  A time-stepping mode (Newton per slab) reaches the same discrete
solution and serves as an independent cross-check.

Test infrastructure only (see the package docstring).
"""

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


def reaction(u, k, a):
    """f(u) = k u (u - a)(1 - u)  (= -I_ion of the FHN cubic with rest 0, peak 1)."""
    return k * u * (u - a) * (1.0 - u)


def reaction_prime(u, k, a):
    """f'(u) = k (-3 u^2 + 2 (1 + a) u - a)."""
    return k * (-3.0 * u * u + 2.0 * (1.0 + a) * u - a)


@dataclass
class STProblem:
    """One level of the space-time monodomain problem.

    grid      : oracle.grid.Grid
    m         : number of backward-Euler steps on [0, T]
    T         : end time
    u0        : initial state at the nodes, shape (n,)
    fiber_law : see fem.fiber_angles
    source    : optional s(points (p, d), t) -> (p,) external source
    """

    grid: object
    m: int
    T: float
    u0: np.ndarray
    k_react: float = 8.0
    a_react: float = 0.1
    sigma_f0: float = 1e-3
    transverse_ratio: float = 0.1
    fiber_law: str = "diag2d"
    tau_relative: bool = False  # transverse conductivity transverse_ratio * sigma_e instead of * sigma_f0
    source: object = None
    newton_atol: float = 1e-12
    newton_max: int = 50
    theta: float = 1.0  # weight of the new time level in the diffusion term
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def dt(self):
        return self.T / self.m

    @property
    def tau(self):
        return 0.0 if self.tau_relative else self.transverse_ratio * self.sigma_f0

    @property
    def tau_rel(self):
        return self.transverse_ratio if self.tau_relative else 0.0

    def mass(self):
        if "M" not in self._cache:
            self._cache["M"] = fem.assemble_mass(self.grid)
        return self._cache["M"]

    def stiffness(self, sigma):
        theta = fem.fiber_angles(self.grid, self.fiber_law)
        D = fem.diffusion_tensors(sigma, theta, self.tau, self.grid.dim, self.tau_rel)
        return fem.assemble_stiffness(self.grid, D)

    def load(self, t, nq=3):
        """b_i = int s(x, t) psi_i(x) dx by tensor Gauss quadrature (nq per axis)."""
        if self.source is None:
            return np.zeros(self.grid.n)
        g = self.grid
        d = g.dim
        xq, wq = np.polynomial.legendre.leggauss(nq)
        en = g.element_nodes()
        lo = g.nodes()[en[:, 0]]  # lower corner of every element
        b = np.zeros(g.n)
        for qi in itertools.product(range(nq), repeat=d):
            s = np.array([0.5 * (xq[qi[a]] + 1.0) for a in range(d)])  # in [0,1]^d
            w = np.prod([0.5 * g.h[a] * wq[qi[a]] for a in range(d)])
            pts = lo + s[None, :] * np.array(g.h)[None, :]
            val = self.source(pts, t)
            for v in range(2 ** d):
                phi = np.prod([s[a] if (v >> a) & 1 else 1.0 - s[a] for a in range(d)])
                np.add.at(b, en[:, v], w * phi * val)
        return b


def source_term(prob, k):
    """b_k = theta l(t_k) + (1 - theta) l(t_{k-1}), 1-based slab index k."""
    th, dt = prob.theta, prob.dt
    b = th * prob.load(k * dt)
    if th != 1.0:
        b = b + (1.0 - th) * prob.load((k - 1) * dt)
    return b


def residual(prob, K, U):
    """R[k-1] = M (u_k - u_{k-1})/dt + K (theta u_k + (1 - theta) u_{k-1})
    - M f(u_k) - b_k, k = 1..m; U (m, n)."""
    M = prob.mass()
    dt, th = prob.dt, prob.theta
    R = np.empty_like(U)
    prev = prob.u0
    for k in range(prob.m):
        uk = U[k]
        R[k] = ((M @ (uk - prev)) / dt + K @ (th * uk + (1.0 - th) * prev)
                - M @ reaction(uk, prob.k_react, prob.a_react))
        if prob.source is not None:
            R[k] -= source_term(prob, k + 1)
        prev = uk
    return R


def slab_matrix(prob, K, uk):
    """A_k = M/dt + theta K - M diag f'(u_k)."""
    M = prob.mass()
    fp = reaction_prime(uk, prob.k_react, prob.a_react)
    return (M / prob.dt + prob.theta * K - M @ sp.diags(fp)).tocsc()


def sub_matrix(prob, K):
    """B = -M/dt + (1 - theta) K, the block coupling slab k to slab k-1."""
    return (-prob.mass() / prob.dt + (1.0 - prob.theta) * K).tocsc()


def jacobian(prob, K, U):
    """The assembled nm x nm block lower-bidiagonal space-time Jacobian."""
    M = prob.mass()
    m = prob.m
    blocks = [[None] * m for _ in range(m)]
    for k in range(m):
        blocks[k][k] = slab_matrix(prob, K, U[k])
        if k > 0:
            blocks[k][k - 1] = sub_matrix(prob, K)
    return sp.bmat(blocks, format="csc")


def _solve_block_forward(prob, K, U, R):
    """delta = -J^-1 R by forward substitution over the diagonal blocks."""
    B = sub_matrix(prob, K)
    delta = np.empty_like(U)
    prev = np.zeros(prob.grid.n)
    for k in range(prob.m):
        rhs = -R[k] - B @ prev
        delta[k] = spla.splu(slab_matrix(prob, K, U[k])).solve(rhs)
        prev = delta[k]
    return delta


def _solve_monolithic(prob, K, U, R):
    J = jacobian(prob, K, U)
    return spla.splu(J).solve(-R.ravel()).reshape(U.shape)


@dataclass
class NewtonStats:
    iterations: int = 0
    final_step: float = np.inf
    final_residual: float = np.inf
    converged: bool = False
    damped_steps: int = 0


def newton(prob, sigma, guess=None, mode="block"):
    """Newton on the whole space-time system; returns (U (m, n), NewtonStats).

    mode 'block'      : linear solves by exact block forward substitution
    mode 'monolithic' : linear solves by LU of the assembled space-time matrix
    mode 'timestep'   : Newton slab by slab (each slab to convergence)
    """
    K = prob.stiffness(sigma)
    if mode == "timestep":
        return _newton_timestep(prob, K, guess)
    U = np.tile(prob.u0, (prob.m, 1)) if guess is None else np.array(guess, dtype=np.float64)
    solve = _solve_block_forward if mode == "block" else _solve_monolithic
    st = NewtonStats()
    R = residual(prob, K, U)
    rnorm = np.abs(R).max()
    for it in range(prob.newton_max):
        delta = solve(prob, K, U, R)
        t = 1.0
        while True:  # halve the step while the residual grows (rarely needed)
            Un = U + t * delta
            Rn = residual(prob, K, Un)
            if np.abs(Rn).max() <= rnorm or t < 1e-3 or np.abs(t * delta).max() <= prob.newton_atol:
                break
            t *= 0.5
            st.damped_steps += 1
        U, R = Un, Rn
        rnorm = np.abs(R).max()
        st.iterations = it + 1
        st.final_step = float(np.abs(t * delta).max())
        st.final_residual = float(rnorm)
        if st.final_step <= prob.newton_atol:
            st.converged = True
            break
    return U, st


def _newton_timestep(prob, K, guess):
    M = prob.mass()
    dt, th = prob.dt, prob.theta
    U = np.empty((prob.m, prob.grid.n))
    st = NewtonStats(converged=True)
    prev = prob.u0
    for k in range(prob.m):
        uk = prev.copy() if guess is None else np.array(guess[k], dtype=np.float64)
        b = source_term(prob, k + 1) if prob.source is not None else 0.0
        for it in range(prob.newton_max):
            r = ((M @ (uk - prev)) / dt + K @ (th * uk + (1.0 - th) * prev)
                 - M @ reaction(uk, prob.k_react, prob.a_react) - b)
            d = spla.splu(slab_matrix(prob, K, uk)).solve(-r)
            uk = uk + d
            st.iterations = max(st.iterations, it + 1)
            if np.abs(d).max() <= prob.newton_atol:
                break
        else:
            st.converged = False
        U[k] = uk
        prev = uk
    R = residual(prob, K, U)
    st.final_residual = float(np.abs(R).max())
    st.final_step = 0.0
    return U, st
