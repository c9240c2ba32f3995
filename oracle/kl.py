"""Truncated Karhunen-Loeve expansion of the fibre conductivity (oracle).

Sec. 2.2 of the paper writes the random conductivity as a truncated KL
expansion (eq. KL-expansion): eigenpairs (lambda_k, phi_k) of the covariance
operator of a spatial correlation kernel, weighted by sqrt(lambda_k) and by
independent random coefficients.  The workloads here take the lognormal form
of that expansion,

    sigma(x) = sigma_f0 * exp( sum_{k<M} sqrt(lambda_k) phi_k(x) xi_k ),
    xi_k ~ N(0, 1),

with the exponential kernel C(x, y) = s2 * exp(-|x - y| / ell) (Euclidean
distance, as the paper's kernel is a function of the Euclidean distance,
Sec. 4 "Parameters for KL expansion").

The eigenpairs of the integral operator (C phi)(x) = int C(x, y) phi(y) dy
are approximated by the Nystrom method with trapezoid (lumped Q1) weights on a
KL grid, and extended to arbitrary points by the Nystrom interpolation formula.
The closed-form 1D eigenpairs of the exponential kernel are also given here;
they pin the Nystrom solver.

Test infrastructure only (see the package docstring).
"""

import numpy as np
import scipy.linalg
import scipy.optimize


def exp_kernel(x, y, ell, s2):
    """s2 * exp(-|x - y| / ell) for point sets x (p, d), y (q, d)."""
    x = np.atleast_2d(x)
    y = np.atleast_2d(y)
    d2 = ((x[:, None, :] - y[None, :, :]) ** 2).sum(axis=2)
    return s2 * np.exp(-np.sqrt(d2) / ell)


class NystromKL:
    """Nystrom eigenpairs of the exponential covariance operator on a grid.

    grid : oracle.grid.Grid on which the operator is discretised
    n_modes : number of leading eigenpairs kept
    """

    def __init__(self, grid, ell, s2, n_modes):
        self.grid = grid
        self.ell = float(ell)
        self.s2 = float(s2)
        self.pts = grid.nodes()
        self.w = grid.lumped_weights()
        C = exp_kernel(self.pts, self.pts, self.ell, self.s2)
        sw = np.sqrt(self.w)
        Ksym = sw[:, None] * C * sw[None, :]
        lam, V = scipy.linalg.eigh(Ksym)
        order = np.argsort(lam)[::-1]
        self.all_lambdas = lam[order]
        lam = lam[order][:n_modes]
        V = V[:, order][:, :n_modes]
        psi = V / sw[:, None]           # eigenfunction values at the KL nodes
        # sign convention: positive mean, else first significant entry positive
        for k in range(psi.shape[1]):
            mean = self.w @ psi[:, k]
            if abs(mean) > 1e-10:
                s = np.sign(mean)
            else:
                j = np.argmax(np.abs(psi[:, k]) > 1e-12)
                s = np.sign(psi[j, k])
            psi[:, k] *= s
        self.lambdas = lam
        self.psi_nodes = psi

    def eigenfunctions(self, points):
        """Nystrom extension phi_k(x) = lambda_k^-1 sum_j w_j C(x, x_j) phi_k(x_j)."""
        C = exp_kernel(points, self.pts, self.ell, self.s2)
        return (C * self.w[None, :]) @ self.psi_nodes / self.lambdas[None, :]

    def modes(self, points):
        """modes[e, k] = sqrt(lambda_k) phi_k(x_e): the scaled KL basis."""
        return self.eigenfunctions(points) * np.sqrt(self.lambdas)[None, :]


def exp_kernel_1d_eigenpairs(ell, s2, n, length=1.0):
    """Closed-form eigenpairs of s2 exp(-|x-y|/ell) on [0, length].

    On the symmetric interval [-a, a] (a = length / 2) with c = 1 / ell the
    eigenfunctions are cos(w t) (even) with c - w tan(w a) = 0, and sin(w t)
    (odd) with w + c tan(w a) = 0, and lambda = 2 c s2 / (w^2 + c^2).
    Returns the n largest eigenvalues (descending) and a callable giving the
    L2-normalised eigenfunctions at points x in [0, length].
    """
    a = 0.5 * length
    c = 1.0 / ell
    roots = []
    # even roots: w in ((j - 1/2) pi / a ... ) -- one root per branch of tan
    for j in range(n + 2):
        lo = j * np.pi / a + 1e-12
        hi = (j + 0.5) * np.pi / a - 1e-12
        f = lambda w: c * np.cos(w * a) - w * np.sin(w * a)  # noqa: E731
        roots.append(("even", scipy.optimize.brentq(f, lo, hi, xtol=1e-15, rtol=1e-15)))
        lo = (j + 0.5) * np.pi / a + 1e-12
        hi = (j + 1.0) * np.pi / a - 1e-12
        g = lambda w: w * np.cos(w * a) + c * np.sin(w * a)  # noqa: E731
        roots.append(("odd", scipy.optimize.brentq(g, lo, hi, xtol=1e-15, rtol=1e-15)))
    pairs = [(2 * c * s2 / (w * w + c * c), kind, w) for kind, w in roots]
    pairs.sort(key=lambda p: -p[0])
    pairs = pairs[:n]
    lambdas = np.array([p[0] for p in pairs])

    def funcs(x):
        t = np.asarray(x) - a
        cols = []
        for _, kind, w in pairs:
            if kind == "even":
                norm = np.sqrt(a + np.sin(2 * w * a) / (2 * w))
                cols.append(np.cos(w * t) / norm)
            else:
                norm = np.sqrt(a - np.sin(2 * w * a) / (2 * w))
                cols.append(np.sin(w * t) / norm)
        return np.stack(cols, axis=1)

    return lambdas, funcs


def synthesize_sigma(modes, xi, sigma_f0):
    """sigma[s, e] = sigma_f0 * exp(sum_k modes[e, k] xi[s, k])."""
    modes = np.asarray(modes, dtype=np.float64)
    xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))
    g = xi @ modes.T
    return sigma_f0 * np.exp(g)


# ---------------------------------------------------------------------------
# The paper's own random field (Sec. 2.2, eq. KL-expansion; Sec. 4, "Parameters
# for KL expansion"): an additive expansion G = G_0 + s sum_k sqrt(lambda_k)
# phi_k(x) y_k with y_k ~ U(-1, 1), the Gaussian correlation kernel
# exp(-d^2 / sigma_KL), and the stochastic dimension M fixed by a low-rank
# pivoted Cholesky factor of the covariance matrix on the mesh points.
# ---------------------------------------------------------------------------


def gauss_kernel(x, y, sig_kl):
    """exp(-|x - y|^2 / sig_kl) for point sets x (p, d), y (q, d)."""
    x = np.atleast_2d(x)
    y = np.atleast_2d(y)
    d2 = ((x[:, None, :] - y[None, :, :]) ** 2).sum(axis=2)
    return np.exp(-d2 / sig_kl)


class PivotedCholeskyKL:
    """Rank-M pivoted Cholesky of the covariance matrix C_ij = k(x_i, x_j).

    The factor is built one column at a time, each time pivoting on the
    largest remaining diagonal entry of C - L L^T (Harbrecht, Peters and
    Schneider's low-rank approximation, the method the paper names), so only
    M columns of C are ever formed.  The KL pairs are those of the low-rank
    matrix L L^T: with L^T L = Q diag(lambda) Q^T, its eigenvectors are
    phi = L Q lambda^-1/2, so sqrt(lambda_k) phi_k(x_i) = (L Q)_ik at the mesh
    points.  Away from them the factor row of a point x is the one that
    reproduces the pivot columns, L(x) = C(x, P) L_P^-T (L_P: the pivot rows
    of L), which agrees with L at the mesh points.

    points : (N, d) mesh points;  rank : M;  sig_kl : the kernel's sigma_KL
    """

    def __init__(self, points, sig_kl, rank):
        pts = np.asarray(points, dtype=np.float64)
        N = pts.shape[0]
        M = int(rank)
        if not 1 <= M <= N:
            raise ValueError("rank must be in 1..N")
        self.pts = pts
        self.sig_kl = float(sig_kl)
        L = np.zeros((N, M))
        d = np.ones(N)  # diagonal of C (unit variance kernel)
        piv = []
        for m in range(M):
            p = int(np.argmax(d))
            piv.append(p)
            col = gauss_kernel(pts, pts[p:p + 1], self.sig_kl)[:, 0] - L[:, :m] @ L[p, :m]
            L[:, m] = col / np.sqrt(d[p])
            d = d - L[:, m] ** 2
            d[piv] = 0.0
        self.L = L
        self.piv = np.array(piv)
        self.trace_error = float(N - (L * L).sum())  # trace(C - L L^T), C_ii = 1
        lam, Q = np.linalg.eigh(L.T @ L)
        order = np.argsort(lam)[::-1]
        lam = lam[order]
        Q = Q[:, order]
        V = L @ Q
        for k in range(M):  # sign: positive sum over the mesh points, else first significant entry
            tot = V[:, k].sum()
            if abs(tot) > 1e-10 * np.abs(V[:, k]).sum():
                sgn = np.sign(tot)
            else:
                j = int(np.argmax(np.abs(V[:, k]) > 1e-12 * np.abs(V[:, k]).max()))
                sgn = np.sign(V[j, k])
            Q[:, k] *= sgn
        self.lambdas = lam
        self.Q = Q

    def factor_rows(self, x):
        """L(x) = C(x, P) L_P^-T, shape (p, M)."""
        Cx = gauss_kernel(x, self.pts[self.piv], self.sig_kl)
        LP = self.L[self.piv, :]
        return np.linalg.solve(LP, Cx.T).T

    def modes(self, x):
        """modes[e, k] = sqrt(lambda_k) phi_k(x_e), shape (p, M)."""
        return self.factor_rows(x) @ self.Q


def damping(modes_on_mesh, s, delta):
    """The factor s of the expansion, lowered where needed so that
    s * max_x sum_k |sqrt(lambda_k) phi_k(x)| <= delta: the largest
    perturbation over all y in [-1, 1]^M then stays within delta G_0, the
    paper's uniform-ellipticity requirement (Sec. 2.2)."""
    bound = np.abs(modes_on_mesh).sum(axis=1).max()
    return min(float(s), float(delta) / bound)


def synthesize_additive(modes, y, g0):
    """G[s, e] = g0 * (1 + sum_k modes[e, k] y[s, k]) with the damping folded into modes."""
    modes = np.asarray(modes, dtype=np.float64)
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    return g0 * (1.0 + y @ modes.T)
