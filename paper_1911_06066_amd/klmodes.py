"""Offline construction of the KL modes fed to the KL synthesis kernel.

The paper computes the truncated KL basis once, before sampling, by a low-rank
factorisation of the covariance (Sec. 2.2; pivoted Cholesky in the paper).
For the exponential kernel s2 exp(-|x - y| / ell) of the lognormal workloads
the covariance operator is discretised by the Nystrom method on a structured
grid with trapezoid weights, its leading eigenpairs are taken from the
symmetrised weighted kernel matrix, and the eigenfunctions are evaluated at
element centroids by the Nystrom formula.  The paper's own Gaussian kernel is
factored by pivoted Cholesky (GaussLowRankBasis).
The result, modes[e, k] = sqrt(lambda_k) phi_k(x_e), is plain input data of
the library; this host step is not on the sampling path.
"""

import numpy as np
import scipy.linalg
from scipy.spatial.distance import cdist


def _axis(n, length):
    x = np.linspace(0.0, length, n)
    w = np.full(n, length / (n - 1))
    w[[0, -1]] *= 0.5
    return x, w


def _tensor_points(shape, lengths):
    axes = [_axis(n, L) for n, L in zip(shape, lengths)]
    mesh = np.meshgrid(*[a[0] for a in axes], indexing="xy" if len(shape) == 2 else "ij")
    if len(shape) == 2:
        pts = np.stack([mesh[0].ravel(), mesh[1].ravel()], axis=1)
        w = np.outer(axes[1][1], axes[0][1]).ravel()
    else:
        # x fastest: build by broadcasting explicitly
        xs, ys, zs = (a[0] for a in axes)
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        wz, wy, wx = axes[2][1], axes[1][1], axes[0][1]
        w = (wz[:, None, None] * wy[None, :, None] * wx[None, None, :]).ravel()
    return pts, w


def element_centroids(shape, lengths):
    """Centroids of the Q1 elements of a grid with `shape` nodes, x fastest."""
    cs = [(np.arange(n - 1) + 0.5) * (L / (n - 1)) for n, L in zip(shape, lengths)]
    if len(shape) == 2:
        Y, X = np.meshgrid(cs[1], cs[0], indexing="ij")
        return np.stack([X.ravel(), Y.ravel()], axis=1)
    Z, Y, X = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


class KLBasis:
    """Leading eigenpairs of the exponential covariance on the workload box."""

    def __init__(self, kl_shape, lengths, ell, s2, n_modes):
        self.ell, self.s2 = float(ell), float(s2)
        self.pts, self.w = _tensor_points(kl_shape, lengths)
        n = self.pts.shape[0]
        sw = np.sqrt(self.w)
        A = self.s2 * np.exp(-cdist(self.pts, self.pts) / self.ell)
        A *= sw[:, None]
        A *= sw[None, :]
        lam, vec = scipy.linalg.eigh(A, subset_by_index=[n - n_modes, n - 1])
        order = np.argsort(-lam)
        self.lam = lam[order]
        phi = vec[:, order] / sw[:, None]
        # orientation: positive weighted mean, else positive first significant value
        for k in range(phi.shape[1]):
            mu = float(self.w @ phi[:, k])
            if abs(mu) <= 1e-10:
                mu = phi[np.flatnonzero(np.abs(phi[:, k]) > 1e-12)[0], k]
            if mu < 0:
                phi[:, k] = -phi[:, k]
        self.phi = phi

    def modes_at(self, points, block=65536):
        """sqrt(lambda_k) phi_k(x) at points (p, d) by Nystrom interpolation."""
        out = np.empty((points.shape[0], self.lam.size))
        coef = (self.w[:, None] * self.phi) / np.sqrt(self.lam)[None, :]  # w_j phi_k(x_j) / sqrt(lam)
        for a in range(0, points.shape[0], block):
            C = self.s2 * np.exp(-cdist(points[a:a + block], self.pts) / self.ell)
            out[a:a + block] = C @ coef
        return out


class GaussLowRankBasis:
    """The paper's own field (Sec. 2.2, Sec. 4 "Parameters for KL expansion"):
    correlation exp(-d^2 / sig_kl) between the nodes of a grid (the finest
    mesh), approximated to rank M by pivoted Cholesky -- each step takes the
    node with the largest remaining variance as pivot and forms only that
    kernel column -- and rotated onto the eigenvectors of the low-rank
    covariance F^T F (F: the M x N factor), so that the modes are
    sqrt(lambda_k) phi_k at the nodes.  Other points get the factor rows that
    reproduce the kernel's pivot columns."""

    def __init__(self, kl_shape, lengths, sig_kl, n_modes):
        pts, _ = _tensor_points(kl_shape, lengths)
        n = pts.shape[0]
        if not 1 <= n_modes <= n:
            raise ValueError("n_modes must be in 1..%d" % n)
        self.sig_kl = float(sig_kl)
        F = np.zeros((n_modes, n))
        var = np.ones(n)  # remaining variance of each node
        piv = []
        for m in range(n_modes):
            j = int(np.argmax(var))
            col = np.exp(-cdist(pts[j:j + 1], pts, "sqeuclidean")[0] / self.sig_kl)
            if m:
                col -= F[:m, j] @ F[:m]
            F[m] = col / np.sqrt(var[j])
            var -= F[m] * F[m]
            piv.append(j)
            var[piv] = 0.0
        self.pivots = pts[piv]
        self.residual_trace = float(n - np.einsum("ij,ij->", F, F))
        # eigen-rotation of the low-rank covariance F^T F (same nonzero spectrum as F F^T)
        lam, R = scipy.linalg.eigh(F @ F.T)
        order = np.argsort(-lam)
        lam, R = lam[order], R[:, order]
        at_nodes = F.T @ R
        for k in range(n_modes):  # orientation: positive sum over the nodes, else first significant value
            total = float(at_nodes[:, k].sum())
            if abs(total) <= 1e-10 * float(np.abs(at_nodes[:, k]).sum()):
                big = np.abs(at_nodes[:, k]) > 1e-12 * float(np.abs(at_nodes[:, k]).max())
                total = at_nodes[np.flatnonzero(big)[0], k]
            if total < 0:
                R[:, k] = -R[:, k]
        self.lam = lam
        self.rot = R
        self.piv_factor = np.ascontiguousarray(F[:, piv])  # M x M, upper triangular (F[m, piv[j]] = 0 for m > j)
        self.node_modes = F.T @ R

    def modes_at(self, points, block=65536):
        """Rows of the rank-M factor at arbitrary points, rotated: (p, M)."""
        out = np.empty((points.shape[0], self.lam.size))
        for a in range(0, points.shape[0], block):
            K = np.exp(-cdist(points[a:a + block], self.pivots, "sqeuclidean") / self.sig_kl)
            # factor rows f(x) with f(x) . F[:, piv] = K(x, piv)
            rows = scipy.linalg.solve_triangular(self.piv_factor, K.T, trans="T", lower=False).T
            out[a:a + block] = rows @ self.rot
        return out


def additive_damping(node_modes, s, delta):
    """s, lowered if needed so that s max_x sum_k |mode_k(x)| <= delta: every
    y in [-1, 1]^M then keeps the conductivity within (1 +- delta) G_0, the
    uniform ellipticity the paper asks of its expansion (Sec. 2.2)."""
    worst = float(np.max(np.sum(np.abs(node_modes), axis=1)))
    return min(float(s), float(delta) / worst)


def workload_modes(wl):
    """Modes of every level of a workload (list of (E_l, M) float64 arrays)."""
    if wl.get("kernel", "exp") == "gauss":
        basis = GaussLowRankBasis(wl["kl_grid"], wl["lengths"], wl["sig_kl"], wl["n_modes"])
        scale = additive_damping(basis.node_modes, wl["kl_s"], wl["kl_delta"]) \
            if wl.get("field", "lognormal") == "additive" else 1.0
    else:
        basis = KLBasis(wl["kl_grid"], wl["lengths"], wl["ell"], wl["s2"], wl["n_modes"])
        scale = 1.0
    return [np.ascontiguousarray(basis.modes_at(element_centroids(shape, wl["lengths"])) * scale)
            for shape in wl["levels"]]
