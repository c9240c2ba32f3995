"""Offline construction of the KL modes fed to the KL synthesis kernel.

The paper computes the truncated KL basis once, before sampling, by a low-rank
factorisation of the covariance (Sec. 2.2; pivoted Cholesky in the paper).
Here the covariance operator of s2 exp(-|x - y| / ell) is discretised by the
Nystrom method on a structured grid with trapezoid weights, its leading
eigenpairs are taken from the symmetrised weighted kernel matrix, and the
eigenfunctions are evaluated at element centroids by the Nystrom formula.
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


def workload_modes(wl):
    """Modes of every level of a workload (list of (E_l, M) float64 arrays)."""
    basis = KLBasis(wl["kl_grid"], wl["lengths"], wl["ell"], wl["s2"], wl["n_modes"])
    return [np.ascontiguousarray(basis.modes_at(element_centroids(shape, wl["lengths"])))
            for shape in wl["levels"]]
