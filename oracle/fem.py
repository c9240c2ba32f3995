"""Q1 mass and stiffness matrices, assembled as sparse CSR (oracle).

Follows the definitions of Sec. 3.2 of the paper: M_h = [int psi_i psi_j],
K_h = [int (G grad psi_i) . grad psi_j], with the nodal (here tensor-product
Q1) basis.  G is the element-constant conductivity tensor
D_e = sigma_e a_e a_e^T + tau (I - a_e a_e^T) of a fibre direction a_e: the
random fibre conductivity sigma_e and a fixed transverse conductivity tau.
Element integrals use tensor Gauss quadrature with 2 points per axis, exact for
products of Q1 functions and their derivatives on axis-aligned boxes.

Test infrastructure only (see the package docstring).
"""

import itertools

import numpy as np
import scipy.sparse as sp


def _gauss_1d(h, nq):
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * h * (x + 1.0), 0.5 * h * w


def _basis_1d(s, h, bit):
    return (s / h) if bit else (1.0 - s / h)


def _dbasis_1d(s, h, bit):
    return np.full_like(s, (1.0 / h) if bit else (-1.0 / h))


def element_matrices(h, nq=2):
    """Reference Q1 element integrals on the box prod_a [0, h_a].

    Returns (Me, G): Me[v, w] = int phi_v phi_w and
    G[a, b, v, w] = int d_a phi_v d_b phi_w, for the 2^d local vertices
    (vertex v has offset bit a = (v >> a) & 1 along axis a).
    """
    d = len(h)
    nv = 2 ** d
    pts = [_gauss_1d(h[a], nq) for a in range(d)]
    Me = np.zeros((nv, nv))
    G = np.zeros((d, d, nv, nv))
    for qidx in itertools.product(range(nq), repeat=d):
        x = [pts[a][0][qidx[a]] for a in range(d)]
        wq = np.prod([pts[a][1][qidx[a]] for a in range(d)])
        phi = np.empty(nv)
        grad = np.empty((d, nv))
        for v in range(nv):
            bits = [(v >> a) & 1 for a in range(d)]
            vals = [_basis_1d(np.array(x[a]), h[a], bits[a]) for a in range(d)]
            ders = [_dbasis_1d(np.array(x[a]), h[a], bits[a]) for a in range(d)]
            phi[v] = np.prod(vals)
            for a in range(d):
                grad[a, v] = np.prod([ders[b] if b == a else vals[b] for b in range(d)])
        Me += wq * np.outer(phi, phi)
        for a in range(d):
            for b in range(d):
                G[a, b] += wq * np.outer(grad[a], grad[b])
    return Me, G


def fiber_directions(theta, dim):
    """Unit fibre vectors a_e for angles theta (in the x-y plane)."""
    theta = np.asarray(theta, dtype=np.float64)
    if dim == 1:
        return np.ones((theta.size, 1))
    a = np.zeros((theta.size, dim))
    a[:, 0] = np.cos(theta)
    a[:, 1] = np.sin(theta)
    return a


def diffusion_tensors(sigma, theta, tau, dim, tau_rel=0.0):
    """D_e = sigma_e a a^T + (tau + tau_rel sigma_e) (I - a a^T), array (n_el, dim, dim).

    tau_rel = 0: a constant transverse conductivity tau (the fibre model);
    tau = 0, tau_rel = 1: the isotropic scalar field D_e = sigma_e I of the
    paper's experiments (Sec. 2.1 takes G scalar and isotropic)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    a = fiber_directions(theta, dim)
    aa = a[:, :, None] * a[:, None, :]
    eye = np.eye(dim)[None, :, :]
    t = tau + tau_rel * sigma
    return sigma[:, None, None] * aa + t[:, None, None] * (eye - aa)


def fiber_angles(grid, law):
    """Fibre angle of every element centroid.

    law 'diag2d'  : theta = pi/4 + 0.5 y  (2D workloads)
    law 'rot3d'   : theta = -pi/3 + (2 pi / 3) z / L_z  (rotation through the slab)
    law 'x'       : theta = 0 (fibres along x)
    law 'diag'    : theta = pi/4 everywhere
    """
    c = grid.centroids()
    if law == "diag2d":
        return np.pi / 4 + 0.5 * c[:, 1]
    if law == "rot3d":
        return -np.pi / 3 + (2 * np.pi / 3) * c[:, 2] / grid.lengths[2]
    if law == "x":
        return np.zeros(grid.n_el)
    if law == "diag":
        return np.full(grid.n_el, np.pi / 4)
    raise ValueError(law)


def _assemble(grid, blocks):
    """Sum element matrices blocks[e] (n_el, nv, nv) into an n x n CSR."""
    en = grid.element_nodes()
    nv = en.shape[1]
    rows = np.repeat(en, nv, axis=1).ravel()
    cols = np.tile(en, (1, nv)).ravel()
    A = sp.coo_matrix((blocks.reshape(-1), (rows, cols)), shape=(grid.n, grid.n))
    return A.tocsr()


def assemble_mass(grid):
    Me, _ = element_matrices(grid.h)
    blocks = np.broadcast_to(Me, (grid.n_el,) + Me.shape)
    return _assemble(grid, np.ascontiguousarray(blocks))


def assemble_stiffness(grid, D):
    """K = sum_e sum_ab D_e[a, b] int d_a phi d_b phi, D of shape (n_el, d, d)."""
    _, G = element_matrices(grid.h)
    blocks = np.einsum("eab,abvw->evw", D, G)
    return _assemble(grid, blocks)
