"""Structured tensor-product grids for Q1 finite elements (oracle).

The paper uses a nested hierarchy of meshes with mesh size h_l ~ 2^-l
(Sec. 3.1.2) obtained by uniform coarsening (Sec. 4.1, Sec. 4.2).  Here every
level is an axis-aligned box [0, L_x] x [0, L_y] x [0, L_z] split into equal
boxes (Q1 elements).  Nodes are numbered lexicographically with x fastest,
then y, then z; elements likewise.

Test infrastructure only (see the package docstring).
"""

import numpy as np


class Grid:
    """A structured grid of ``shape`` nodes per axis on the box ``lengths``.

    shape   : tuple of node counts per axis, len 1, 2 or 3 (x first)
    lengths : tuple of box side lengths, same length as shape
    """

    def __init__(self, shape, lengths=None):
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        if lengths is None:
            lengths = (1.0,) * self.dim
        self.lengths = tuple(float(v) for v in lengths)
        assert len(self.lengths) == self.dim
        assert all(s >= 2 for s in self.shape)
        self.h = tuple(L / (s - 1) for L, s in zip(self.lengths, self.shape))
        self.n = int(np.prod(self.shape))
        self.eshape = tuple(s - 1 for s in self.shape)
        self.n_el = int(np.prod(self.eshape))

    # -- coordinates -------------------------------------------------------
    def axis_nodes(self, a):
        return np.arange(self.shape[a]) * self.h[a]

    def nodes(self):
        """Node coordinates, array (n, dim), x fastest."""
        axes = [self.axis_nodes(a) for a in range(self.dim)]
        mesh = np.meshgrid(*axes[::-1], indexing="ij")  # slowest axis first
        return np.stack([m.ravel() for m in mesh[::-1]], axis=1)

    def centroids(self):
        """Element centroids, array (n_el, dim), x fastest."""
        axes = [(np.arange(self.eshape[a]) + 0.5) * self.h[a] for a in range(self.dim)]
        mesh = np.meshgrid(*axes[::-1], indexing="ij")
        return np.stack([m.ravel() for m in mesh[::-1]], axis=1)

    # -- connectivity ------------------------------------------------------
    def node_index(self, idx):
        """Flat node index of a multi-index (tuple of int arrays, x first)."""
        flat = np.zeros_like(np.asarray(idx[0]))
        stride = 1
        for a in range(self.dim):
            flat = flat + np.asarray(idx[a]) * stride
            stride *= self.shape[a]
        return flat

    def element_nodes(self):
        """(n_el, 2^dim) flat node indices of every element.

        Local vertex v has offset bit a = (v >> a) & 1 along axis a.
        """
        axes = [np.arange(self.eshape[a]) for a in range(self.dim)]
        mesh = np.meshgrid(*axes[::-1], indexing="ij")
        lo = [m.ravel() for m in mesh[::-1]]  # per axis, x first
        out = np.empty((self.n_el, 2 ** self.dim), dtype=np.int64)
        for v in range(2 ** self.dim):
            idx = [lo[a] + ((v >> a) & 1) for a in range(self.dim)]
            out[:, v] = self.node_index(idx)
        return out

    def lumped_weights(self):
        """Trapezoid-rule (lumped Q1 mass) quadrature weight of every node."""
        w = np.ones(1)
        for a in reversed(range(self.dim)):
            wa = np.full(self.shape[a], self.h[a])
            wa[0] = wa[-1] = 0.5 * self.h[a]
            w = np.kron(w, wa)
        return w

    def volume(self):
        return float(np.prod(self.lengths))


def space_time_dofs(grid, m):
    """Space-time degrees of freedom counted with the t = 0 layer, n (m + 1).

    Reading of the paper's Tables 2-3: the printed Dof counts are the products
    of spatial node counts and time-node counts (including the initial layer).
    """
    return grid.n * (m + 1)


def cube_hierarchy_level(l):
    """Cube level l of Table 2: h = 0.2 / 2^l on [0,1]^3, dt = 0.04 / 2^l, T = 0.96.

    Returns (Grid, m).  (5 * 2^l + 1)^3 nodes and 24 * 2^l time steps.
    """
    s = 5 * 2 ** l + 1
    return Grid((s, s, s), (1.0, 1.0, 1.0)), 24 * 2 ** l
