"""Writes tests/golden/slab3d_prefix2.txt from the oracle only.

The first two slabs of the full-size 3D slab workload (65 x 65 x 17 nodes,
dt = T/256, 64 KL modes of the exponential covariance, fibres rotating
through the thickness), for sample 0 of the workload's seeded KL
coefficients: the oracle's Nystrom modes and conductivity, then Newton slab by
slab with sparse LU.  Slabs 1..k of the full-horizon solution depend only on
the slabs before them (the system is block lower bidiagonal), so these are the
first two slabs of the 256-step solution.

Stored, for k = 1, 2: the 2-norm and the sum of u_k over all nodes, and u_k at
a fixed set of nodes: every node within distance 0.2 of the stimulus centre
(where u changes most) and 300 seeded others.  The conductivity the oracle
solved with is stored beside it (slab3d_prefix2_sigma.npy, float64 per
element): the exponential covariance on this machine has degenerate eigenpairs
(x <-> y symmetry), within which a symmetric eigensolver may return any
orthonormal basis, so modes computed on another machine can give another,
equally valid field.  The test solves with the stored field.

Run from the repository root (several minutes of sparse LU):
    python tests/golden/make_slab3d_prefix.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.api as oapi  # noqa: E402
import stinputs  # noqa: E402

OUT = os.path.join(HERE, "slab3d_prefix2.txt")
OUT_SIGMA = os.path.join(HERE, "slab3d_prefix2_sigma.npy")
K = 2


def golden_nodes(wl):
    g = oapi.level_grid(wl, 0)
    x = g.nodes()
    near = np.flatnonzero(((x - np.asarray(wl["ic_center"])) ** 2).sum(axis=1) <= 0.2 ** 2)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([1911, 65, 17])))
    other = rng.choice(np.setdiff1d(np.arange(g.n), near), size=300, replace=False)
    return np.sort(np.concatenate([near, other]))


def main():
    wl = stinputs.workload("slab3d", precision="fp64")
    basis = oapi.kl_basis(wl)
    modes = oapi.kl_modes(wl, 0, basis)
    xi = stinputs.xi("slab3d", 0, 1, wl["n_modes"])
    sig = oapi.kl_synthesize(modes, xi, wl["sigma_f0"])
    np.save(OUT_SIGMA, sig[0])
    wp = dict(wl)
    wp["steps"] = [K]
    wp["T"] = wl["T"] * K / wl["steps"][0]
    U, st = oapi.st_solve(wp, 0, sig, mode="timestep")
    U = U[0]
    idx = golden_nodes(wl)
    with open(OUT, "w") as f:
        f.write("# oracle: first %d slabs of slab3d (65x65x17 nodes, dt = 1/256), sample 0; written by "
                "tests/golden/make_slab3d_prefix.py (oracle only)\n" % K)
        f.write("# newton iterations per slab (max): %d\n" % st[0].iterations)
        for k in range(K):
            f.write("norm2 %d %.17e\n" % (k + 1, np.linalg.norm(U[k])))
            f.write("sum %d %.17e\n" % (k + 1, U[k].sum()))
        for i in idx:
            f.write("node %d %s\n" % (i, " ".join("%.17e" % U[k, i] for k in range(K))))


if __name__ == "__main__":
    main()
