"""Plain, slow FP64 CPU oracle of the space-time MLMC monodomain method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only ``tests/``, the smoke check and the CPU-baseline leg
of ``bench.py`` may use it.  It shares no code with the HIP path.

What it computes follows the paper "Space-time multilevel Monte Carlo methods
and their application to cardiac electrophysiology" (Ben Bader, Benedusi,
Quaglino, Zulian, Krause):

* grid.py       structured nested Q1 grids (Sec. 3.1.2 nested hierarchy,
                Tables 1-3 for the paper's own level sizes)
* kl.py         truncated Karhunen-Loeve expansion of the conductivity
                (Sec. 2.2, eq. KL-expansion), Nystrom eigenpairs of the
                covariance operator, closed-form 1D exponential-kernel pairs
* fem.py        mass and stiffness matrices (Sec. 3.2, definitions of M_h, K_h)
* spacetime.py  the block lower-bidiagonal space-time system (Sec. 3.2,
                eq. system_C) with the nonlinear reaction term and its Jacobian
                (Sec. 3.3, eq. mono_disc), Newton's method (Sec. 3.5) by
                direct sparse solves
* qoi.py        activation-time map of a space-time solution
* mlmc.py       MC and MLMC estimators (Sec. 3.1.2, eqs. MC-estimator and
                MLMC-estimator), Welford / two-pass statistics, nested Q1
                interpolation, work model (Sec. 4.2.2, eq. work)
* api.py        the four calls of the library boundary, same names

Every floating-point quantity is float64.
"""

from . import grid, kl, fem, spacetime, qoi, mlmc, api  # noqa: F401
from .api import kl_synthesize, st_solve, activation_map, mlmc_estimate  # noqa: F401
