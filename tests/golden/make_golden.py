"""Writes the stored expected values under tests/golden/ from the oracle only.

kl_exp1d_ell0.2_s0.1.txt : the 8 largest eigenvalues of the exponential
    covariance 0.1 exp(-|x - y| / 0.2) on [0, 1], from the closed-form
    transcendental equations (oracle.kl.exp_kernel_1d_eigenpairs).

Run from the repository root:  python tests/golden/make_golden.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import kl  # noqa: E402


def main():
    lam, _ = kl.exp_kernel_1d_eigenpairs(0.2, 0.1, 8)
    np.savetxt(os.path.join(HERE, "kl_exp1d_ell0.2_s0.1.txt"), lam, fmt="%.12e",
               header="closed-form eigenvalues, exponential kernel, ell=0.2, variance=0.1, [0,1]")


if __name__ == "__main__":
    main()
