"""Monte Carlo and multilevel Monte Carlo estimators (oracle).

* MC estimator (Sec. 3.1.2, eq. MC-estimator): the sample mean of N i.i.d.
  solutions.
* MLMC estimator (Sec. 3.1.2, eq. MLMC-estimator): the sum over levels of MC
  means of the differences u_l - u_{l-1}, with u_{-1} = 0; a fine/coarse pair
  shares its random input.
* The paper transfers fields from a coarse to a refined mesh by standard
  finite-element interpolation (Sec. 3.4).  Every per-level quantity is
  interpolated to the finest grid before any statistic is taken.
* Variance reading: Var = sum_l [s^2(P Q_l) - s^2(P Q_{l-1})] with unbiased
  sample variances (the same common-input pairs), which telescopes exactly.
* Work model of Sec. 4.2.2 (eq. work and the asymptotic forms).

Test infrastructure only (see the package docstring).
"""

import numpy as np


# -- transfer ---------------------------------------------------------------

def interpolate(coarse, field, fine):
    """Q1 interpolation of a nodal field on grid ``coarse`` at the nodes of ``fine``.

    Both grids cover the same box.  Plain multilinear interpolation inside the
    coarse element containing each fine node.
    """
    pts = fine.nodes()
    d = coarse.dim
    lo_idx = []
    frac = []
    for a in range(d):
        s = pts[:, a] / coarse.h[a]
        i = np.clip(np.floor(s).astype(np.int64), 0, coarse.shape[a] - 2)
        lo_idx.append(i)
        frac.append(s - i)
    out = np.zeros(pts.shape[0])
    field = np.asarray(field, dtype=np.float64)
    for v in range(2 ** d):
        w = np.ones(pts.shape[0])
        idx = []
        for a in range(d):
            b = (v >> a) & 1
            w = w * (frac[a] if b else 1.0 - frac[a])
            idx.append(lo_idx[a] + b)
        out += w * field[coarse.node_index(idx)]
    return out


# -- statistics -------------------------------------------------------------

def two_pass(samples):
    """(mean, unbiased variance) over axis 0 by the two-pass formula."""
    x = np.asarray(samples, dtype=np.float64)
    n = x.shape[0]
    mean = x.sum(axis=0) / n
    var = ((x - mean) ** 2).sum(axis=0) / (n - 1) if n > 1 else np.zeros_like(mean)
    return mean, var


class Welford:
    """Running (count, mean, M2) over a stream of arrays (Welford's update)."""

    def __init__(self, shape):
        self.count = 0
        self.mean = np.zeros(shape)
        self.m2 = np.zeros(shape)

    def push(self, x):
        self.count += 1
        d = x - self.mean
        self.mean = self.mean + d / self.count
        self.m2 = self.m2 + d * (x - self.mean)

    def variance(self):
        return self.m2 / (self.count - 1) if self.count > 1 else np.zeros_like(self.mean)

    @staticmethod
    def merge(a, b):
        """Chan et al. pairwise combination of two partial states."""
        out = Welford(a.mean.shape)
        out.count = a.count + b.count
        if out.count == 0:
            return out
        d = b.mean - a.mean
        out.mean = a.mean + d * (b.count / out.count)
        out.m2 = a.m2 + b.m2 + d * d * (a.count * b.count / out.count)
        return out


# -- MLMC combination -------------------------------------------------------

def mlmc_combine(fine_q, coarse_q, weights, vol=None):
    """Combine per-level samples already interpolated to the finest grid.

    fine_q[l]   : (N_l, n_L) samples of P Q_l
    coarse_q[l] : (N_l, n_L) samples of P Q_{l-1} with the same inputs
                  (None for l = 0, meaning Q_{-1} = 0)
    weights     : (n_L,) quadrature weights of the finest grid

    Returns dict: mean, var (n_L,), level_mean, level_var (Y_l fields),
    V (per-level scalar |D|^-1 int s^2(Y_l)), counts.  vol: the measure the
    integral is divided by (default: the sum of the weights).
    """
    L1 = len(fine_q)
    vol = weights.sum() if vol is None else vol
    mean = 0.0
    var = 0.0
    level_mean, level_var, V = [], [], []
    for l in range(L1):
        qf = np.asarray(fine_q[l])
        mf, vf = two_pass(qf)
        if coarse_q[l] is None:
            y = qf
            vc = 0.0
        else:
            qc = np.asarray(coarse_q[l])
            _, vc = two_pass(qc)
            y = qf - qc
        my, vy = two_pass(y)
        mean = mean + my
        var = var + (vf - vc)
        level_mean.append(my)
        level_var.append(vy)
        V.append(float(weights @ vy / vol))
    return {
        "mean": np.asarray(mean),
        "var": np.asarray(var),
        "level_mean": np.array(level_mean),
        "level_var": np.array(level_var),
        "V": np.array(V),
        "counts": np.array([len(q) for q in fine_q]),
    }


def giles_allocation(V, C, eps):
    """Sample counts N_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k)).

    Minimises the total cost sum N_l C_l subject to the estimator variance
    sum V_l / N_l <= eps^2 / 2 (half of the mean-square-error budget; the other
    half is left to the bias).
    """
    V = np.asarray(V, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    s = np.sum(np.sqrt(V * C))
    return np.ceil(2.0 / eps ** 2 * np.sqrt(V / C) * s).astype(np.int64)


# -- work model (Sec. 4.2.2) --------------------------------------------------

def work_fixed_setting(Wp, N):
    """(W_MC, W_MLMC) of eq. work: W_l = W'_{l-1} + W'_l, W'_{-1} = 0."""
    Wp = np.asarray(Wp, dtype=np.float64)
    N = np.asarray(N, dtype=np.float64)
    Wl = Wp + np.concatenate([[0.0], Wp[:-1]])
    return Wp[-1] * N[-1], float(np.sum(Wl * N))


def work_asymptotic_sum(gd, L):
    """sum_{l=0}^{L} 2^{gd l} 2^{4 (L - l)}: the MLMC asymptotic work as a plain sum."""
    return float(sum(2.0 ** (gd * l) * 2.0 ** (4 * (L - l)) for l in range(L + 1)))
