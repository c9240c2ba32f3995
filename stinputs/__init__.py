"""Seeded synthetic inputs and workload descriptions shared by tests and bench.

This module holds data only -- workload sizes, parameters and the seeded
random draws of the KL coefficients -- and none of the method's arithmetic.
Both the CPU oracle and the HIP library receive what it produces as plain
arrays and numbers.

Workloads (2D sizes count nodes per axis; 3D sizes count nodes per axis of a
grid whose element counts are 64 x 64 x 16 etc.):

  small_mc_2d   33^2 nodes, 64 steps, 16 KL modes, 32 samples, FP64, one level
  mlmc3_2d      33^2/65^2/129^2 with 64/128/256 steps, 32 modes,
                512/128/32 fine/coarse pairs, FP64 batched, warm start
  mlmc4_2d_mixed  33^2 ... 257^2 with 64 ... 512 steps, 64 modes,
                1024/256/64/16 pairs, mixed precision
  slab3d        [0,1]^2 x [0,0.25], 65 x 65 x 17 nodes, 256 steps, 64 modes
                (ell 0.15, s2 0.2), 256 samples, mixed precision
  mlmc5_3d      five 3D levels 9x9x3 ... 129x129x33 nodes, 32 ... 512 steps,
                128 modes, sample counts chosen adaptively
  cable1d       the 1D+1 hierarchy of Table 1 (all six levels) as a strip of one
                element row: 31 2^l elements of 0.032 / 2^l cm, 4 2^l steps of 0.16 / 2^l ms,
                the cube's physics and field, space-time QoI E[u]
  cube4_3d      the paper's cube: [0,1]^3 cm, 6^3 ... 41^3 nodes, 24 ... 192
                steps to 0.96 ms, isotropic additive uniform field (Gaussian
                kernel, 66 modes), 1024/256/64/16 pairs, FP64
"""

import numpy as np

DEFAULT_SEED = 1911

_COMMON_2D = dict(
    dim=2,
    lengths=(1.0, 1.0),
    T=1.0,
    k_react=8.0,
    a_react=0.1,
    sigma_f0=1e-3,
    transverse_ratio=0.1,
    fiber_law="diag2d",
    ic_center=(0.0, 0.0),
    ic_radius=0.1,
    threshold=0.5,
    theta=1.0,  # time scheme: 1 backward Euler, 0.5 Crank-Nicolson
    ell=0.2,
    s2=0.1,
    kl_grid=(41, 41),
)

_COMMON_3D = dict(
    dim=3,
    lengths=(1.0, 1.0, 0.25),
    T=1.0,
    k_react=8.0,
    a_react=0.1,
    sigma_f0=1e-3,
    transverse_ratio=0.1,
    fiber_law="rot3d",
    ic_center=(0.0, 0.0, 0.0),
    ic_radius=0.1,
    threshold=0.5,
    theta=1.0,
    ell=0.15,
    s2=0.2,
    kl_grid=(21, 21, 6),
)


# The paper's cube experiment (Sec. 4, "Parameters for the experiments",
# "Parameters for KL expansion", Table 2).  Lengths in cm, times in ms, the
# potential in units of u_peak = 115 mV: the FHN current
# alpha (u - 0)(u - 28)(u - 115) becomes k v (v - a)(1 - v) with
# k = alpha u_peak^2 and a = u_th / u_peak.  Isotropic conductivity
# G = G_0 (1 + s sum_k sqrt(lambda_k) phi_k(x) y_k), y_k ~ U(-1, 1), Gaussian
# kernel exp(-d^2 / sigma_KL); the Gaussian stimulus of width 0.5 cm is the
# initial state; Crank-Nicolson as in the paper.
_ALPHA, _U_TH, _U_PEAK = 1.4e-3, 28.0, 115.0
_CUBE_3D = dict(
    dim=3,
    lengths=(1.0, 1.0, 1.0),
    T=0.96,
    k_react=_ALPHA * _U_PEAK * _U_PEAK,
    a_react=_U_TH / _U_PEAK,
    sigma_f0=3.325e-3,
    transverse_ratio=1.0,
    tau_relative=1,
    fiber_law="x",
    ic_kind="gauss",
    ic_center=(0.0, 0.0, 0.0),
    ic_radius=0.5,
    threshold=0.5,
    theta=0.5,
    field="additive",
    kernel="gauss",
    sig_kl=0.25,
    kl_s=0.3,
    kl_delta=0.5,
    xi_dist="uniform",
)


def _w(base, **kw):
    d = dict(base)
    d.update(kw)
    return d


WORKLOADS = {
    "small_mc_2d": _w(_COMMON_2D, name="small_mc_2d", levels=[(33, 33)], steps=[64],
                      n_modes=16, samples=[32], precision="fp64"),
    "mlmc3_2d": _w(_COMMON_2D, name="mlmc3_2d", levels=[(33, 33), (65, 65), (129, 129)],
                   steps=[64, 128, 256], n_modes=32, samples=[512, 128, 32],
                   precision="fp64"),
    "mlmc4_2d_mixed": _w(_COMMON_2D, name="mlmc4_2d_mixed",
                         levels=[(33, 33), (65, 65), (129, 129), (257, 257)],
                         steps=[64, 128, 256, 512], n_modes=64,
                         samples=[1024, 256, 64, 16], precision="mixed"),
    "slab3d": _w(_COMMON_3D, name="slab3d", levels=[(65, 65, 17)], steps=[256],
                 n_modes=64, samples=[256], precision="mixed"),
    # adaptive counts: pilot samples per level, then the optimal allocation
    # for an RMSE of target_rmse * T, up to `capacity` samples per level.  One
    # finest sample costs about 90 workgroup-seconds, so the pilot is 8
    "mlmc5_3d": _w(_COMMON_3D, name="mlmc5_3d",
                   levels=[(9, 9, 3), (17, 17, 5), (33, 33, 9), (65, 65, 17), (129, 129, 33)],
                   steps=[32, 64, 128, 256, 512], n_modes=128, samples=None,
                   target_rmse=1e-3, pilot=8, capacity=[2048, 1024, 512, 128, 32], precision="mixed"),
    "cube4_3d": _w(_CUBE_3D, name="cube4_3d",
                   levels=[(6, 6, 6), (11, 11, 11), (21, 21, 21), (41, 41, 41)],
                   steps=[24, 48, 96, 192], n_modes=66, kl_grid=(41, 41, 41),
                   samples=[1024, 256, 64, 16], precision="fp64"),
    # the 1D+1 study (Sec. 4.1, Table 1): the interval of 31 elements of
    # h = 0.032 cm, refined 2:1 in space and time; a 2D strip one element
    # high (half as high as the finest element is long) whose data do not
    # depend on y solves the 1D problem exactly -- the stimulus is centred on
    # the strip's midline, so both node rows see the same initial state.  The
    # study checks the convergence theory of Sec. 3.1.2, which is stated for
    # the stochastic heat equation: no ionic current (k_react = 0)
    "cable1d": _w(_CUBE_3D, name="cable1d", dim=2, lengths=(0.992, 0.002), T=0.64, k_react=0.0,
                  ic_center=(0.0, 0.001), ic_radius=0.25,
                  levels=[(32, 2), (63, 2), (125, 2), (249, 2), (497, 2), (993, 2)],
                  steps=[4, 8, 16, 32, 64, 128],
                  n_modes=16, kl_grid=(249, 2), samples=[4096, 256, 16, 2, 2, 2], qoi="spacetime",
                  precision="fp64"),
}

WORKLOAD_IDS = {name: i for i, name in enumerate(WORKLOADS)}


def workload(name, **overrides):
    """A copy of a workload description with optional overrides."""
    w = dict(WORKLOADS[name])
    w.update(overrides)
    return w


def xi(name, level, n_samples, n_modes, seed=DEFAULT_SEED, start=0):
    """KL coefficients (n_samples, n_modes) for one MLMC level: standard normal,
    or uniform on [-1, 1] for workloads whose xi_dist is 'uniform'.

    One PCG64 stream per (seed, workload, level), drawn in sample order, so a
    longer draw extends a shorter one (prefix stable): rows start .. start+n.
    """
    ss = np.random.SeedSequence([seed, WORKLOAD_IDS.get(name, 99), level])
    g = np.random.Generator(np.random.PCG64(ss))
    if WORKLOADS.get(name, {}).get("xi_dist", "normal") == "uniform":
        full = g.uniform(-1.0, 1.0, size=(start + n_samples, n_modes))
    else:
        full = g.standard_normal((start + n_samples, n_modes))
    return np.ascontiguousarray(full[start:])


def uniform_field(n, seed, lo=0.0, hi=1.0):
    """Seeded uniform values, e.g. test vectors or perturbed states."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
    return g.uniform(lo, hi, size=n)


def normal_field(shape, seed):
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    return g.standard_normal(shape)
