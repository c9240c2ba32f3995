"""Space-time multilevel Monte Carlo for the monodomain equation on MI355X.

Thin Python binding of the C library (include/stmlmc.h): argument marshalling
only.  Every step of the hot path -- KL synthesis, the nonlinear space-time
solves, activation maps and MLMC statistics -- runs in the library's HIP
kernels.  PyTorch provides device memory and the stream; the library fails
loudly when it has not been built.

    ctx = Context(workload_dict)
    sigma = ctx.kl_synthesize(level, modes, xi)
    u, stats = ctx.st_solve(level, sigma)
    t_act, censored = ctx.activation_map(level, u)
    out = ctx.mlmc_estimate(N, modes_per_level, xi_per_level)
"""

import ctypes
import sys

from . import _lib

__all__ = ["Context", "StmError", "problem_from_workload"]


class StmError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        self.code = _lib.STATUS.get(status, str(status))
        super().__init__("%s: %s" % (self.code, msg))


def _torch():
    import torch
    return torch


def problem_from_workload(wl, **overrides):
    """Fill an StmProblem from a workload description (plain dict)."""
    p = _lib.StmProblem()
    dim = int(wl["dim"])
    p.dim = dim
    L = list(wl["lengths"]) + [1.0] * (3 - dim)
    p.lx, p.ly, p.lz = L[0], L[1], L[2]
    p.T = wl["T"]
    p.k_react = wl["k_react"]
    p.a_react = wl["a_react"]
    p.sigma_f0 = wl["sigma_f0"]
    p.transverse_ratio = wl["transverse_ratio"]
    p.fiber_law = _lib.FIBER_LAWS[wl["fiber_law"]]
    c = list(wl["ic_center"]) + [0.0] * (3 - len(wl["ic_center"]))
    for i in range(3):
        p.ic_center[i] = c[i]
    p.ic_radius = wl["ic_radius"]
    p.threshold = wl["threshold"]
    levels = wl["levels"]
    p.n_levels = len(levels)
    for i, (shape, m) in enumerate(zip(levels, wl["steps"])):
        p.levels[i].nx = shape[0]
        p.levels[i].ny = shape[1]
        p.levels[i].nz = shape[2] if dim == 3 else 1
        p.levels[i].m = m
    for i, t in enumerate(overrides.pop("level_tuning", None) or []):
        if t is not None:
            p.levels[i].smooth_sweeps = int(t[0])
            p.levels[i].cheb_ratio = float(t[1])
            for g, sec in enumerate((t[2] if len(t) > 2 else None) or []):
                if g < 32:
                    p.levels[i].team_seconds[g] = float(sec)
    p.n_modes = wl["n_modes"]
    p.theta = wl.get("theta", 1.0)
    p.field_kind = _lib.FIELD_KINDS[wl.get("field", "lognormal")]
    p.tau_relative = int(wl.get("tau_relative", 0))
    p.ic_kind = _lib.IC_KINDS[wl.get("ic_kind", "ball")]
    p.qoi = _lib.QOIS[wl.get("qoi", "activation")]
    prec = overrides.pop("precision", wl.get("precision", "fp64"))
    p.precision = _lib.PRECISIONS[prec]
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _check_dev(t, name, dtype=None, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s" % (name, dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


class Context:
    """A library context for one problem on the current device and stream."""

    def __init__(self, wl, stream=None, **overrides):
        torch = _torch()
        self.lib = _lib.load()
        self.wl = dict(wl)
        self.problem = problem_from_workload(self.wl, **overrides)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = self.lib.stm_create(ctypes.byref(self.problem), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h))
        if st != 0:
            raise StmError(st, "stm_create failed (see stderr)")
        self.h = h
        self.sizes = [self.level_size(l) for l in range(self.problem.n_levels)]

    def close(self):
        """Release the library context (synchronises its stream).  Call it, or use
        the context as a `with` block, before the process exits: the library's
        HIP calls must not run while the interpreter and the HIP runtime shut
        down."""
        if getattr(self, "h", None):
            self.lib.stm_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        # During interpreter shutdown the HIP runtime may already be tearing
        # down (or a profiler's tool library finalising); an unclosed context
        # is then left to the process exit instead of calling into HIP.
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        if st != 0:
            raise StmError(st, self.lib.stm_last_error(self.h).decode())

    def timings(self):
        """Device phase times (ms) and algorithmic bytes of the last call."""
        t = _lib.StmTimings()
        self._raise(self.lib.stm_get_timings(self.h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in t._fields_}

    def level_size(self, level):
        n, e, m = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._raise(self.lib.stm_level_size(self.h, level, ctypes.byref(n), ctypes.byref(e), ctypes.byref(m)))
        return n.value, e.value, m.value

    # -- the four calls -----------------------------------------------------
    def kl_synthesize(self, level, modes, xi, out=None):
        torch = _torch()
        n, E, m = self.sizes[level]
        M = self.problem.n_modes
        _check_dev(modes, "modes", torch.float64, (E, M))
        S = xi.shape[0]
        _check_dev(xi, "xi", torch.float64, (S, M))
        if out is None:
            out = torch.empty((S, E), dtype=torch.float64, device=modes.device)
        _check_dev(out, "sigma", torch.float64, (S, E))
        self._raise(self.lib.stm_kl_synthesize(self.h, level, _ptr(modes), _ptr(xi), S, _ptr(out)))
        return out

    def st_solve(self, level, sigma, u0_guess=None, out=None, stats=True, noalloc=False):
        """noalloc: through stm_st_solve_noalloc (the library allocates no device
        memory; pass `out` to allocate none here either)."""
        torch = _torch()
        n, E, m = self.sizes[level]
        S = sigma.shape[0]
        _check_dev(sigma, "sigma", torch.float64, (S, E))
        if u0_guess is not None:
            _check_dev(u0_guess, "u0_guess", torch.float64, (S, m, n))
        if out is None:
            out = torch.empty((S, m, n), dtype=torch.float64, device=sigma.device)
        _check_dev(out, "u", torch.float64, (S, m, n))
        st_arr = (_lib.StmSolveStats * max(S, 1))() if stats else None
        fn = self.lib.stm_st_solve_noalloc if noalloc else self.lib.stm_st_solve
        st = fn(self.h, level, _ptr(sigma), _ptr(u0_guess), S, _ptr(out), st_arr if stats else None)
        self._raise(st)
        if not stats:
            return out, None
        return out, [dict(status=s.status, newton_max_per_slab=s.newton_max_per_slab,
                          newton_iters=s.newton_iters, krylov_iters=s.krylov_iters,
                          final_step=s.final_step, device_seconds=s.device_seconds,
                          algorithmic_bytes=s.algorithmic_bytes, model_bytes=s.model_bytes,
                          damped_steps=s.damped_steps,
                          phase_seconds=list(s.phase_seconds))
                     for s in st_arr[:S]]

    def activation_map(self, level, u, out=None):
        torch = _torch()
        n, E, m = self.sizes[level]
        S = u.shape[0]
        _check_dev(u, "u", torch.float64, (S, m, n))
        if out is None:
            out = torch.empty((S, n), dtype=torch.float64, device=u.device)
        _check_dev(out, "t_act", torch.float64, (S, n))
        cen = (ctypes.c_int * max(S, 1))()
        self._raise(self.lib.stm_activation_map(self.h, level, _ptr(u), S, _ptr(out), cen))
        return out, list(cen[:S])

    def prolong_st(self, level, u_coarse, out=None):
        """Space-time prolongation of level-1 solutions (S, m_{l-1}, n_{l-1}) to level."""
        torch = _torch()
        nc, _, mc = self.sizes[level - 1]
        nf, _, mf = self.sizes[level]
        S = u_coarse.shape[0]
        _check_dev(u_coarse, "u_coarse", torch.float64, (S, mc, nc))
        if out is None:
            out = torch.empty((S, mf, nf), dtype=torch.float64, device=u_coarse.device)
        _check_dev(out, "u_fine", torch.float64, (S, mf, nf))
        self._raise(self.lib.stm_prolong_st(self.h, level, _ptr(u_coarse), S, _ptr(out)))
        return out

    def mlmc_estimate(self, N, modes, xi, capacity=None, target_rmse=0.0, pilot=0, level_fields=True):
        """N: samples per level (None = adaptive).  modes[l]: (E_l, M); xi[l]: (cap_l, M)."""
        torch = _torch()
        L1 = self.problem.n_levels
        M = self.problem.n_modes
        nL = self.sizes[-1][0]
        for l in range(L1):
            _check_dev(modes[l], "modes[%d]" % l, torch.float64, (self.sizes[l][1], M))
            _check_dev(xi[l], "xi[%d]" % l, torch.float64, (xi[l].shape[0], M))
        dev = modes[0].device
        P = nL * (self.sizes[-1][2] if self.problem.qoi == _lib.QOIS["spacetime"] else 1)
        mean = torch.empty(P, dtype=torch.float64, device=dev)
        var = torch.empty(P, dtype=torch.float64, device=dev)
        lmean = torch.empty((L1, P), dtype=torch.float64, device=dev) if level_fields else None
        lvar = torch.empty((L1, P), dtype=torch.float64, device=dev) if level_fields else None
        res = _lib.StmMlmcResult()
        res.mean, res.var = mean.data_ptr(), var.data_ptr()
        res.level_mean = lmean.data_ptr() if lmean is not None else None
        res.level_var = lvar.data_ptr() if lvar is not None else None
        mp = (ctypes.c_void_p * L1)(*[m.data_ptr() for m in modes])
        xp = (ctypes.c_void_p * L1)(*[x.data_ptr() for x in xi])
        cap = (ctypes.c_int * L1)(*[(capacity[l] if capacity is not None else xi[l].shape[0]) for l in range(L1)])
        Np = (ctypes.c_int * L1)(*N) if N is not None else None
        self._raise(self.lib.stm_mlmc_estimate(self.h, Np, mp, xp, cap, float(target_rmse), int(pilot),
                                               ctypes.byref(res)))
        return dict(mean=mean, var=var, level_mean=lmean, level_var=lvar,
                    N=list(res.N[:L1]), V=list(res.V[:L1]), cost=list(res.cost[:L1]),
                    bias_estimate=res.bias_estimate, newton_iters=res.newton_iters,
                    krylov_iters=res.krylov_iters, censored=res.censored, rounds=res.rounds,
                    worst_status=res.worst_status, algorithmic_bytes=res.algorithmic_bytes,
                    model_bytes=res.model_bytes, dof_steps=res.dof_steps)
