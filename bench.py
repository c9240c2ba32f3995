#!/usr/bin/env python3
"""Benchmark: one MLMC estimate of the activation-map mean and variance per step.

A step is one pass of the whole hot path over one batch of synthetic input:
KL synthesis of every sample's conductivity (fine and coarse member of each
pair), the nonlinear space-time solve of every sample, the activation maps,
and the MLMC mean/variance accumulation.  Inputs (KL modes, KL coefficients)
are resident on the GPU before the timed region.

Prints one JSON line.  Default workload: the five-level 3D MLMC
(9x9x3 ... 129x129x33 nodes, 32 ... 512 steps, 128 KL modes, mixed
precision) whose sample counts are set adaptively for an RMSE of 1e-3 T.
The adaptive rounds (pilot samples, then the optimal-allocation rule) run
once before the timed region; every warm-up and timed step is then the
estimate at the counts they found -- the same samples, so the same RMSE.
Fixed-count workloads (--workload mlmc3_2d, ...) time their own counts.
The library's scheduler prices samples from what its earlier launches
measured, and its estimates settle after two warm-up steps.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL = "st_team_kernel"


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the HIP sources the solver kernel is built from."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1911_06066_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload):
    """HBM bytes per launch of the solver kernel from the committed counter summary.

    The summary holds FETCH_SIZE + WRITE_SIZE of the solver launch scaled by the
    same counters on a copy of known size.  Returns None when no summary exists
    for the workload or the kernel sources changed since it was taken.
    """
    path = os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.md" % (KERNEL, workload))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("#", "|", "*", " ")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def _oracle_worker(args):
    """One oracle sample on a causal prefix of k slabs (same dt): KL field,
    space-time Newton/SuperLU, activation map (CPU, FP64).  Returns seconds."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    wl, level, modes, xi, k = args
    import oracle.api as oapi
    wp = dict(wl)
    wp["steps"] = list(wl["steps"])
    wp["T"] = wl["T"] * k / wl["steps"][level]
    wp["steps"][level] = k
    sig = oapi.kl_synthesize(modes, xi[None, :], wl["sigma_f0"], wl.get("field", "lognormal"))
    t0 = time.perf_counter()
    U, _ = oapi.st_solve(wp, level, sig, mode="timestep")
    oapi.activation_map(wp, level, U)
    return time.perf_counter() - t0


def cpu_baseline(wl, modes, N, budget_s):
    """The oracle timed on a bounded sample of every level of the workload.

    Per level, one sample's causal prefix of k slabs (same dt; k doubled from
    1 while it stays within half the level's share of the budget, at most the
    whole horizon) runs on one core, then `cores` copies of it run at once on
    a pool of `cores` processes: seconds per slab on one core and, from the
    pool's wall time, per slab and core with every core busy.  Scaled by the
    level's steps they give seconds per sample.  A level whose single slab
    would exceed its share (the two finest 3D grids: a sparse LU of 70k-550k
    unknowns per Newton step) is not run; its seconds per slab are extrapolated
    from the two finest measured levels by the growth of seconds per node and
    slab, and the result names it.  The estimate's CPU time is
    sum_l N_l (t_l + t_{l-1}); `cores` is the host's CPU share per GPU (at
    most 16 processes).
    """
    import multiprocessing as mp
    import numpy as np
    import stinputs
    cores = max(1, min(16, os.cpu_count() or 1))
    L1 = len(wl["levels"])
    share = budget_s / L1
    xi = stinputs.xi(wl["name"], 0, 1, wl["n_modes"])[0]
    nodes = [int(np.prod(s)) for s in wl["levels"]]
    one, full, prefix = [None] * L1, [None] * L1, [0] * L1
    with mp.get_context("spawn").Pool(cores) as pool:
        for l in range(L1):
            m = wl["steps"][l]
            if l >= 2 and one[l - 1] is not None and one[l - 1] * nodes[l] / nodes[l - 1] > share / 2:
                break
            k, t = 1, _oracle_worker((wl, l, modes[l], xi, 1))
            while k < m and t * 2 <= share / 2:
                k = min(m, 2 * k)
                t = _oracle_worker((wl, l, modes[l], xi, k))
            one[l] = t / k
            prefix[l] = k
            t0 = time.perf_counter()
            pool.map(_oracle_worker, [(wl, l, modes[l], xi, k)] * cores)
            full[l] = (time.perf_counter() - t0) / (cores * k)
    known = [l for l in range(L1) if one[l] is not None]
    a, b = known[-2], known[-1]
    growth = (one[b] / nodes[b]) / (one[a] / nodes[a])  # per node and slab, per refinement
    for l in range(L1):
        if one[l] is None:
            one[l] = one[l - 1] * nodes[l] / nodes[l - 1] * growth
            full[l] = full[l - 1] * nodes[l] / nodes[l - 1] * growth

    def estimate_seconds(per_slab):
        t = [per_slab[l] * wl["steps"][l] for l in range(L1)]
        return sum(N[l] * (t[l] + (t[l - 1] if l > 0 else 0.0)) for l in range(L1))

    samples = float(sum(N))
    t1, tc = estimate_seconds(one), estimate_seconds(full)
    skipped = [l for l in range(L1) if l not in known]
    return {
        "value": samples / tc,
        "unit": "MLMC samples/s",
        "cores": cores,
        "kind": "oracle",
        "value_1core": samples / t1,
        "sample": "one sample per level, causal prefix of %s slabs (same dt), KL + Newton/SuperLU + activation; "
                  "seconds per slab %s on one core and %s of wall time per slab with %d processes each solving "
                  "one; levels %s not run (one slab above the level's %.0f s share), extrapolated by the "
                  "measured growth x%.2f of seconds per node and slab per refinement; the estimate's %d samples "
                  "(N_l %s, fine and coarse member each) take %.4g s of wall time on %d cores, %.4g s on one"
                  % (prefix, ["%.3g" % v for v in one], ["%.3g" % v for v in full], cores,
                     skipped or "none", share, growth, int(samples), list(N), tc, cores, t1),
        "extrapolated_levels": skipped,
    }


def warm_starts(wl, modes, xi, k=4):
    """First Newton iterates on the finest level, one workgroup per sample:
    the previous sample's solution (one lane solving k samples in turn), the
    space-time prolongation of the pair's coarse solution (Sec. 3.4), and the
    initial state (cold).  Per-sample Newton and Krylov iterations and device
    seconds (the coarse solve and the prolongation are reported apart)."""
    import torch

    from paper_1911_06066_amd import Context

    L = len(wl["levels"]) - 1
    y = xi[L][:k + 1].contiguous()
    out = {"samples": k, "level": L}

    def summary(st):
        return {"newton_per_sample": sum(s["newton_iters"] for s in st) / len(st),
                "krylov_per_sample": sum(s["krylov_iters"] for s in st) / len(st),
                "seconds_per_sample": sum(s["device_seconds"] for s in st) / len(st)}

    from paper_1911_06066_amd import autotune
    tun = autotune.level_tuning(wl, wl["precision"])
    over = {"level_tuning": tun} if tun else {}
    with Context(wl, max_lanes=1, team_size=1, **over) as one, Context(wl, max_lanes=k, team_size=1, **over) as many:
        sf_all = many.kl_synthesize(L, modes[L], y)
        _, st = one.st_solve(L, sf_all)
        out["previous_sample"] = summary(st[1:])  # the lane's first sample starts cold
        sf = sf_all[1:].contiguous()
        sc = many.kl_synthesize(L - 1, modes[L - 1], y[1:].contiguous())
        uc, stc = many.st_solve(L - 1, sc)
        guess = many.prolong_st(L, uc)
        torch.cuda.synchronize()
        pro_ms = many.timings()["stats_ms"]
        _, st = many.st_solve(L, sf, u0_guess=guess)
        out["prolonged_coarse"] = summary(st)
        out["prolonged_coarse"]["coarse_seconds_per_sample"] = summary(stc)["seconds_per_sample"]
        out["prolonged_coarse"]["prolongation_ms"] = pro_ms
        _, st = many.st_solve(L, sf)
        out["initial_state"] = summary(st)
    return out


def compare_paths(wl, N, modes, xi, value, out, tuning_by_precision):
    """The same MLMC estimate (same samples, so the same RMSE) through

    * the batched path in the other precision (float64 for a mixed-precision
      workload, mixed for a float64 one): one persistent launch per step;
    * the plain float64 single-sample path: one stm_st_solve call per sample
      (the library picks the sample's team), timed on a few pairs of each
      level (one on 3D levels) and scaled to the workload's sample counts.

    The mixed estimate's deviation from the float64 one is reported next to
    the estimator's sampling error sqrt(sum_l V_l / N_l): max-norm of the mean
    difference (absolute, against 1e-6 T) and of the variance difference
    relative to the variance's max-norm and 2-norm (against 1e-4).  Outside the
    timed region of the main measurement.
    """
    import numpy as np
    import torch

    from paper_1911_06066_amd import Context

    res = {}
    other = "fp64" if wl["precision"] == "mixed" else "mixed"
    wlo = dict(wl, precision=other)
    tun = tuning_by_precision(other)
    heavy = wl["dim"] == 3
    with Context(wlo, **({"level_tuning": tun} if tun else {})) as ctx:
        for _ in range(1 if heavy else 2):  # warm-up: the schedule settles from measured launches
            oo = ctx.mlmc_estimate(N, modes, xi)
        torch.cuda.synchronize()
        steps = 1 if heavy else 3
        t0 = time.perf_counter()
        for _ in range(steps):
            oo = ctx.mlmc_estimate(N, modes, xi)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
    other_value = float(sum(N)) / (ms / 1e3)
    progress("%s batched: %.1f ms per step" % (other, ms))
    mixed, fp64 = (out, oo) if wl["precision"] == "mixed" else (oo, out)
    dv = (mixed["var"] - fp64["var"]).double()
    err = {"mean_abs_maxnorm": float((mixed["mean"] - fp64["mean"]).abs().max()),
           "mean_abs_tolerance": 1e-6 * wl["T"],
           "var_rel_maxnorm": float(dv.abs().max() / fp64["var"].abs().max()),
           "var_rel_2norm": float(dv.norm() / fp64["var"].norm()),
           "var_tolerance": 1e-4,
           "sampling_rmse": float(np.sqrt(sum(v / n for v, n in zip(fp64["V"], N))))}
    res["%s_batched" % other] = {"value": other_value, "ms_per_step": ms, "steps": steps,
                                 "smoother_per_level": [list(t[:2]) for t in tun] if tun else "defaults"}
    res["mixed_vs_fp64_error"] = err
    # plain float64, one sample per call
    tun64 = tuning_by_precision("fp64")
    wl64 = dict(wl, precision="fp64")
    per = []
    k = 1 if heavy else 3
    with Context(wl64, **({"level_tuning": tun64} if tun64 else {})) as ctx1:
        sig = ctx1.kl_synthesize(0, modes[0], xi[0][:1].contiguous())
        ctx1.st_solve(0, sig, stats=False)  # warm-up (module load, first launch)
        for l in range(len(N)):
            tl = 0.0
            for lv in ([l, l - 1] if l > 0 else [l]):
                sig = ctx1.kl_synthesize(lv, modes[lv], xi[l][:k].contiguous())
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for i in range(k):
                    u, _ = ctx1.st_solve(lv, sig[i:i + 1].contiguous(), stats=False)
                    ctx1.activation_map(lv, u)
                    del u
                torch.cuda.synchronize()
                tl += (time.perf_counter() - t0) / k
            per.append(tl)
            progress("single-sample float64 path, level %d: %.3f s per pair" % (l, tl))
    total = float(np.dot(per, N))
    single_value = float(sum(N)) / total
    res["fp64_single_sample"] = {"value": single_value, "seconds_per_pair": per,
                                 "sample": "%d pair(s) per level, one st_solve call per sample, scaled to N" % k}
    if not heavy:
        res["warm_start_finest"] = warm_starts(wl, modes, xi)
    mixed_value = value if wl["precision"] == "mixed" else other_value
    fp64_value = other_value if wl["precision"] == "mixed" else value
    res["mixed_batched_over_fp64_single"] = mixed_value / single_value
    res["fp64_batched_over_fp64_single"] = fp64_value / single_value
    res["mixed_batched_over_fp64_batched"] = mixed_value / fp64_value
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mlmc5_3d")
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--max-lanes", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=24.0, help="seconds of oracle work (0 = skip)")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the per-level smoother tuning file")
    ap.add_argument("--st-mode", default="slab", choices=["slab", "global"],
                    help="slab: Newton slab by slab (default); global: Newton on the whole space-time "
                         "system with one GMRES over all slabs")
    ap.add_argument("--compare", type=int, default=1,
                    help="also time the batched path in the other precision and the single-sample float64 "
                         "path (0 = skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus %d is not supported" % args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import stinputs
    from paper_1911_06066_amd import Context, autotune, klmodes

    dev = torch.device("cuda:0")
    wl = stinputs.workload(args.workload)
    if args.precision:
        wl["precision"] = args.precision
    M = wl["n_modes"]
    modes_h = klmodes.workload_modes(wl)
    modes = [torch.from_numpy(m).to(dev) for m in modes_h]

    def tuning_by_precision(prec):
        return None if args.no_tuning else autotune.level_tuning(wl, prec)

    over = {}
    tuning = tuning_by_precision(wl["precision"])
    if tuning:
        over["level_tuning"] = tuning
    if args.max_lanes:
        over["max_lanes"] = args.max_lanes
    if args.block:
        over["block_threads"] = args.block
    if args.st_mode == "global":
        over["st_mode"] = 1
    allocation = None
    with Context(wl, **over) as ctx:
        if wl["samples"] is None:
            # adaptive counts: pilot rounds and the optimal allocation, once,
            # before the timed region; the steps then estimate at the counts found
            cap = list(wl["capacity"])
            xi = [torch.from_numpy(stinputs.xi(wl["name"], l, cap[l], M)).to(dev) for l in range(len(cap))]
            t0 = time.perf_counter()
            progress("adaptive allocation for RMSE %g T, pilot %d" % (wl["target_rmse"], wl["pilot"]))
            a = ctx.mlmc_estimate(None, modes, xi, capacity=cap, target_rmse=wl["target_rmse"] * wl["T"],
                                  pilot=wl["pilot"])
            torch.cuda.synchronize()
            N = list(a["N"])
            progress("allocation N = %s in %d rounds, %.1f s" % (N, a["rounds"], time.perf_counter() - t0))
            allocation = {"target_rmse": wl["target_rmse"] * wl["T"], "pilot": wl["pilot"], "capacity": cap,
                          "rounds": a["rounds"], "N": N, "V": a["V"], "cost_s": a["cost"],
                          "variance_part_of_mse": float(sum(v / n for v, n in zip(a["V"], N) if n > 0)),
                          "bias_estimate": a["bias_estimate"], "seconds": time.perf_counter() - t0}
            xi = [x[:n].contiguous() for x, n in zip(xi, N)]
        else:
            N = list(wl["samples"])
            xi = [torch.from_numpy(stinputs.xi(wl["name"], l, N[l], M)).to(dev) for l in range(len(N))]

        for i in range(args.warmup):
            ctx.mlmc_estimate(N, modes, xi)
            progress("warm-up step %d/%d" % (i + 1, args.warmup))
        torch.cuda.synchronize()
        solve_ms, solve_bytes, model_bytes = [], [], []
        t0 = time.perf_counter()
        for i in range(args.steps):
            out = ctx.mlmc_estimate(N, modes, xi)
            tm = ctx.timings()
            solve_ms.append(tm["solve_ms"])
            solve_bytes.append(tm["solve_bytes"])
            model_bytes.append(tm["solve_bytes_model"])
            progress("step %d/%d: %.1f ms in the solver" % (i + 1, args.steps, tm["solve_ms"]))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    samples = float(sum(N))
    value = samples / (ms / 1e3)
    dof_steps = float(out["dof_steps"])
    kernel_s = float(np.mean(solve_ms)) * 1e-3
    achieved = float(np.mean(model_bytes)) / kernel_s / 1e9
    achieved_fused = float(np.mean(solve_bytes)) / kernel_s / 1e9
    default_cfg = not (args.precision or args.max_lanes or args.block or args.no_tuning or args.st_mode != "slab")
    traffic = profiled_traffic(wl["name"]) if default_cfg else None

    line = {
        "metric": "MLMC samples/sec & DOF*steps/s at fixed RMSE; stencil HBM GB/s vs peak",
        "value": value,
        "unit": "MLMC samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl["precision"] == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": wl["name"],
            "levels": [list(s) for s in wl["levels"]],
            "time_steps": wl["steps"],
            "samples_per_level": N,
            "sample_counts": ("adaptive: set before the timed region for RMSE %g T (pilot %d per level), then "
                              "fixed" % (wl["target_rmse"], wl["pilot"])) if allocation else "fixed",
            "kl_modes": M,
            "precision": wl["precision"],
            "parallelism": "single GPU, one workgroup team per sample",
            "smoother_per_level": [list(t[:2]) for t in tuning] if tuning else "defaults",
            "st_mode": args.st_mode,
        },
        "dof_steps_per_s": dof_steps / (ms / 1e3),
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": KERNEL,
            "kernel_ms": float(np.mean(solve_ms)),
            "algorithmic_bytes_per_launch": float(np.mean(model_bytes)),
            "bytes_model": "per node: 4 float64 words per Newton residual; per Krylov iteration j 4 (Jacobian "
                           "product) + 5 per smoother sweep + 2j + 3 (Arnoldi) inner words",
            "achieved_fused_passes": achieved_fused,
            "fused_passes_note": "the same launch with a fused smoother pass counted as one pass",
        },
        "detail": {
            "kl_ms": tm["kl_ms"], "solve_ms": tm["solve_ms"], "stats_ms": tm["stats_ms"],
            "teams": tm["solve_teams"], "workgroups": tm["solve_blocks"], "block": tm["solve_block"],
            "newton_iters": out["newton_iters"], "krylov_iters": out["krylov_iters"],
            "algorithmic_bytes": out["model_bytes"], "censored_nodes": out["censored"],
            "V": out["V"], "cost_s": out["cost"], "bias_estimate": out["bias_estimate"],
        },
    }
    if allocation:
        line["detail"]["allocation"] = allocation
    if args.compare:
        progress("comparison paths")
        line["detail"]["comparison"] = compare_paths(wl, N, modes, xi, value, out, tuning_by_precision)
    if args.cpu_budget > 0:
        progress("oracle baseline on the host")
        line["cpu_baseline"] = cpu_baseline(wl, modes_h, N, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
