#!/usr/bin/env python3
"""Benchmark: one MLMC estimate of the activation-map mean and variance per step.

A step is one pass of the whole hot path over one batch of synthetic input:
KL synthesis of every sample's conductivity (fine and coarse member of each
pair), the nonlinear space-time solve of every sample, the activation maps,
and the MLMC mean/variance accumulation.  Inputs (KL modes, KL coefficients)
are resident on the GPU before the timed region.

Prints one JSON line.  Default workload: the three-level float64 MLMC
(33^2/65^2/129^2 grids, 64/128/256 steps, 512/128/32 pairs, 32 KL modes).
Two untimed warm-up steps by default: the library's scheduler prices samples
from what its earlier launches measured, and its estimates settle after two.
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
    """One oracle sample: KL field, space-time solve, activation map (CPU, FP64)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    wl, level, modes, xi = args
    import oracle.api as oapi
    sig = oapi.kl_synthesize(modes, xi[None, :], wl["sigma_f0"])
    t0 = time.perf_counter()
    U, _ = oapi.st_solve(wl, level, sig)
    oapi.activation_map(wl, level, U)
    return time.perf_counter() - t0


def cpu_baseline(wl, modes, N, total_dof_steps, budget_s):
    """Time the oracle on a bounded sample of the workload's coarsest-level solves.

    The rate is measured in solved dof*steps per second and converted to the
    workload's MLMC samples per second (samples / total dof*steps of a step).
    """
    import multiprocessing as mp
    import numpy as np
    import stinputs
    cores = max(1, min(16, os.cpu_count() or 1))
    n = wl["levels"][0]
    nodes = int(np.prod(n))
    m = wl["steps"][0]
    xi = stinputs.xi(wl["name"], 0, 64, wl["n_modes"])
    # one probe sample fixes the count that fits the budget
    t_one = _oracle_worker((wl, 0, modes[0], xi[0]))
    per_core = max(1, int(budget_s / max(t_one, 1e-3) / cores))
    count = min(64, per_core * cores)
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        times = pool.map(_oracle_worker, [(wl, 0, modes[0], xi[i % 64]) for i in range(count)])
    wall = time.perf_counter() - t0
    rate = count * nodes * m / wall
    samples = float(sum(N))
    return {
        "value": rate * samples / total_dof_steps,
        "unit": "MLMC samples/s (from oracle dof*steps/s)",
        "cores": cores,
        "kind": "oracle",
        "sample": "%d level-0 solves (%s nodes x %d steps, KL + Newton/SuperLU + activation) on %d "
                  "processes, %.1f s wall, %.1f s CPU; converted via the workload's %d samples / %.4g dof*steps"
                  % (count, "x".join(map(str, n)), m, cores, wall, sum(times), int(samples), total_dof_steps),
        "dof_steps_per_s": rate,
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
    one = Context(wl, max_lanes=1, team_size=1, **over)
    many = Context(wl, max_lanes=k, team_size=1, **over)
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


def compare_paths(wl, N, modes, xi, fp64_value, fp64_out):
    """The same MLMC estimate (same samples, so the same RMSE) through

    * the batched mixed-precision path: one persistent launch, float32 Krylov
      and multigrid vectors and split-f16 KL inside float64 Newton;
    * the plain float64 single-sample path: one stm_st_solve call per sample
      (the library picks the sample's team), timed on a few samples of each
      level and scaled to the workload's sample counts.

    The mixed estimate's deviation from the float64 one (max-norm of the
    mean and variance fields, relative to their max-norm) is reported next
    to the estimator's sampling error sqrt(sum_l V_l / N_l).  Outside the
    timed region of the main measurement.
    """
    import numpy as np
    import torch

    from paper_1911_06066_amd import Context, autotune

    out = {}
    wlm = dict(wl, precision="mixed")
    tun = autotune.level_tuning(wl, "mixed")
    ctx = Context(wlm, **({"level_tuning": tun} if tun else {}))
    for _ in range(2):  # warm-up, as for the main measurement: the schedule settles after two
        mo = ctx.mlmc_estimate(N, modes, xi)
    torch.cuda.synchronize()

    def rel(a, b):
        return float((a - b).abs().max() / b.abs().max())

    err = {"mean_rel_maxnorm": rel(mo["mean"], fp64_out["mean"]),
           "var_rel_maxnorm": rel(mo["var"], fp64_out["var"]),
           "mean_abs_maxnorm": float((mo["mean"] - fp64_out["mean"]).abs().max()),
           "sampling_rmse": float(np.sqrt(sum(v / n for v, n in zip(fp64_out["V"], N))))}
    steps = 3
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.mlmc_estimate(N, modes, xi)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    mixed_value = float(sum(N)) / (ms / 1e3)
    out["mixed_batched"] = {"value": mixed_value, "ms_per_step": ms,
                            "smoother_per_level": [list(t[:2]) for t in tun] if tun else "defaults",
                            "error_vs_fp64": err}
    # plain float64, one sample per call
    ctx1 = Context(wl)
    per = []
    k = 3
    for l in range(len(N)):
        tl = 0.0
        for lv in ([l, l - 1] if l > 0 else [l]):
            sig = ctx1.kl_synthesize(lv, modes[lv], xi[l][:k].contiguous())
            ctx1.st_solve(lv, sig[:1].contiguous(), stats=False)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(k):
                u, _ = ctx1.st_solve(lv, sig[i:i + 1].contiguous(), stats=False)
                ctx1.activation_map(lv, u)
            torch.cuda.synchronize()
            tl += (time.perf_counter() - t0) / k
        per.append(tl)
    total = float(np.dot(per, N))
    single_value = float(sum(N)) / total
    out["fp64_single_sample"] = {"value": single_value, "seconds_per_pair": per,
                                 "sample": "%d pairs per level, one st_solve call per sample, scaled to N" % k}
    out["warm_start_finest"] = warm_starts(wl, modes, xi)
    out["mixed_batched_over_fp64_single"] = mixed_value / single_value
    out["fp64_batched_over_fp64_single"] = fp64_value / single_value
    out["mixed_batched_over_fp64_batched"] = mixed_value / fp64_value
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mlmc3_2d")
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--max-lanes", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work (0 = skip)")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the per-level smoother tuning file")
    ap.add_argument("--compare", type=int, default=1,
                    help="also time the batched mixed-precision path and the single-sample float64 path (0 = skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus %d is not supported" % args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import stinputs
    from paper_1911_06066_amd import Context, klmodes

    dev = torch.device("cuda:0")
    wl = stinputs.workload(args.workload)
    if args.precision:
        wl["precision"] = args.precision
    N = list(wl["samples"])
    M = wl["n_modes"]
    modes_h = klmodes.workload_modes(wl)
    modes = [torch.from_numpy(m).to(dev) for m in modes_h]
    xi = [torch.from_numpy(stinputs.xi(wl["name"], l, N[l], M)).to(dev) for l in range(len(N))]
    over = {}
    from paper_1911_06066_amd import autotune
    tuning = None if args.no_tuning else autotune.level_tuning(wl, wl["precision"])
    if tuning:
        over["level_tuning"] = tuning
    if args.max_lanes:
        over["max_lanes"] = args.max_lanes
    if args.block:
        over["block_threads"] = args.block
    ctx = Context(wl, **over)

    for _ in range(args.warmup):
        ctx.mlmc_estimate(N, modes, xi)
    torch.cuda.synchronize()
    solve_ms, solve_bytes = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.mlmc_estimate(N, modes, xi)
        tm = ctx.timings()
        solve_ms.append(tm["solve_ms"])
        solve_bytes.append(tm["solve_bytes"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    samples = float(sum(N))
    value = samples / (ms / 1e3)
    dof_steps = float(out["dof_steps"])
    achieved = float(np.mean(solve_bytes)) / (float(np.mean(solve_ms)) * 1e-3) / 1e9
    default_cfg = not (args.precision or args.max_lanes or args.block or args.no_tuning)
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
            "kl_modes": M,
            "precision": wl["precision"],
            "parallelism": "single GPU, one workgroup team per sample",
            "smoother_per_level": [list(t[:2]) for t in tuning] if tuning else "defaults",
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
        },
        "detail": {
            "kl_ms": tm["kl_ms"], "solve_ms": tm["solve_ms"], "stats_ms": tm["stats_ms"],
            "teams": tm["solve_teams"], "workgroups": tm["solve_blocks"], "block": tm["solve_block"],
            "newton_iters": out["newton_iters"], "krylov_iters": out["krylov_iters"],
            "algorithmic_bytes": out["algorithmic_bytes"], "censored_nodes": out["censored"],
            "V": out["V"], "cost_s": out["cost"],
        },
    }
    if args.compare and wl["precision"] == "fp64":
        line["detail"]["comparison"] = compare_paths(wl, N, modes, xi, value, out)
    if args.cpu_budget > 0:
        line["cpu_baseline"] = cpu_baseline(wl, modes_h, N, dof_steps, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
