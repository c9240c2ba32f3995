"""Per-level smoother and team-size tuner with a JSON cache.

The slab operators M/dt + K - M diag f'(u) of a level have a spectrum set by
h and dt, so the best Jacobi sweep count K and Chebyshev interval ratio differ
between levels: more sweeps make each preconditioner application dearer but
cut Krylov (and, through the inexact-Newton forcing, Newton) iterations.  The
tuner solves a batch of samples of each level with every candidate (one
workgroup per sample, as in the MLMC launch), keeps the candidate with the
smallest mean workgroup-seconds per sample among those whose samples all
converge.  With that smoother it then measures the seconds per sample for
teams of G workgroups (a sample's space-time solve split over G workgroups):
the MLMC scheduler's starting cost model, refined by every later launch.
Choices and measurements go to a JSON file.  The conductivity fields come
from the level's KL modes with standard normal coefficients drawn from their
own seed, not from the workload's samples.

    python -m paper_1911_06066_amd.autotune --workload mlmc3_2d --out tuning.json

With --refine the choice is then checked on the whole MLMC estimate (refine).
"""

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_DIR = os.path.join(HERE, "tuning")

CANDIDATES = [(8, 10.0), (10, 10.0), (12, 10.0), (14, 10.0), (16, 10.0), (16, 20.0), (20, 10.0), (24, 10.0)]
# 3D levels measured faster with wider Chebyshev intervals (ratio 20 against
# 10 on the 65x65x17 slab), so their list spans ratios 10 to 30.
CANDIDATES_3D = [(8, 10.0), (12, 10.0), (8, 20.0), (12, 20.0), (16, 20.0), (24, 20.0), (12, 30.0), (16, 30.0),
                 (24, 30.0)]
TEAM_SIZES = (1, 2, 3, 4, 6, 8, 10, 12, 16, 24, 32)
MAX_TEAM = 32
LARGE_TEAM_SIZES = (8, 16, 24, 32)
# Levels of more than LARGE nodes x steps per sample (the finest 3D grids,
# about 90 workgroup-seconds per sample on one workgroup) are tuned on
# LARGE_SAMPLES samples solved by teams of the largest size, over a causal
# prefix of LARGE_PREFIX steps with the level's dt (the smoother's effect per
# slab does not depend on the horizon); their team table holds LARGE_TEAM_SIZES.
LARGE = 1e8
LARGE_SAMPLES = 4
LARGE_PREFIX = 128


def tuning_path(workload, precision):
    return os.path.join(TUNING_DIR, "%s_%s.json" % (workload, precision))


def _level_key(wl, l):
    return {"grid": list(wl["levels"][l]), "steps": int(wl["steps"][l])}


def tune(wl, precision=None, samples=32, candidates=None, seed=4242, block=0, log=print):
    """Measure every candidate on every level; return the tuning record."""
    import torch

    from . import Context, klmodes

    if candidates is None:
        candidates = CANDIDATES_3D if wl.get("dim", 2) == 3 else CANDIDATES

    precision = precision or wl.get("precision", "fp64")
    dev = torch.device("cuda:0")
    modes = [torch.from_numpy(m).to(dev) for m in klmodes.workload_modes(wl)]
    gen = torch.Generator().manual_seed(seed)
    M = wl["n_modes"]
    rec = {"workload": wl["name"], "precision": precision, "device": torch.cuda.get_device_name(0),
           "samples": samples, "seed": seed, "levels": []}
    counts = wl.get("samples")
    for l in range(len(wl["levels"])):
        S = max(2, min(samples, int(counts[l]) if counts else samples))
        m = int(wl["steps"][l])
        gmax = max(1, min(MAX_TEAM, int(wl["levels"][l][1]) // 3))
        large = float(np.prod(wl["levels"][l])) * m > LARGE
        wl_t, G_t, scale = wl, 1, 1.0
        if large:
            S, G_t = min(S, LARGE_SAMPLES), gmax
            k = min(m, LARGE_PREFIX)
            wl_t = dict(wl, steps=list(wl["steps"]), T=wl["T"] * k / m)
            wl_t["steps"][l] = k
            scale = m / k
        xi = torch.randn(S, M, generator=gen, dtype=torch.float64).to(dev)
        results = []
        for sweeps, ratio in candidates:
            tune_l = [None] * len(wl["levels"])
            tune_l[l] = (sweeps, ratio)
            over = dict(precision=precision, level_tuning=tune_l, team_size=G_t, max_lanes=S * G_t)
            if block:
                over["block_threads"] = block
            ctx = Context(wl_t, **over)
            sig = ctx.kl_synthesize(l, modes[l], xi)
            t0 = time.perf_counter()
            try:
                _, st = ctx.st_solve(l, sig)
                ok = all(s["status"] == 0 for s in st)
            except Exception as e:  # a candidate that fails to converge is skipped, not fatal
                log("level %d sweeps %d ratio %g: %s" % (l, sweeps, ratio, e))
                st, ok = [], False
            wall = time.perf_counter() - t0
            r = {"smooth_sweeps": sweeps, "cheb_ratio": ratio, "ok": ok, "wall_s": wall}
            if large:
                r["team"] = G_t
                r["prefix_steps"] = wl_t["steps"][l]
            if st:
                r["seconds_per_sample"] = scale * sum(s["device_seconds"] for s in st) / len(st)
                r["newton_per_sample"] = sum(s["newton_iters"] for s in st) / len(st)
                r["krylov_per_sample"] = sum(s["krylov_iters"] for s in st) / len(st)
            results.append(r)
            log("level %d %s" % (l, json.dumps(r)))
            ctx.close()
        good = [r for r in results if r["ok"]]
        best = min(good, key=lambda r: r["seconds_per_sample"]) if good else None
        entry = dict(_level_key(wl, l))
        entry["smooth_sweeps"] = best["smooth_sweeps"] if best else 0
        entry["cheb_ratio"] = best["cheb_ratio"] if best else 0.0
        entry["results"] = results
        # seconds per sample against team size, with the chosen smoother (a
        # large level: the full horizon at the large team sizes only)
        team = [0.0] * MAX_TEAM
        if best:
            tune_l = [None] * len(wl["levels"])
            tune_l[l] = (best["smooth_sweeps"], best["cheb_ratio"])
            for G in (LARGE_TEAM_SIZES if large else TEAM_SIZES):
                if G > gmax:
                    break
                over = dict(precision=precision, level_tuning=tune_l, team_size=G, max_lanes=S * G)
                if block:
                    over["block_threads"] = block
                ctx = Context(wl, **over)
                sig = ctx.kl_synthesize(l, modes[l], xi)
                try:
                    _, st = ctx.st_solve(l, sig)
                    team[G - 1] = sum(s["device_seconds"] for s in st) / len(st)
                except Exception as e:
                    log("level %d team %d: %s" % (l, G, e))
                ctx.close()
                log("level %d team %d: %.4f s per sample" % (l, G, team[G - 1]))
        entry["team_seconds"] = team
        rec["levels"].append(entry)
    return rec


def measure_teams(wl, rec, level, samples=None, seed=4343, log=print):
    """Re-measure one level's team table (seconds per sample against team
    size, full horizon) with the smoother the record holds for it."""
    import torch

    from . import Context, klmodes

    dev = torch.device("cuda:0")
    precision = rec["precision"]
    modes = torch.from_numpy(klmodes.workload_modes(wl)[level]).to(dev)
    M = wl["n_modes"]
    e = rec["levels"][level]
    m = int(wl["steps"][level])
    gmax = max(1, min(MAX_TEAM, int(wl["levels"][level][1]) // 3))
    large = float(np.prod(wl["levels"][level])) * m > LARGE
    S = samples or (LARGE_SAMPLES if large else 32)
    xi = torch.randn(S, M, generator=torch.Generator().manual_seed(seed), dtype=torch.float64).to(dev)
    tune_l = [None] * len(wl["levels"])
    tune_l[level] = (e["smooth_sweeps"], e["cheb_ratio"])
    team = list(e.get("team_seconds", [])) + [0.0] * MAX_TEAM
    team = team[:MAX_TEAM]
    for G in (LARGE_TEAM_SIZES if large else TEAM_SIZES):
        if G > gmax:
            break
        with Context(wl, precision=precision, level_tuning=tune_l, team_size=G, max_lanes=S * G) as ctx:
            sig = ctx.kl_synthesize(level, modes, xi)
            _, st = ctx.st_solve(level, sig)
        team[G - 1] = sum(s["device_seconds"] for s in st) / len(st)
        log("level %d team %d: %.4f s per sample" % (level, G, team[G - 1]))
    e["team_seconds"] = team
    return rec


def refine(wl, rec, modes, xi, steps=2, warmup=2, deltas=(-2, 2), log=print):
    """Check the per-level sweep counts on the whole MLMC estimate.

    Per-level times measured in isolation do not always carry over to the
    fused launch: samples of all levels share the chip, and the iteration
    counts can be sharply non-monotone in the sweep count.  Each level's count
    is moved by each of `deltas` in turn, finest level first, and a move is kept
    when the estimate's wall time per step falls by more than 1%.  modes[l],
    xi[l]: device inputs of the estimate, as in the benchmark.
    """
    import time

    import torch

    from . import Context

    N = list(wl["samples"])

    def measure(tun):
        ctx = Context(wl, precision=rec["precision"], level_tuning=tun)
        for _ in range(warmup):
            ctx.mlmc_estimate(N, modes, xi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.mlmc_estimate(N, modes, xi)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        ctx.close()
        return ms

    cur = [(e["smooth_sweeps"], e["cheb_ratio"], e["team_seconds"]) for e in rec["levels"]]
    best = measure(cur)
    trials = [{"sweeps": [c[0] for c in cur], "ms_per_step": best}]
    log("refine: %s %.1f ms per step" % ([c[0] for c in cur], best))
    for l in reversed(range(len(cur))):
        base = cur
        for d in deltas:
            k = base[l][0] + d
            if k < 1 or k > 32:
                continue
            cand = list(base)
            cand[l] = (k, base[l][1], None)  # team times of another sweep count do not apply
            try:
                ms = measure(cand)
            except Exception as e:
                log("refine: %s failed: %s" % ([c[0] for c in cand], e))
                continue
            trials.append({"sweeps": [c[0] for c in cand], "ms_per_step": ms})
            log("refine: %s %.1f ms per step" % ([c[0] for c in cand], ms))
            if ms < 0.99 * best:
                best, cur = ms, cand
    for e, c in zip(rec["levels"], cur):
        if e["smooth_sweeps"] != c[0]:
            # its team table was measured at the old sweep count: cleared, so
            # that the scheduler starts from its model and learns the times
            e["smooth_sweeps"] = c[0]
            e["team_seconds"] = [0.0] * MAX_TEAM
            e["team_seconds_note"] = "cleared: the refinement changed the sweep count"
    rec["refine"] = {"steps": steps, "warmup": warmup, "trials": trials, "ms_per_step": best}
    return rec


def level_tuning(wl, precision=None, path=None):
    """(sweeps, ratio, team_seconds) per level from a tuning file, or None
    when there is no file or it was measured for other grids."""
    precision = precision or wl.get("precision", "fp64")
    path = path or tuning_path(wl["name"], precision)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("precision") != precision or len(rec.get("levels", [])) != len(wl["levels"]):
        return None
    out = []
    for l, e in enumerate(rec["levels"]):
        if e["grid"] != list(wl["levels"][l]) or e["steps"] != int(wl["steps"][l]):
            return None
        out.append((int(e["smooth_sweeps"]), float(e["cheb_ratio"]), list(e.get("team_seconds", []))))
    return out


def main():
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    import stinputs

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="mlmc3_2d")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--samples", type=int, default=32)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--refine", action="store_true",
                    help="then check each level's sweep count (+-2) on the whole MLMC estimate")
    ap.add_argument("--teams-only", type=int, default=-1, metavar="LEVEL",
                    help="only re-measure this level's team table in the existing tuning file")
    a = ap.parse_args()
    wl = stinputs.workload(a.workload)
    if a.teams_only >= 0:
        precision = a.precision or wl.get("precision", "fp64")
        path = tuning_path(wl["name"], precision)
        # an existing output file accumulates the tables of several runs
        src = a.out if a.out and os.path.exists(a.out) else path
        with open(src) as f:
            rec = json.load(f)
        measure_teams(wl, rec, a.teams_only, log=lambda s: print(s, flush=True))
        out = a.out or path
        with open(out, "w") as f:
            json.dump(rec, f, indent=1)
        print("wrote", out, flush=True)
        return
    rec = tune(wl, a.precision, a.samples, block=a.block, log=lambda s: print(s, flush=True))
    if a.refine and wl.get("samples"):
        import torch

        from . import klmodes
        dev = torch.device("cuda:0")
        w = dict(wl, precision=rec["precision"])
        modes = [torch.from_numpy(m).to(dev) for m in klmodes.workload_modes(w)]
        xi = [torch.from_numpy(stinputs.xi(w["name"], l, n, w["n_modes"])).to(dev) for l, n in enumerate(w["samples"])]
        refine(w, rec, modes, xi, log=lambda s: print(s, flush=True))
    out = a.out or tuning_path(wl["name"], rec["precision"])
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", out, [(e["smooth_sweeps"], e["cheb_ratio"]) for e in rec["levels"]], flush=True)


if __name__ == "__main__":
    main()
