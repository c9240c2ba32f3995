"""Controlled-convergence study of MC and MLMC in 1D+1 (Sec. 4.1, Table 1).

For each finest level L the MC estimator uses N_L = 16^L samples of level L
and the MLMC estimator N_0 = 16^L samples on level 0 and 16 times fewer on
each finer level (at least 2), both of E[u] on level L's space-time grid.  The
error e = v_L - v_ref against a reference mean v_ref (MC on the finest level)
is measured in L^2(0, T; L^2(D)), and the root mean square over R independent
repetitions is reported together with the work (solver workgroup-seconds).
Every estimate runs through the library's space-time QoI path.

    python -m paper_1911_06066_amd.study1d --reference 20000 --repeats 8
"""

import argparse
import json
import os
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="cable1d")
    ap.add_argument("--reference", type=int, default=20000)
    ap.add_argument("--repeats", type=int, default=8)
    ap.add_argument("--levels", type=int, default=0,
                    help="number of levels to study (default: all); the reference is always MC on the finest")
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import stinputs
    from paper_1911_06066_amd import Context, klmodes

    wl = stinputs.workload(a.workload)
    if wl.get("qoi") != "spacetime":
        raise SystemExit("the study needs a workload with the space-time QoI")
    dev = torch.device("cuda:0")
    Lmax = len(wl["levels"]) - 1  # the reference level
    Lstudy = (a.levels or len(wl["levels"])) - 1
    modes_all = [torch.from_numpy(m).to(dev) for m in klmodes.workload_modes(wl)]
    M = wl["n_modes"]

    def sub(L):  # the workload cut at level L (coarse levels 0 .. L)
        return dict(wl, levels=wl["levels"][:L + 1], steps=wl["steps"][:L + 1])

    def weights(L):
        w = sub(L)
        nx, ny = w["levels"][L]
        hx, hy = w["lengths"][0] / (nx - 1), w["lengths"][1] / (ny - 1)
        wx = np.full(nx, hx)
        wx[[0, -1]] *= 0.5
        wy = np.full(ny, hy)
        wy[[0, -1]] *= 0.5
        m = w["steps"][L]
        dt = w["T"] / m
        wt = np.full(m, dt)
        wt[-1] *= 0.5
        return (wt[:, None] * np.outer(wy, wx).ravel()[None, :]).ravel()

    def estimate(L, N, seed, single_level):
        """Mean field on level L's space-time grid and the solver work."""
        if single_level:  # plain MC on level L: a one-level workload whose level is L
            w = dict(wl, levels=[wl["levels"][L]], steps=[wl["steps"][L]])
            modes = [modes_all[L]]
        else:
            w = sub(L)
            modes = modes_all[:L + 1]
        ctx = Context(w)
        xi = [torch.from_numpy(stinputs.xi(wl["name"], l + (L if single_level else 0), N[l], M, seed=seed)).to(dev)
              for l in range(len(N))]
        out = ctx.mlmc_estimate(N, modes, xi, level_fields=False)
        work = float(sum(n * c for n, c in zip(out["N"], out["cost"])))
        mean = out["mean"].cpu().numpy()
        ctx.close()
        return mean, work

    # reference: plain MC on the finest level
    vref, wref = estimate(Lmax, [a.reference], 99991, True)
    print(json.dumps({"reference": {"level": Lmax, "samples": a.reference, "work_s": wref}}), flush=True)
    for L in range(Lstudy + 1):
        # the reference restricted to level L's space-time points: nested in space and time
        nxL, nyL = wl["levels"][L]
        nxF, nyF = wl["levels"][Lmax]
        rx = (nxF - 1) // (nxL - 1)
        rt = wl["steps"][Lmax] // wl["steps"][L]
        vr = vref.reshape(wl["steps"][Lmax], nyF, nxF)[rt - 1::rt, :, ::rx].reshape(-1)
        w = weights(L)
        res = {"level": L}
        for name, single in (("mc", True), ("mlmc", False)):
            if single:
                N = [max(2, 16 ** L)]
            else:
                N = [max(2, 16 ** L // 16 ** l) for l in range(L + 1)]
            errs, works = [], []
            for r in range(a.repeats):
                v, wk = estimate(L, N, 1000 + 37 * r, single)
                errs.append(float(w @ (v - vr) ** 2))
                works.append(wk)
            res[name] = {"N": N, "rmse": float(np.sqrt(np.mean(errs))), "work_s": float(np.mean(works))}
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
