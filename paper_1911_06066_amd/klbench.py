"""KL synthesis throughput: sigma[s, e] = sigma_f0 exp(sum_k modes[e, k] xi[s, k]).

Times the library's KL kernel (float64 MFMA, or split-f16 MFMA for the mixed
precision) on a workload level, with inputs resident on the device, and prints
one JSON line: effective GB/s (sigma written + modes and xi read once) and
TFLOP/s (2 E S M flops of the contraction).

    python -m paper_1911_06066_amd.klbench --workload slab3d --level 0 --samples 256
"""

import argparse
import json
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="slab3d")
    ap.add_argument("--level", type=int, default=0)
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--precision", default=None)
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import stinputs
    from paper_1911_06066_amd import Context, klmodes

    wl = stinputs.workload(a.workload)
    prec = a.precision or wl["precision"]
    dev = torch.device("cuda:0")
    modes = torch.from_numpy(klmodes.workload_modes(wl)[a.level]).to(dev)
    M = wl["n_modes"]
    xi = torch.from_numpy(stinputs.xi(wl["name"], a.level, a.samples, M)).to(dev)
    with Context(wl, precision=prec) as ctx:
        run(ctx, a, modes, xi, M, prec)


def run(ctx, a, modes, xi, M, prec):
    import torch
    E = modes.shape[0]
    out = torch.empty((a.samples, E), dtype=torch.float64, device=modes.device)
    ctx.kl_synthesize(a.level, modes, xi, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = 0.0
    for _ in range(a.iters):
        ctx.kl_synthesize(a.level, modes, xi, out=out)
        ms += ctx.timings()["kl_ms"]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / a.iters
    kernel_s = ms / a.iters * 1e-3
    bytes_ = 8.0 * (a.samples * E + E * M + a.samples * M)
    flops = 2.0 * a.samples * E * M
    print(json.dumps({"workload": a.workload, "level": a.level, "precision": prec, "E": E, "M": M,
                      "S": a.samples, "kernel_ms": kernel_s * 1e3, "wall_ms": wall * 1e3,
                      "GBps": bytes_ / kernel_s / 1e9, "TFLOPs": flops / kernel_s / 1e12}), flush=True)


if __name__ == "__main__":
    main()
