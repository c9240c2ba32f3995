"""Copy kernel of known size, used to calibrate the HBM byte counters.

Runs `iters` device-to-device copies of an `mib` MiB float64 buffer on
cuda:0 and prints the expected bytes per copy and the achieved bandwidth.
Profiling it with the FETCH_SIZE / WRITE_SIZE counters gives the counter
reading of a launch that moves exactly `mib` MiB each way.

    python -m paper_1911_06066_amd.copycal --mib 1024 --iters 5
"""

import argparse
import json
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=5)
    a = ap.parse_args()
    import torch
    n = a.mib * 1024 * 1024 // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.iters):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.iters
    print(json.dumps({"bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
                      "copy_GBps_read_plus_write": 2 * n * 8 / dt / 1e9}))


if __name__ == "__main__":
    main()
