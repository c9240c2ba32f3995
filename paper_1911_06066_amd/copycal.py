"""Copy kernel of known size, used to calibrate the HBM byte counters.

Runs `iters` device-to-device copies of an `mib` MiB buffer on cuda:0 with
the library's own copy kernel (libstmcal.so), reading and writing `width`-byte
elements (8: float64, as the solver's float64 fields and conductivities; 4:
float32, as its mixed-precision Krylov vectors), and prints the bytes per copy
and the achieved bandwidth.  Profiling it with the FETCH_SIZE / WRITE_SIZE
counters gives the counter reading of a launch that moves exactly `mib` MiB
each way with that access width.

    python -m paper_1911_06066_amd.copycal --mib 1024 --iters 3 --width 8
"""

import argparse
import ctypes
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=3)
    ap.add_argument("--width", type=int, default=8, choices=[4, 8])
    a = ap.parse_args()
    import torch
    path = os.path.join(HERE, "libstmcal.so")
    if not os.path.exists(path):
        raise RuntimeError("libstmcal.so not built (python -m paper_1911_06066_amd.build)")
    lib = ctypes.CDLL(path)
    lib.stmcal_copy.restype = ctypes.c_int
    lib.stmcal_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    nbytes = a.mib * 1024 * 1024
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def copy():
        e = lib.stmcal_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes, a.width, stream)
        if e != 0:
            raise RuntimeError("copy kernel launch failed: %d" % e)

    copy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.iters):
        copy()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.iters
    assert bool((dst == src).all())
    print(json.dumps({"width": a.width, "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "copy_GBps_read_plus_write": 2 * nbytes / dt / 1e9}))


if __name__ == "__main__":
    main()
