"""Build the HIP library libstmlmc.so for gfx950 in-tree with hipcc."""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstmlmc.so")
CAL_LIB = os.path.join(HERE, "libstmcal.so")  # copy kernels for counter calibration (not the solver interface)
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["st_solver.hip", "kl_gemm.hip", "qoi_mlmc.hip", "stm_api.hip"]

# Packed-fp32 instructions stay off: the compiler otherwise forms them from
# plain float code.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return path


def _compile(src, extra=(), build_dir=BUILD_DIR):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + FLAGS + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(verbose=False, lib=LIB, defines=(), build_dir=BUILD_DIR):
    """Compile every source and link the library (always rebuilds).

    defines: extra -D flags, e.g. ("STM_PHASE_TIMERS",) for a phase-timed
    development build written to another path.
    """
    os.makedirs(build_dir, exist_ok=True)
    extra = ["-D" + d for d in defines]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, extra, build_dir), SOURCES))
    tmp = lib + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    if lib != LIB:
        return lib
    cal_obj = _compile("copycal.hip", extra, build_dir)
    tmp = CAL_LIB + ".tmp"
    r = subprocess.run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, cal_obj],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, CAL_LIB)
    if verbose:
        print("built", CAL_LIB)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
