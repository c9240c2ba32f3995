"""Host-side checks of the C interface that need no GPU.

The library loads and exports every symbol include/stmlmc.h declares, the
ctypes layouts match the header, and invalid problems are rejected before any
device work.
"""

import ctypes
import os
import re

import pytest

import stinputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stmlmc.h")


def _lib():
    from paper_1911_06066_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libstmlmc.so not built")
    return L, L.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    names = _declared_functions()
    assert set(names) == set(L.SIGNATURES), names
    for n in names:
        assert hasattr(lib, n), n


def _c_layout(struct, fields):
    """sizeof and offsetof of a header struct, printed by a C program built with gcc."""
    import shutil
    import subprocess
    import tempfile
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "stmlmc.h"', "int main(void) {",
             '  printf("%%zu\\n", sizeof(%s));' % struct]
    for f in fields:
        lines.append('  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f))
    lines.append("  return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        open(src, "w").write("\n".join(lines))
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("cname,pyname", [("stm_problem", "StmProblem"), ("stm_solve_stats", "StmSolveStats"),
                                          ("stm_mlmc_result", "StmMlmcResult"), ("stm_level", "StmLevel"),
                                          ("stm_timings", "StmTimings")])
def test_struct_layouts_match_header(cname, pyname):
    L, _ = _lib()
    cls = getattr(L, pyname)
    fields = [f[0] for f in cls._fields_]
    got = _c_layout(cname, fields)
    assert got[0] == ctypes.sizeof(cls)
    for f, off in zip(fields, got[1:]):
        assert getattr(cls, f).offset == off, f


@pytest.mark.parametrize("field,value", [
    ("dim", 4), ("n_levels", 0), ("n_modes", 0), ("precision", 7), ("gmres_restart", 31),
    ("block_threads", 100), ("fiber_law", 9), ("theta", 0.3), ("theta", 1.5),
    ("field_kind", 2), ("tau_relative", 3), ("ic_kind", 5), ("qoi", 2), ("ic_radius", -1.0),
])
def test_invalid_problem_rejected_before_device_work(field, value):
    L, lib = _lib()
    from paper_1911_06066_amd import problem_from_workload
    p = problem_from_workload(stinputs.workload("small_mc_2d"))
    setattr(p, field, value)
    h = ctypes.c_void_p()
    st = lib.stm_create(ctypes.byref(p), None, ctypes.byref(h))
    assert st == -1 and not h.value


def test_gaussian_initial_state_needs_a_radius():
    L, lib = _lib()
    from paper_1911_06066_amd import problem_from_workload
    p = problem_from_workload(stinputs.workload("cube4_3d", ic_radius=0.0))
    h = ctypes.c_void_p()
    assert lib.stm_create(ctypes.byref(p), None, ctypes.byref(h)) == -1 and not h.value


@pytest.mark.parametrize("mg_levels", [-2, 9])
def test_multigrid_depth_out_of_range_rejected(mg_levels):
    """V-cycle depths outside -1 (deepest) .. 8 grids are invalid arguments."""
    L, lib = _lib()
    from paper_1911_06066_amd import problem_from_workload
    p = problem_from_workload(stinputs.workload("small_mc_2d"), mg_levels=mg_levels)
    h = ctypes.c_void_p()
    assert lib.stm_create(ctypes.byref(p), None, ctypes.byref(h)) == -1 and not h.value


@pytest.mark.parametrize("over", [dict(st_mode=2), dict(st_mode=-1), dict(st_mode=1, block_threads=1024)])
def test_space_time_mode_out_of_range_rejected(over):
    """st_mode is 0 (slab by slab) or 1 (global space-time GMRES, 256 or 512
    threads per workgroup)."""
    L, lib = _lib()
    from paper_1911_06066_amd import problem_from_workload
    p = problem_from_workload(stinputs.workload("small_mc_2d"), **over)
    h = ctypes.c_void_p()
    assert lib.stm_create(ctypes.byref(p), None, ctypes.byref(h)) == -1 and not h.value


def test_non_nested_levels_rejected():
    L, lib = _lib()
    from paper_1911_06066_amd import problem_from_workload
    p = problem_from_workload(stinputs.workload("mlmc3_2d", levels=[(33, 33), (64, 64), (129, 129)]))
    h = ctypes.c_void_p()
    assert lib.stm_create(ctypes.byref(p), None, ctypes.byref(h)) == -1
