"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol declared in include/mlb.h, the ctypes layouts match the C
structs, and parameter validation rejects bad input."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1902_02999_amd import mlb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlb.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mlb_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = mlb.lib()
    names = declared_symbols()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    # and the binding covers exactly the declared API
    assert set(mlb.SIGNATURES) == set(names)


def test_struct_layouts_match_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "mlb.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(mlb_params), offsetof(mlb_params, edge),
         offsetof(mlb_params, extrap_order), sizeof(mlb_diag_t), offsetof(mlb_diag_t, rle),
         sizeof(mlb_exec_opts));
  return 0;
}""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = list(map(int, subprocess.check_output([str(exe)]).split()))
    want = [C.sizeof(mlb.Params), mlb.Params.edge.offset, mlb.Params.extrap_order.offset,
            C.sizeof(mlb.Diag), mlb.Diag.rle.offset, C.sizeof(mlb.ExecOpts)]
    assert got == want


def ws_bytes(**kw):
    p = mlb.make_params(**kw)
    n = C.c_size_t()
    rc = mlb.lib().mlb_grid_workspace_bytes(C.byref(p), C.byref(n))
    return rc, n.value


def test_workspace_size_and_validation():
    rc, n = ws_bytes(nx=100, ny=50, dx=1.0, nu=1.0)
    assert rc == 0
    ld = 128
    assert n == 256 + 7 * ((ld * 50 * 4 + 255) // 256 * 256)
    # periodic edges must come in pairs
    rc, _ = ws_bytes(nx=10, ny=10, dx=1.0, nu=1.0, edges=(mlb.PERIODIC, mlb.WALL, mlb.WALL, mlb.WALL))
    assert rc == -1
    # adjacent open edges are rejected
    rc, _ = ws_bytes(nx=10, ny=10, dx=1.0, nu=1.0, edges=(mlb.DEPTH, mlb.WALL, mlb.DISCHARGE, mlb.WALL))
    assert rc == -1
    # too small for open edges
    rc, _ = ws_bytes(nx=4, ny=10, dx=1.0, nu=1.0, edges=(mlb.DEPTH, mlb.WALL, mlb.WALL, mlb.WALL))
    assert rc == -1
    # non-positive viscosity
    rc, _ = ws_bytes(nx=10, ny=10, dx=1.0, nu=0.0)
    assert rc == -1
    assert mlb.lib().mlb_last_error() == b"dx, nu, g and rho_w must be positive"
    rc, _ = ws_bytes(nx=10, ny=10, dx=1.0, nu=1.0, edges=(mlb.PERIODIC, mlb.WALL, mlb.WALL, mlb.WALL))
    assert rc == -1
    assert b"periodic" in mlb.lib().mlb_last_error()
    rc, _ = ws_bytes(nx=10, ny=10, dx=1.0, nu=1.0, extrap_order=3)
    assert rc == -1
    assert mlb.lib().mlb_status_str(-4) == b"unstable parameters (g H > e^2)"


def test_no_gpu_reports_an_error_not_a_crash():
    try:
        import torch
        if torch.cuda.device_count() > 0:
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = C.c_void_p()
    rc = mlb.lib().mlb_ctx_create(0, None, C.byref(h))
    assert rc in (-1, -3) and not h.value
