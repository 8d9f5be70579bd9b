"""Builds libmlb.so (the gfx950 HIP library behind include/mlb.h) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmlb.so")
SOURCES = ["mlb_kernels.hip", "mlb_kernels2.hip", "mlb_persist.hip", "mlb_noalloc.hip", "mlb_api.hip", "nn_kernels.hip", "nn_api.hip", "elab_kernels.hip", "elab_api.hip"]
ARCH = os.environ.get("MLB_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # one rounding per written operation: fused multiply-adds only where the
    # source asks for them, so every kernel variant rounds identically
    "-ffp-contract=off",
    # no packed FP32 (v_pk_*_f32) code generation
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source into libmlb.so (always recompiles): one hipcc per
    translation unit in parallel, then one link."""
    from concurrent.futures import ThreadPoolExecutor
    tag = "%d" % os.getpid()
    objs = [out + ".%s.%s.o" % (os.path.splitext(s)[0], tag) for s in SOURCES]
    base = [f for f in FLAGS if f != "-shared"] + ["-D" + d for d in defines]

    def cc(i):
        cmd = ["hipcc", "-c"] + base + [os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 1))
    try:
        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(cc, range(len(SOURCES))))
        for r in results:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError("hipcc failed building libmlb.so")
        tmp = out + ".tmp" + tag
        cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libmlb.so")
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


def asm(out_dir: str) -> None:
    """Write the gfx950 assembly of the kernels (for inspection)."""
    os.makedirs(out_dir, exist_ok=True)
    cmd = ["hipcc"] + [f for f in FLAGS if f not in ("-shared", "-fPIC")] + [
        "--cuda-device-only", "-S", os.path.join(CSRC, "mlb_kernels.hip"),
        "-o", os.path.join(out_dir, "mlb_kernels.s")]
    subprocess.check_call(cmd)


if __name__ == "__main__":
    print(build(verbose=True))
