"""Build libafps.so (HIP for gfx950) in-tree.

Every source under csrc/ is compiled by hipcc in parallel into _build/, then
linked into paper_2208_08795_amd/libafps.so.  kernels.hip is compiled once per
wave count.  Flags: -O3, no floating-point contraction (the distance must be
((dx*dx + dy*dy) + dz*dz) with separate roundings), no packed fp32 ops.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libafps.so")
ARCH = os.environ.get("AFPS_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _units():
    units = [("kernels.hip", "kernels_w%d.o" % w, ["-DAFPS_WAVES=%d" % w]) for w in (1, 2, 4, 8, 16)]
    units += [("kernels_npdu.hip", "kernels_npdu.o", []), ("kernels_pool.hip", "kernels_pool.o", []),
              ("fps_grid.hip", "fps_grid.o", []), ("check.hip", "check.o", []),
              ("binning.hip", "binning.o", []),
              ("group.hip", "group.o", []),
              ("planner.cpp", "planner.o", []),
              ("afps_api.cpp", "afps_api.o", ["-x", "hip"])]
    return units


def _compile(unit):
    src, obj, extra = unit
    out = os.path.join(BUILD, obj)
    cmd = ["hipcc", "--offload-arch=" + ARCH, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return out


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, _units()))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else None))
