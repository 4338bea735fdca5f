"""CPU oracle for FPS / AFPS / NPDU-AFPS (Li et al., arXiv 2208.08795) and the
grouping around the samples (ball query).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports this
package, and this package imports nothing from the GPU library.

The arithmetic lives in ``afps_oracle.c`` (plain C, fp32, contraction off); this
module only compiles it (gcc) when the shared library is missing and marshals
NumPy arrays through ctypes.  Parity status of each function is recorded in
the C file's header and the design notes: every function here is pinned by the
tests under ``tests/`` (hand examples, brute force, closed forms, invariants).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "afps_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# x86-64 SSE fp32: every operation is one IEEE rounding; no contraction.
GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]

_lock = threading.Lock()
_lib = None


def build(path: str = _LIB_PATH, src: str = _SRC) -> str:
    """Compile the oracle into a shared library (gcc)."""
    tmp = path + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *GCC_FLAGS, src, "-o", tmp], check=True)
    os.replace(tmp, path)
    return path


def load(path: str | None = None):
    """Load the oracle library, compiling it first if it is not there."""
    global _lib
    with _lock:
        if path is None and _lib is not None:
            return _lib
        p = path or _LIB_PATH
        if not os.path.exists(p):
            build(p)
        lib = ctypes.CDLL(p)
        i32, i64p = ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
        fptr, iptr = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32)
        lib.oracle_afps.argtypes = [fptr, i32, i32, i32, i32, i32, iptr, fptr, i64p]
        lib.oracle_afps.restype = ctypes.c_int
        lib.oracle_afps_ex.argtypes = [fptr, i32, i32, i32, i32, i32, i32, iptr, fptr, i64p]
        lib.oracle_afps_ex.restype = ctypes.c_int
        lib.oracle_fps.argtypes = [fptr, i32, i32, i32, iptr, fptr, i64p]
        lib.oracle_fps.restype = ctypes.c_int
        lib.oracle_sector.argtypes = [i32, i32, i32, i32, iptr, iptr, iptr, iptr]
        lib.oracle_sector.restype = None
        lib.oracle_ball_query.argtypes = [fptr, i32, iptr, i32, ctypes.c_float, i32, i32, iptr, iptr]
        lib.oracle_ball_query.restype = ctypes.c_int
        if path is None:
            _lib = lib
        return lib


class OracleError(RuntimeError):
    pass


def _points(points) -> np.ndarray:
    p = np.ascontiguousarray(points, dtype=np.float32)
    if p.ndim != 2 or p.shape[1] != 3:
        raise ValueError("points must be (N, 3)")
    return p


# NPDU readings other than the default (bit flags; see afps_oracle.c).
NPDU_FIRST_FULL, NPDU_SHIFT_EDGES, NPDU_K_WITH_SELF = 1, 2, 4


def afps(points, c: int, m: int = 1, k: int | None = None, start: int = 0,
         with_state: bool = False, lib=None, flags: int = 0):
    """AFPS (Sec. III-B) with M sectors, NPDU window k (Sec. III-C) or None.

    Returns int32 global indices (sector-major, pick order inside a sector).
    With ``with_state`` also returns the final Distance array and the number of
    distance evaluations.  ``flags`` selects NPDU readings (NPDU_*).
    """
    lib = lib or load()
    p = _points(points)
    n = p.shape[0]
    out = np.empty(max(c, 0), dtype=np.int32)
    dist = np.empty(max(n, 0), dtype=np.float32)
    evals = ctypes.c_int64(0)
    rc = lib.oracle_afps_ex(
        p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, c, m,
        -1 if k is None else int(k), int(flags), start,
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        dist.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(evals))
    if rc != 0:
        raise OracleError("oracle_afps returned %d" % rc)
    if with_state:
        return out, dist, int(evals.value)
    return out


def fps(points, c: int, start: int = 0, with_state: bool = False, lib=None):
    """Plain FPS (Algorithm 1)."""
    return afps(points, c, 1, None, start, with_state, lib)


def sector(n: int, c: int, m: int, s: int, lib=None):
    """(first_point, num_points, first_sample, num_samples) of sector s."""
    lib = lib or load()
    vals = [ctypes.c_int32() for _ in range(4)]
    lib.oracle_sector(n, c, m, s, *[ctypes.byref(v) for v in vals])
    return tuple(v.value for v in vals)


def ball_query(points, centers, radius: float, k: int, window: int | None = None, lib=None):
    """Grouping around the samples (the consumer the paper names, Sec. I and
    II-A): up to ``k`` neighbours per centre with squared fp32 distance below
    fp32(radius * radius), in increasing index order, padded with the first
    found (the centre itself when none is); ``window`` bounds the candidates
    to storage positions within ``window`` of the centre (None: all points).

    Returns (idx int32 (C, k), count int32 (C,))."""
    lib = lib or load()
    p = _points(points)
    ctr = np.ascontiguousarray(centers, dtype=np.int32)
    c = ctr.shape[0]
    idx = np.empty((c, k), dtype=np.int32)
    cnt = np.empty(c, dtype=np.int32)
    iptr = ctypes.POINTER(ctypes.c_int32)
    rc = lib.oracle_ball_query(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.shape[0],
                               ctr.ctypes.data_as(iptr), c, float(radius), int(k),
                               -1 if window is None else int(window), idx.ctypes.data_as(iptr),
                               cnt.ctypes.data_as(iptr))
    if rc != 0:
        raise OracleError("oracle_ball_query returned %d" % rc)
    return idx, cnt
