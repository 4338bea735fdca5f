"""Binning of a cloud along one axis -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU baseline leg of the benchmark
may import this module; the GPU library never uses it and shares no code with
it.

Sec. III-A notes that a cloud without dimensional locality can be binned
instead of sorted: AFPS (Sec. III-B) and NPDU (Sec. III-C) need only the
approximate order of the paper's footnote to Table II, where every point of a
later bin has a larger coordinate than every point of an earlier bin and
points inside a bin are in no particular order.

bin_points(points, axis, bins) computes, in fp32 (the paper fixes no
precision; the coordinates are fp32, and a float that decides an integer bin
must be taken in one stated arithmetic, so this reading of Sec. III-A fixes
fp32 with one correctly rounded division and no fused multiply-add):
    lo, hi = smallest and largest coordinate along `axis`
    scale  = bins / (hi - lo)                    (one correctly rounded division;
                                                  0 when hi == lo)
    t_j    = (x_j - lo) * scale                  (two fp32 operations)
    bin_j  = min(bins - 1, floor(t_j))
and returns the stable order of the points by bin (the points of a bin keep
their storage order), with every point's bin.
"""
from __future__ import annotations

import numpy as np


def bins_of(points, axis: int, bins: int) -> np.ndarray:
    """Bin of every point (int64)."""
    p = np.ascontiguousarray(points, dtype=np.float32)
    if p.ndim != 2 or p.shape[1] != 3 or p.shape[0] < 1:
        raise ValueError("points must be (N, 3) with N >= 1")
    if axis not in (0, 1, 2) or bins < 1:
        raise ValueError("axis in {0, 1, 2} and bins >= 1")
    x = p[:, axis]
    lo, hi = np.float32(x.min()), np.float32(x.max())
    scale = np.float32(bins) / np.float32(hi - lo) if hi > lo else np.float32(0)
    t = (x - lo) * scale
    return np.minimum(t.astype(np.int64), bins - 1)


def bin_points(points, axis: int, bins: int):
    """(perm, bin): perm[i] is the storage index of the i-th point in binned
    order (int32), bin[j] the bin of point j."""
    b = bins_of(points, axis, bins)
    perm = np.argsort(b, kind="stable").astype(np.int32)
    return perm, b
