"""Independent brute-force sampler used to pin the oracle (tests only).

It shares nothing with ``oracle/``: sectors come from ``numpy.array_split``,
and instead of carrying a running Distance array it recomputes, before every
pick, each point's distance from scratch as the minimum over all earlier
samples (for NPDU: over the earlier samples whose window covered the point),
with the paper's initial 1e10 where no sample covered it.  The pick is
``numpy.argmax`` (first maximum = lowest index).

Distances are fp32 in the operation order ((dx*dx + dy*dy) + dz*dz); NumPy
evaluates each float32 operation with one rounding and never fuses, so the
result is bit-identical to any implementation using that order.
"""
from __future__ import annotations

import numpy as np

INIT = np.float32(1e10)
FIRST_FULL, SHIFT_EDGES, K_WITH_SELF = 1, 2, 4   # NPDU readings (bit flags)


def _sq(block: np.ndarray, p: np.ndarray) -> np.ndarray:
    dx = block[:, 0] - p[0]
    dy = block[:, 1] - p[1]
    dz = block[:, 2] - p[2]
    return (dx * dx + dy * dy) + dz * dz


def _window(t: int, n: int, k, flags: int = 0, first: bool = False):
    """Inclusive range of points whose distance sample t updates."""
    if k is None or (first and flags & FIRST_FULL):
        return 0, n - 1
    # points below and above the sample
    below, above = ((k - 1) // 2, k - 1 - (k - 1) // 2) if flags & K_WITH_SELF else (k // 2, (k + 1) // 2)
    if flags & SHIFT_EDGES:
        width = below + above + 1                      # kept whole where the sector allows
        if width >= n:
            return 0, n - 1
        lo = int(np.clip(t - below, 0, n - width))
        return lo, lo + width - 1
    return max(0, t - below), min(n - 1, t + above)


def sector_sample(points: np.ndarray, c: int, k, start: int, flags: int = 0) -> list[int]:
    """Local indices picked in one sector by recomputation from scratch."""
    n = points.shape[0]
    picks = [start % n]
    while len(picks) < c:
        dist = np.full(n, INIT, dtype=np.float32)
        for i, t in enumerate(picks):
            lo, hi = _window(t, n, k, flags, first=(i == 0))
            dist[lo:hi + 1] = np.minimum(dist[lo:hi + 1], _sq(points[lo:hi + 1], points[t]))
        picks.append(int(np.argmax(dist)))
    return picks


def afps(points, c: int, m: int = 1, k=None, start: int = 0, flags: int = 0) -> np.ndarray:
    p = np.asarray(points, dtype=np.float32)
    n = p.shape[0]
    assert 1 <= m <= c <= n and 0 <= start < n
    point_parts = np.array_split(np.arange(n), m)
    sample_parts = np.array_split(np.arange(c), m)
    out = np.empty(c, dtype=np.int32)
    for pts, smp in zip(point_parts, sample_parts):
        local = sector_sample(p[pts], len(smp), k, start, flags)
        out[smp] = pts[np.asarray(local)]
    return out
