"""Sampling quality as coverage radius (evaluation only, not on the sampling path).

The paper judges a sampler by downstream task accuracy with a pre-trained
PointNet++ (Sec. IV), which needs datasets and weights that are not available
here.  Coverage radius is a task-free stand-in: the largest distance from any
point of the cloud to its nearest sample,

    r = max_j min_t || P_j - P_{idx_t} ||_2 ,

over all points and all samples (not per sector), evaluated in fp64 on the
fp32 coordinates.  Plain FPS is the greedy 2-approximation of the minimum
coverage radius (k-center), so r(method) / r(FPS) measures what a heuristic
gives up.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def coverage_radius(points, indices) -> float:
    p = np.asarray(points, dtype=np.float64)
    idx = np.asarray(indices, dtype=np.int64)
    if idx.size == 0:
        raise ValueError("empty sample set")
    tree = cKDTree(p[np.unique(idx)])
    dist, _ = tree.query(p, k=1)
    return float(dist.max())
