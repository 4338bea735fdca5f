"""Pins of the grouping oracle (the ball query around the samples that the
paper names as their consumer, Sec. I and II-A, with the readings in the
oracle's header): hand-derived cases, scipy's k-d tree as an independent
neighbour search, and planted mistakes that must fail the pins."""
import os
import shutil

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "afps_oracle.c")
LINE = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0], [10, 0, 0], [10, 0, 0]], np.float32)


def _hand_cases_pass(lib) -> bool:
    """Collinear integer points: every squared distance is exact in fp32."""
    cases = [
        # radius 1.5 (r2 = 2.25): from 0, points 0 and 1; from 2, points 1, 2, 3; point 4 has a
        # duplicate (5) at distance 0.  K = 4: padding repeats the first found.
        (dict(centers=[0, 2, 4], radius=1.5, k=4), [[0, 1, 0, 0], [1, 2, 3, 1], [4, 5, 4, 4]], [2, 3, 2]),
        # radius 1 (r2 = 1): a neighbour at squared distance exactly 1 is outside (strict <).
        (dict(centers=[1], radius=1.0, k=3), [[1, 1, 1]], [1]),
        # K = 1: the lowest index within the ball, not the centre.
        (dict(centers=[2], radius=2.5, k=1), [[0]], [1]),
        # window 1 around centre 2: only 1, 2, 3 are candidates.
        (dict(centers=[2], radius=2.5, k=5, window=1), [[1, 2, 3, 1, 1]], [3]),
        # window 0: the centre alone.
        (dict(centers=[3], radius=9.0, k=2, window=0), [[3, 3]], [1]),
        # radius 0: nothing found, every slot holds the centre.
        (dict(centers=[3], radius=0.0, k=2), [[3, 3]], [0]),
        # window past both ends is the whole cloud.
        (dict(centers=[0], radius=100.0, k=6, window=1 << 30), [[0, 1, 2, 3, 4, 5]], [6]),
    ]
    for kw, want_idx, want_cnt in cases:
        try:
            idx, cnt = oracle.ball_query(LINE, lib=lib, **kw)
        except oracle.OracleError:
            return False
        if idx.tolist() != want_idx or cnt.tolist() != want_cnt:
            return False
    return True


def _kdtree_cases_pass(lib) -> bool:
    """scipy's k-d tree (fp64, independent code) gives the neighbour sets;
    centres with a point within rounding reach of the ball's surface are
    left out, where fp32 and fp64 may disagree."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(31)
    for trial in range(6):
        n = int(rng.integers(50, 400))
        pts = rng.random((n, 3), dtype=np.float32)
        pts[rng.integers(0, n, 5)] = pts[rng.integers(0, n, 5)]     # a few duplicates
        radius = float(rng.uniform(0.1, 0.4))
        k = int(rng.integers(1, 40))
        window = [None, 7, 40][trial % 3]
        centers = rng.integers(0, n, 30).astype(np.int32)
        try:
            idx, cnt = oracle.ball_query(pts, centers, radius, k, window, lib=lib)
        except oracle.OracleError:
            return False
        r2 = float(np.float32(radius) * np.float32(radius))
        p64 = pts.astype(np.float64)
        tree = cKDTree(p64)
        for q, ci in enumerate(centers):
            d2 = ((p64 - p64[ci]) ** 2).sum(axis=1)
            if np.any(np.abs(d2 - r2) < 1e-5 * r2):
                continue
            ball = sorted(tree.query_ball_point(p64[ci], np.sqrt(r2)))
            if window is not None:
                ball = [j for j in ball if abs(j - int(ci)) <= window]
            want = ball[:k]
            if cnt[q] != len(want) or idx[q, :len(want)].tolist() != want:
                return False
            if want and np.any(idx[q, len(want):] != want[0]):
                return False
    return True


def pins_pass(lib) -> bool:
    return _hand_cases_pass(lib) and _kdtree_cases_pass(lib)


def test_grouping_pins():
    assert pins_pass(oracle.load())


def test_exact_is_the_widest_window():
    rng = np.random.default_rng(5)
    pts = rng.random((300, 3), dtype=np.float32)
    centers = rng.integers(0, 300, 50)
    a = oracle.ball_query(pts, centers, 0.3, 16)
    b = oracle.ball_query(pts, centers, 0.3, 16, window=299)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_argument_errors():
    with pytest.raises(oracle.OracleError):
        oracle.ball_query(LINE, [6], 1.0, 2)          # centre out of range
    with pytest.raises(oracle.OracleError):
        oracle.ball_query(LINE, [0], 1.0, 0)          # K < 1
    with pytest.raises(oracle.OracleError):
        oracle.ball_query(LINE, [0], -1.0, 2)         # negative radius


MUTANTS = {
    "ball_includes_surface": ("< r2) row[found++] = j;", "<= r2) row[found++] = j;"),
    "radius_not_squared": ("const float r2 = radius * radius;", "const float r2 = radius;"),
    "window_low_edge_off": ("lo = ci - window < 0 ? 0 : ci - window;",
                            "lo = ci - window < 0 ? 0 : ci - window + 1;"),
    "pad_with_centre": ("const int32_t fill = found > 0 ? row[0] : ci;", "const int32_t fill = ci;"),
    "stops_one_short": ("j <= hi && found < K;", "j <= hi && found < K - 1;"),
    "distance_to_point_0": ("squared_distance(P + 3 * (int64_t)j, P + 3 * (int64_t)ci) < r2",
                            "squared_distance(P + 3 * (int64_t)j, P) < r2"),
}


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return tmp_path_factory.mktemp("grouping_mutants")


def test_unmutated_copy_passes(workdir):
    path = str(workdir / "liboracle_copy.so")
    shutil.copy(SRC, str(workdir / "copy.c"))
    oracle.build(path, str(workdir / "copy.c"))
    assert pins_pass(oracle.load(path))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, workdir):
    old, new = MUTANTS[name]
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, "mutation anchor not found: " + name
    src = workdir / (name + ".c")
    src.write_text(text.replace(old, new))
    path = str(workdir / ("lib" + name + ".so"))
    oracle.build(path, str(src))
    assert not pins_pass(oracle.load(path)), "pins did not catch mutant " + name
