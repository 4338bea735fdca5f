"""Pins of the CPU oracle against things other than itself.

* hand-derived worked examples (tests/golden/hand_examples.json);
* an independent brute force that recomputes every distance from scratch;
* closed forms the paper fixes: M = 1 is FPS, M = C takes one sample per
  sector, an NPDU window spanning the sector is plain local FPS, k = 0 and the
  start-0 NPDU sweep have explicit answers;
* invariants: sector confinement, unique picks on distinct points, FPS
  non-increasing pick distances, the Gonzalez 2-approximation, NPDU distances
  never below the true nearest-sample distance, exact update counts.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from tests import bruteforce

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_hand_examples(case):
    pts = np.array(case["points"], dtype=np.float32)
    flags = case.get("flags", 0)
    got = oracle.afps(pts, case["c"], case["m"], case["k"], case["start"], flags=flags)
    assert got.tolist() == case["expected"]
    # the brute force agrees with the hand derivation as well
    bf = bruteforce.afps(pts, case["c"], case["m"], case["k"], case["start"], flags)
    assert bf.tolist() == case["expected"]


def _random_cloud(rng, n, kind):
    if kind == "uniform":
        return rng.random((n, 3), dtype=np.float32)
    if kind == "grid":      # many exact distance ties
        return rng.integers(0, 3, (n, 3)).astype(np.float32)
    if kind == "sorted":
        p = rng.standard_normal((n, 3)).astype(np.float32)
        return p[np.argsort(p[:, 0], kind="stable")]
    if kind == "dups":      # duplicated points: zero distances, repeated picks
        base = rng.random((max(1, n // 3), 3), dtype=np.float32)
        return base[rng.integers(0, base.shape[0], n)]
    raise ValueError(kind)


def _random_params(rng, n):
    c = int(rng.integers(1, n + 1))
    m = int(rng.integers(1, c + 1))
    k = [None, 0, 1, 2, 3, 4, 5, 8, 13, 2 * n][int(rng.integers(0, 10))]
    start = int(rng.integers(0, n))
    return c, m, k, start


@pytest.mark.parametrize("kind", ["uniform", "grid", "sorted", "dups"])
def test_bruteforce_agreement(kind):
    rng = np.random.default_rng(1234 + hash(kind) % 1000)
    for _ in range(60):
        n = int(rng.integers(1, 48))
        pts = _random_cloud(rng, n, kind)
        c, m, k, start = _random_params(rng, n)
        want = bruteforce.afps(pts, c, m, k, start)
        got = oracle.afps(pts, c, m, k, start)
        assert got.tolist() == want.tolist(), (n, c, m, k, start)


def test_bruteforce_agreement_larger():
    rng = np.random.default_rng(77)
    for n, c, m, k in [(256, 64, 1, None), (256, 64, 4, None), (200, 50, 3, 8),
                       (256, 64, 8, 32), (241, 37, 5, 7), (256, 32, 32, None)]:
        pts = _random_cloud(rng, n, "sorted")
        start = int(rng.integers(0, n))
        assert oracle.afps(pts, c, m, k, start).tolist() == \
            bruteforce.afps(pts, c, m, k, start).tolist()


def test_sector_plan_matches_array_split():
    for n in range(1, 40):
        for c in range(1, n + 1):
            for m in range(1, c + 1):
                pp = np.array_split(np.arange(n), m)
                ss = np.array_split(np.arange(c), m)
                for s in range(m):
                    b, ns, o, cs = oracle.sector(n, c, m, s)
                    assert (b, ns, o, cs) == (pp[s][0], len(pp[s]), ss[s][0], len(ss[s]))
                    assert 1 <= cs <= ns  # c_s <= n_s whenever c <= n


def test_m_equals_c_one_pick_per_sector():
    rng = np.random.default_rng(5)
    for n, c, start in [(100, 10, 0), (97, 13, 50), (64, 64, 63), (33, 7, 32)]:
        pts = rng.random((n, 3), dtype=np.float32)
        got = oracle.afps(pts, c, c, None, start)
        want = [int(part[start % len(part)]) for part in np.array_split(np.arange(n), c)]
        assert got.tolist() == want


def test_m1_is_greedy_fps_definition():
    """M = 1 without NPDU: each pick maximises the min distance to earlier picks."""
    rng = np.random.default_rng(11)
    pts = rng.random((300, 3), dtype=np.float32)
    got = oracle.afps(pts, 40, 1, None, 17)
    assert got.tolist() == oracle.fps(pts, 40, 17).tolist()
    for i in range(1, len(got)):
        d = np.full(len(pts), np.float32(1e10))
        for t in got[:i]:
            dx, dy, dz = (pts[:, a] - pts[t, a] for a in range(3))
            d = np.minimum(d, (dx * dx + dy * dy) + dz * dz)
        assert got[i] == int(np.flatnonzero(d == d.max())[0])


def test_npdu_window_spanning_sector_is_local_fps():
    rng = np.random.default_rng(3)
    for n, c, m in [(128, 32, 1), (130, 24, 4), (99, 20, 7)]:
        pts = rng.random((n, 3), dtype=np.float32)
        big = 2 * (n // m + 1)          # floor(k/2) >= n_s - 1 for every sector
        assert oracle.afps(pts, c, m, big, 5).tolist() == oracle.afps(pts, c, m, None, 5).tolist()


def test_npdu_k0_sweeps_in_storage_order():
    rng = np.random.default_rng(4)
    pts = rng.random((50, 3), dtype=np.float32)
    got = oracle.afps(pts, 20, 1, 0, 7)
    assert got.tolist() == [7] + [j for j in range(50) if j != 7][:19]


@pytest.mark.parametrize("k", [0, 1, 8, 32, 128])
def test_npdu_start0_stride_sweep(k):
    """Start 0: the first ceil(n/(ceil(k/2)+1)) picks are t*(ceil(k/2)+1)."""
    rng = np.random.default_rng(k)
    n = 1024
    pts = rng.random((n, 3), dtype=np.float32)
    stride = (k + 1) // 2 + 1
    sweep = -(-n // stride)
    got = oracle.afps(pts, min(n, sweep + 3), 1, k, 0)
    assert got[:sweep].tolist() == [t * stride for t in range(sweep)]


def test_composition_of_local_fps():
    rng = np.random.default_rng(8)
    pts = rng.random((517, 3), dtype=np.float32)
    c, m, start = 131, 6, 300
    got = oracle.afps(pts, c, m, None, start)
    parts = []
    for pp, ss in zip(np.array_split(np.arange(517), m), np.array_split(np.arange(c), m)):
        parts.append(pp[0] + oracle.fps(pts[pp], len(ss), start % len(pp)))
    assert got.tolist() == np.concatenate(parts).tolist()


@pytest.mark.parametrize("k", [None, 0, 5, 32])
def test_invariants_confinement_and_uniqueness(k):
    rng = np.random.default_rng(21)
    n, c, m, start = 1000, 200, 7, 123
    pts = rng.random((n, 3), dtype=np.float32)
    got = oracle.afps(pts, c, m, k, start)
    assert len(set(got.tolist())) == c
    for pp, ss in zip(np.array_split(np.arange(n), m), np.array_split(np.arange(c), m)):
        seg = got[ss]
        assert seg.min() >= pp[0] and seg.max() <= pp[-1]
        assert seg[0] == pp[0] + start % len(pp)


def test_fps_pick_distances_non_increasing_and_final_radius():
    rng = np.random.default_rng(9)
    pts = rng.random((400, 3), dtype=np.float32)
    idx, dist, _ = oracle.fps(pts, 60, 0, with_state=True)
    p64 = pts.astype(np.float64)
    d2 = np.full(400, np.inf)
    picked = []
    for i, t in enumerate(idx):
        if i:
            picked.append(d2[t])
        d2 = np.minimum(d2, ((p64 - p64[t]) ** 2).sum(1))
    assert all(a >= b - 1e-6 for a, b in zip(picked, picked[1:]))
    # the loop never applies the last sample's update; applying it gives the
    # squared coverage radius
    last = idx[-1]
    dx, dy, dz = (pts[:, a] - pts[last, a] for a in range(3))
    final = np.minimum(dist, (dx * dx + dy * dy) + dz * dz)
    from paper_2208_08795_amd.quality import coverage_radius
    assert math.isclose(math.sqrt(float(final.max())), coverage_radius(pts, idx), rel_tol=1e-5)


def test_gonzalez_two_approximation():
    rng = np.random.default_rng(13)
    for _ in range(30):
        n = int(rng.integers(3, 10))
        c = int(rng.integers(1, 4))
        pts = rng.random((n, 3), dtype=np.float32)
        p64 = pts.astype(np.float64)

        def radius(sel):
            return max(min(np.linalg.norm(p64[j] - p64[s]) for s in sel) for j in range(n))
        best = min(radius(sel) for sel in itertools.combinations(range(n), c))
        got = oracle.fps(pts, c, int(rng.integers(0, n)))
        assert radius(got) <= 2 * best + 1e-9


@pytest.mark.parametrize("k", [0, 3, 16])
def test_npdu_distance_is_an_upper_bound(k):
    """Under NPDU every stored distance is >= the true squared distance to the
    nearest sample whose update has been applied (all but the last)."""
    rng = np.random.default_rng(k + 40)
    pts = rng.random((300, 3), dtype=np.float32)
    idx, dist, _ = oracle.afps(pts, 50, 1, k, 0, with_state=True)
    applied = idx[:-1]
    d = np.full(300, np.float32(1e10))
    for t in applied:
        dx, dy, dz = (pts[:, a] - pts[t, a] for a in range(3))
        d = np.minimum(d, (dx * dx + dy * dy) + dz * dz)
    assert np.all(dist >= d)


@pytest.mark.parametrize("k", [None, 0, 1, 6, 31])
def test_update_counts_match_complexity(k):
    """AFPS evaluates (c_s - 1) * n_s distances per sector (Sec. III-B); NPDU
    evaluates exactly the window sizes of the samples it updates with, at most
    k + 1 per iteration (Sec. III-C)."""
    rng = np.random.default_rng(2)
    n, c, m, start = 777, 130, 5, 400
    pts = rng.random((n, 3), dtype=np.float32)
    idx, _, evals = oracle.afps(pts, c, m, k, start, with_state=True)
    want = 0
    for pp, ss in zip(np.array_split(np.arange(n), m), np.array_split(np.arange(c), m)):
        ns, cs = len(pp), len(ss)
        if k is None:
            want += (cs - 1) * ns
        else:
            for t in idx[ss][:-1] - pp[0]:
                lo, hi = max(0, t - k // 2), min(ns - 1, t + (k + 1) // 2)
                want += hi - lo + 1
    assert evals == want
    if k is not None:
        assert evals <= (c - m) * (k + 1)


def test_initial_distance_is_exact_in_fp32():
    assert float(np.float32(1e10)) == 1e10 == 9765625 * 2 ** 10


def test_argument_errors():
    pts = np.zeros((4, 3), np.float32)
    for c, m, start in [(0, 1, 0), (5, 1, 0), (2, 3, 0), (2, 0, 0), (2, 1, 4), (2, 1, -1)]:
        with pytest.raises(oracle.OracleError):
            oracle.afps(pts, c, m, None, start)


# ---------------------------------------------------------------- NPDU readings

FF, SH, SELF = oracle.NPDU_FIRST_FULL, oracle.NPDU_SHIFT_EDGES, oracle.NPDU_K_WITH_SELF


@pytest.mark.parametrize("flags", [FF, SH, SELF, FF | SH, FF | SELF, SH | SELF, FF | SH | SELF])
def test_bruteforce_agreement_npdu_readings(flags):
    """Every combination of the alternative NPDU readings equals the
    recomputation from scratch (windows formulated independently there)."""
    rng = np.random.default_rng(4321 + flags)
    for kind in ("uniform", "grid", "sorted", "dups"):
        for _ in range(25):
            n = int(rng.integers(1, 48))
            pts = _random_cloud(rng, n, kind)
            c = int(rng.integers(1, n + 1))
            m = int(rng.integers(1, c + 1))
            k = [1, 2, 3, 4, 5, 8, 13, 2 * n][int(rng.integers(0, 8))]
            start = int(rng.integers(0, n))
            want = bruteforce.afps(pts, c, m, k, start, flags)
            got = oracle.afps(pts, c, m, k, start, flags=flags)
            assert got.tolist() == want.tolist(), (kind, n, c, m, k, start, flags)


def test_k_with_self_is_the_default_window_one_smaller():
    """k points counting the sample = floor((k-1)/2) below and ceil((k-1)/2)
    above, which is the default window of k - 1 neighbours."""
    rng = np.random.default_rng(8)
    for _ in range(40):
        n = int(rng.integers(2, 300))
        pts = rng.random((n, 3), dtype=np.float32)
        c = int(rng.integers(1, n + 1))
        m = int(rng.integers(1, c + 1))
        k = int(rng.integers(1, 70))
        start = int(rng.integers(0, n))
        for extra in (0, FF, SH):
            assert oracle.afps(pts, c, m, k, start, flags=SELF | extra).tolist() == \
                oracle.afps(pts, c, m, k - 1, start, flags=extra).tolist()


def test_first_full_with_k0_picks_by_distance_from_start():
    """After one full update from the start point and windows holding only the
    sample, the picks are the points in decreasing order of their distance
    from the start (ties to the lowest index)."""
    rng = np.random.default_rng(9)
    for n in (5, 17, 64, 200):
        pts = rng.random((n, 3), dtype=np.float32)
        start = int(rng.integers(0, n))
        d = np.array([np.float32(np.float32(np.float32((p[0] - pts[start, 0]) ** 2) + np.float32((p[1] - pts[start, 1]) ** 2))
                                 + np.float32((p[2] - pts[start, 2]) ** 2)) for p in pts], dtype=np.float32)
        order = sorted(range(n), key=lambda j: (-float(d[j]), j))
        got = oracle.afps(pts, n, 1, 0, start, flags=FF)
        assert got.tolist() == [start] + order[:n - 1]


def test_readings_coincide_when_the_window_spans_the_sector():
    """k >= 2 n_s: every window covers the sector, so each reading is local FPS."""
    rng = np.random.default_rng(10)
    pts = rng.random((300, 3), dtype=np.float32)
    for m in (1, 3, 7):
        ref = oracle.afps(pts, 120, m, None, 11)
        for flags in (0, FF, SH, FF | SH, SELF, FF | SH | SELF):
            assert oracle.afps(pts, 120, m, 2 * 300 + 1, 11, flags=flags).tolist() == ref.tolist()


def test_shift_matches_truncation_away_from_the_edges():
    """With the start and every later window clear of both edges the two
    readings update the same points; at k = 0 a window never crosses an edge."""
    rng = np.random.default_rng(11)
    pts = rng.random((200, 3), dtype=np.float32)
    for start in (0, 57, 199):
        assert oracle.afps(pts, 80, 2, 0, start, flags=SH).tolist() == \
            oracle.afps(pts, 80, 2, 0, start).tolist()


def test_reading_flags_are_checked():
    pts = np.zeros((8, 3), np.float32)
    for bad in [dict(k=None, flags=FF), dict(k=0, flags=SELF), dict(k=3, flags=8)]:
        with pytest.raises(oracle.OracleError):
            oracle.afps(pts, 4, 1, bad["k"], 0, flags=bad["flags"])
