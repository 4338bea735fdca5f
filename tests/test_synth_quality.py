"""Seeded generators produce the stated shapes and orderings; the coverage
radius evaluator equals its brute-force definition."""
import math

import numpy as np

from paper_2208_08795_amd import synth
from paper_2208_08795_amd.quality import coverage_radius


def test_uniform_cube_sorted_and_seeded():
    a = synth.uniform_cube(2048, 0)
    assert a.shape == (2048, 3) and a.dtype == np.float32 and a.flags.c_contiguous
    assert np.all(np.diff(a[:, 0]) >= 0)
    assert np.array_equal(a, synth.uniform_cube(2048, 0))
    assert not np.array_equal(a, synth.uniform_cube(2048, 1))


def test_object_cloud_approximately_sorted():
    p = synth.object_cloud(8192, 3, window=16)
    assert p.shape == (8192, 3) and p.dtype == np.float32
    assert abs(np.linalg.norm(p, axis=1).max() - 1.0) < 1e-5
    bins = p[:, 0].reshape(-1, 16)
    # bins are ordered: every point of a later bin >= every point of an earlier bin
    assert np.all(bins.max(axis=1)[:-1] <= bins.min(axis=1)[1:])
    assert not np.all(np.diff(p[:, 0]) >= 0)          # but not exactly sorted
    assert np.unique(p, axis=0).shape[0] == 8192      # distinct points


def test_lidar_scan_firing_order():
    p = synth.lidar_scan(512, 0)
    assert p.shape == (32768, 3) and p.dtype == np.float32
    az = np.arctan2(p[:, 1], p[:, 0]) % (2 * math.pi)
    col = np.arange(32768) // 64
    # azimuth grows with the column (up to noise and the wrap at 2*pi)
    mean_az = np.array([np.median(az[col == c]) for c in range(0, 512, 32)])
    assert np.all(np.diff(mean_az) > 0)
    r = np.linalg.norm(p[:, :2], axis=1)
    assert r.max() < 60.5 and p[:, 2].min() > -0.2
    q = synth.lidar_scan(300, 1, n=19000)
    assert q.shape == (19000, 3)


def test_batch_and_stream():
    clouds = synth.batch_of_objects(8, 0)
    assert len(clouds) == 8 and all(1024 <= c.shape[0] <= 32768 for c in clouds)
    frames = synth.frame_stream(200.0, 3, 0, n_min=16384, n_max=20000)
    assert [f.arrival for f in frames] == sorted(f.arrival for f in frames)
    assert all(f.c == f.points.shape[0] // 8 and f.m in (8, 16, 32) for f in frames)


def test_coverage_radius_brute_force():
    rng = np.random.default_rng(0)
    p = rng.standard_normal((200, 3)).astype(np.float32)
    idx = rng.choice(200, 17, replace=False)
    p64 = p.astype(np.float64)
    want = max(min(math.dist(p64[j], p64[s]) for s in idx) for j in range(200))
    assert math.isclose(coverage_radius(p, idx), want, rel_tol=1e-12)
