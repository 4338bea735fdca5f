"""GPU parity of the grouping kernel (ball query around the samples) with the
oracle: every index and every count, bit for bit (the kernel takes each
decision in fp32 with the oracle's operation order)."""
import numpy as np
import pytest

import oracle
from paper_2208_08795_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_08795_amd import binding
    binding.lib()
    return binding, torch, torch.device("cuda:0")


def _check(env, pts, centers, radius, k, window, label):
    B, torch, dev = env
    print("case %s n=%d c=%d radius=%g k=%d window=%s" % (label, len(pts), len(centers), radius, k, window),
          flush=True)
    xyz = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).to(dev)
    ctr = torch.from_numpy(np.ascontiguousarray(centers, dtype=np.int32)).to(dev)
    idx, cnt = B.ball_query(xyz, ctr, radius, k, window)
    torch.cuda.synchronize()
    want_idx, want_cnt = oracle.ball_query(pts, centers, radius, k, window)
    got_idx, got_cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    assert np.array_equal(got_cnt, want_cnt), label
    if not np.array_equal(got_idx, want_idx):
        bad = np.argwhere(got_idx != want_idx)[0]
        raise AssertionError("%s: first mismatch at centre %d slot %d: got %d want %d" %
                             (label, bad[0], bad[1], got_idx[tuple(bad)], want_idx[tuple(bad)]))


def test_random_clouds(env):
    rng = np.random.default_rng(71)
    for it in range(60):
        n = int(rng.integers(1, 3000))
        pts = synth.object_cloud(n, int(rng.integers(0, 1 << 30))) if it % 2 else rng.random((n, 3), dtype=np.float32)
        c = int(rng.integers(1, 300))
        centers = rng.integers(0, n, c)
        radius = [0.0, 0.02, 0.1, 0.3, 2.0][int(rng.integers(0, 5))]
        k = [1, 2, 16, 32, 63, 64, 65, 100, 257][int(rng.integers(0, 9))]
        window = [None, None, 0, 1, 63, 64, 100, 1000, 1 << 30][int(rng.integers(0, 9))]
        _check(env, pts, centers, radius, k, window, "random-%d" % it)


def test_ties_on_the_sphere(env):
    """Integer grid points: many squared distances equal r2 exactly, and the
    strict comparison decides them."""
    rng = np.random.default_rng(72)
    pts = rng.integers(0, 6, (2000, 3)).astype(np.float32)
    centers = rng.integers(0, 2000, 200)
    for radius in (1.0, 2.0, np.sqrt(np.float32(5.0)), 3.0):
        for window in (None, 40):
            _check(env, pts, centers, float(radius), 48, window, "grid")


def test_edges(env):
    B, torch, dev = env
    rng = np.random.default_rng(73)
    one = rng.random((1, 3), dtype=np.float32)
    _check(env, one, [0, 0], 0.5, 4, None, "one-point")
    pts = rng.random((300, 3), dtype=np.float32)
    _check(env, pts, np.arange(300), 10.0, 400, None, "k-above-n")
    _check(env, pts, np.arange(300), 0.0, 3, 5, "radius-0")
    _check(env, pts, [0, 299, 150], 0.5, 64, 1 << 30, "huge-window")
    dup = np.repeat(rng.random((30, 3), dtype=np.float32), 4, axis=0)
    _check(env, dup, [0, 5, 119], 0.2, 8, 3, "duplicates")
    # a centre outside the cloud: -1 in all its slots and in its count, the others exact
    xyz = torch.from_numpy(pts).to(dev)
    ctr = torch.tensor([3, 300, -1, 7], dtype=torch.int32, device=dev)
    idx, cnt = B.ball_query(xyz, ctr, 0.3, 5)
    torch.cuda.synchronize()
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    assert np.all(idx[1:3] == -1) and cnt[1] == -1 and cnt[2] == -1
    want_idx, want_cnt = oracle.ball_query(pts, [3, 7], 0.3, 5)
    assert np.array_equal(idx[[0, 3]], want_idx) and np.array_equal(cnt[[0, 3]], want_cnt)


def test_lidar_frame_around_its_samples(env):
    """The LiDAR frame of 32768 points, centres from the GPU's own AFPS-NPDU
    samples (M = 16, k = 64, 8192 samples), k = 32 neighbours within 1 m:
    every row for the exact query and for storage windows."""
    B, torch, dev = env
    pts = synth.lidar_scan(512, 0)
    xyz = torch.from_numpy(pts).to(dev)
    samples = B.afps_npdu(xyz, 8192, 16, 64, 0)
    torch.cuda.synchronize()
    centers = samples.cpu().numpy()
    for window in (None, 1024, 256, 64):
        _check(env, pts, centers, 1.0, 32, window, "lidar")


def test_sampling_binning_grouping_in_one_graph(env):
    """The single-cloud sampler, the binning and the ball query are kernel
    launches only: captured together in one graph, every replay (with eager
    work in between) equals the eager results."""
    B, torch, dev = env
    pts = synth.lidar_scan(512, 1)
    xyz = torch.from_numpy(pts).to(dev)

    def pipeline():
        samples = B.afps_npdu(xyz, 8192, 16, 64, 0)
        perm, binned = B.bin_points(xyz, 0, 64)
        idx, cnt = B.ball_query(xyz, samples, 1.0, 32, 256)
        return samples, perm, binned, idx, cnt

    eager = [t.clone() for t in pipeline()]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):          # warm-up on the capture stream
        pipeline()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        static = pipeline()
    for r in range(3):
        for t in static:
            t.fill_(-7)
        graph.replay()
        torch.cuda.synchronize()
        for got, want in zip(static, eager):
            assert torch.equal(got, want), "replay %d" % r
        torch.zeros(1000, device=dev).sum().item()   # eager work between replays
    want_idx, want_cnt = oracle.ball_query(pts, eager[0].cpu().numpy(), 1.0, 32, 256)
    assert np.array_equal(eager[3].cpu().numpy(), want_idx) and np.array_equal(eager[4].cpu().numpy(), want_cnt)
