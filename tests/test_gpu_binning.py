"""Binning along one axis on the GPU (Sec. III-A) against the oracle: the
permutation bit for bit, the binned points, and AFPS on a binned cloud."""
import numpy as np
import pytest

import oracle
from oracle import binning as obin
from paper_2208_08795_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_08795_amd import binding
    binding.lib()
    return torch, binding


def _case(torch, B, pts, axis, bins, label):
    print("binning %s n=%d axis=%d bins=%d" % (label, len(pts), axis, bins), flush=True)
    xyz = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).cuda()
    perm, out = B.bin_points(xyz, axis, bins)
    torch.cuda.synchronize()
    want, _ = obin.bin_points(pts, axis, bins)
    got = perm.cpu().numpy()
    assert np.array_equal(got, want), label
    assert np.array_equal(out.cpu().numpy(), pts[want]), label


def test_binning_matches_oracle(env):
    torch, B = env
    rng = np.random.default_rng(31)
    for n, bins in [(1, 1), (1, 7), (63, 4), (64, 64), (4095, 32), (4096, 32), (4097, 33), (10000, 1),
                    (10000, 8192), (131072, 1024), (300001, 2347)]:
        pts = (rng.standard_normal((n, 3)) * 30).astype(np.float32)
        _case(torch, B, pts, int(rng.integers(0, 3)), bins, "random")
    ties = rng.integers(-5, 6, (20000, 3)).astype(np.float32)      # equal coordinates, crowded bins
    for bins in (3, 11, 128):
        _case(torch, B, ties, 2, bins, "ties")
    const = np.zeros((5000, 3), np.float32)
    const[:, 1] = 7.0
    _case(torch, B, const, 1, 64, "constant")
    scan = synth.lidar_scan(512, 3)
    _case(torch, B, scan[rng.permutation(len(scan))], 0, len(scan) // 128, "shuffled-lidar")


def test_afps_on_binned_cloud(env):
    """An unsorted cloud binned on the GPU, then AFPS / NPDU on it, equals the
    oracle's AFPS on the oracle's binning."""
    torch, B = env
    rng = np.random.default_rng(32)
    pts = synth.object_cloud(8192, 5)
    pts = pts[rng.permutation(len(pts))]
    xyz = torch.from_numpy(pts).cuda()
    _, binned = B.bin_points(xyz, 0, 64)
    want_pts = pts[obin.bin_points(pts, 0, 64)[0]]
    for m, k in [(8, None), (32, None), (8, 32)]:
        got = (B.afps(binned, 2048, m, 0) if k is None else B.afps_npdu(binned, 2048, m, k, 0)).cpu().numpy()
        assert np.array_equal(got, oracle.afps(want_pts, 2048, m, k, 0)), (m, k)
