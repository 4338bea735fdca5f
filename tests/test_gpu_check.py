"""Input check (afps_check_points / checking mode) on the GPU: non-finite
coordinates and extents whose squared distances could reach the initial 1e10
are reported with the offending point or cloud, before anything is sampled."""
import numpy as np
import pytest

from paper_2208_08795_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_08795_amd import binding
    binding.lib()
    yield torch, binding
    binding.set_checking(False)


def _dev(torch, pts):
    return torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).cuda()


def test_check_points_accepts_and_rejects(env):
    torch, B = env
    good = synth.object_cloud(5000, 3)
    B.check_points(_dev(torch, good))
    for bad_value, where in ((np.nan, 123), (np.inf, 4999), (-np.inf, 0)):
        pts = good.copy()
        pts[where, 1] = bad_value
        print("case non-finite", bad_value, where, flush=True)
        with pytest.raises(B.AfpsError) as e:
            B.check_points(_dev(torch, pts))
        assert e.value.status == -8 and ("point %d " % where) in str(e.value)
    # extent: a diagonal just below and just above 1e5
    inside = np.zeros((3, 3), np.float32)
    inside[1] = (99000.0, 0.0, 0.0)
    inside[2] = (0.0, 13000.0, 0.0)
    B.check_points(_dev(torch, inside))
    outside = inside.copy()
    outside[2] = (0.0, 15000.0, 0.0)          # 99000^2 + 15000^2 > 1e10
    with pytest.raises(B.AfpsError) as e:
        B.check_points(_dev(torch, outside))
    assert e.value.status == -8 and "diagonal" in str(e.value)


def test_checking_mode_rejects_before_sampling(env):
    torch, B = env
    pts = synth.object_cloud(3000, 4)
    pts[1500, 0] = np.nan
    xyz = _dev(torch, pts)
    out = torch.full((600,), 7, dtype=torch.int32, device="cuda")
    B.set_checking(True)
    try:
        for call in (lambda: B.fps(xyz, 600, 0, out=out), lambda: B.afps(xyz, 600, 4, 0, out=out),
                     lambda: B.afps_npdu(xyz, 600, 4, 32, 0, out=out)):
            with pytest.raises(B.AfpsError) as e:
                call()
            assert e.value.status == -8 and "point 1500 " in str(e.value)
        torch.cuda.synchronize()
        assert bool((out == 7).all())                         # nothing was launched
        # a batch: the failing cloud is named, on eager and on graph launches
        clouds = [synth.object_cloud(n, 10 + i) for i, n in enumerate((1500, 2500, 1800))]
        clouds[2][17, 2] = np.inf
        xyz_all = _dev(torch, np.concatenate(clouds))
        plan = B.BatchPlan([len(p) for p in clouds], [300, 500, 360], [4, 4, 4], [32, 32, 32], [0, 0, 0])
        try:
            for graph in (False, True):
                with pytest.raises(B.AfpsError) as e:
                    plan.launch(xyz_all, graph=graph)
                assert e.value.status == -8 and "cloud 2: point 17 " in str(e.value)
        finally:
            plan.close()
        # valid inputs still sample, and equal the unchecked result
        good = _dev(torch, synth.object_cloud(3000, 5))
        a = B.afps_npdu(good, 600, 4, 32, 0).cpu().numpy()
        B.set_checking(False)
        b = B.afps_npdu(good, 600, 4, 32, 0).cpu().numpy()
        assert np.array_equal(a, b)
    finally:
        B.set_checking(False)
