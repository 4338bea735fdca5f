"""afps_plan_launch_noalloc, the batch launch whose workspace is the library's
static per-GPU scratch, against afps_plan_launch with a caller workspace:
identical indices (tolerance 0) on two calls in a row, the second with a
smaller batch, and a plan larger than the scratch rejected before anything
is copied or launched."""
import ctypes

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
    return torch, binding, torch.device("cuda:0")


def _mixed_batch(rng, count):
    """Plain FPS, AFPS and NPDU clouds of uneven size (several launches)."""
    clouds, cs, ms, ks = [], [], [], []
    for i in range(count):
        n = int(rng.integers(300, 12000))
        clouds.append(synth.object_cloud(n, seed=int(rng.integers(0, 1 << 30))))
        cs.append(max(1, n // 8))
        ms.append(1 if i % 3 == 0 else int(rng.integers(2, 9)))
        ks.append(None if i % 3 < 2 else int(rng.integers(0, 70)))
    return clouds, cs, ms, ks


def test_noalloc_launch_equals_workspace_launch(env):
    torch, B, dev = env
    rng = np.random.default_rng(31)
    big = synth.batch_of_objects(256, seed=0)
    cases = [("batch of 256, M=8, k=32", big, [len(p) // 4 for p in big], [8] * 256, [32] * 256)]
    cases.append(("mixed batch of 24",) + _mixed_batch(rng, 24))
    for label, clouds, cs, ms, ks in cases:
        sizes = [len(p) for p in clouds]
        starts = [int(rng.integers(0, n)) for n in sizes]
        print("noalloc case: %s, %d points, %d samples" % (label, sum(sizes), sum(cs)), flush=True)
        plan = B.BatchPlan(sizes, cs, ms, ks, starts, device=dev)
        assert plan.items <= B.lib().afps_noalloc_max_items()
        xyz = torch.from_numpy(np.concatenate(clouds)).to(dev)
        want = plan.launch(xyz)
        got = torch.full_like(want, -7)
        plan.launch_noalloc(xyz, out_all=got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), label
        g = got.cpu().numpy()
        for i in (0, len(clouds) // 2, len(clouds) - 1):
            o = plan.offsets[i]
            assert np.array_equal(g[o:o + cs[i]], oracle.afps(clouds[i], cs[i], ms[i], ks[i], starts[i])), (label, i)
        plan.close()


def test_noalloc_rejects_a_plan_larger_than_the_scratch(env):
    torch, B, dev = env
    limit = int(B.lib().afps_noalloc_max_items())
    count = limit // 32 + 1                      # 32 sectors per cloud: one sector too many at least
    plan = B.BatchPlan([64] * count, [32] * count, [32] * count, [8] * count, [0] * count, device=dev)
    assert plan.items > limit
    xyz = torch.zeros((64 * count, 3), dtype=torch.float32, device=dev)
    out = torch.full((plan.total_samples,), -7, dtype=torch.int32, device=dev)
    with pytest.raises(B.AfpsError) as e:
        plan.launch_noalloc(xyz, out_all=out)
    assert e.value.status == -4 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == -7).all())               # nothing launched
    L = B.lib()
    assert L.afps_plan_launch_noalloc(None, ctypes.c_void_p(xyz.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      None) == -1
    plan.close()
