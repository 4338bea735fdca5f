"""Serving on the GPU: every frame's indices in the mix equal the same frame
sampled alone (tolerance 0), and spot checks against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2208_08795_amd import synth

pytestmark = pytest.mark.gpu


def _requests(torch, frames, fps=False):
    from paper_2208_08795_amd.serve import Request
    reqs = []
    for i, f in enumerate(frames):
        pts = torch.from_numpy(f.points).pin_memory()
        m, k = (1, None) if fps else (f.m, f.k)
        reqs.append(Request(rid=i, n=f.points.shape[0], c=f.c, m=m, k=k, start=f.start,
                            arrival=f.arrival, points=pts))
    return reqs


@pytest.mark.parametrize("fps", [False, True])
def test_served_in_mix_equals_alone(fps):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_08795_amd import binding
    from paper_2208_08795_amd.serve import GpuExecutor, Scheduler, latency_summary
    count = 10 if fps else 24
    frames = synth.frame_stream(rate=3000.0, count=count, seed=5, n_min=4096,
                                n_max=40000 if fps else 60000)
    reqs = _requests(torch, frames, fps)
    budget = 6 << 20
    ex = GpuExecutor(budget, streams=4, keep_results=True)
    s = Scheduler(ex, budget, max_inflight=6, max_batch=8)
    print("serving %d frames (fps=%s)" % (count, fps), flush=True)
    done = s.run(reqs)
    torch.cuda.synchronize()
    print(latency_summary(done), flush=True)
    assert all(r.state == "done" for r in done), [(r.rid, r.state, r.error) for r in done]
    assert s.peak_bytes <= budget
    for r in sorted(done, key=lambda r: r.rid):
        x = torch.from_numpy(frames[r.rid].points).cuda()
        if fps:
            alone = binding.fps(x, r.c, r.start)
        else:
            alone = binding.afps_npdu(x, r.c, r.m, r.k, r.start)
        torch.cuda.synchronize()
        assert np.array_equal(r.result.numpy(), alone.cpu().numpy()), "frame %d" % r.rid
    for r in sorted(done, key=lambda r: r.rid)[:3]:
        want = oracle.afps(frames[r.rid].points, r.c, r.m, r.k, r.start)
        assert np.array_equal(r.result.numpy(), want), "oracle frame %d" % r.rid
