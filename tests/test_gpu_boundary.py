"""GPU tests of the batch entry points around the plan calls: the one-shot
afps_batched, the binding's batched() on the default and an explicit stream
(eager and graph), and the stamped launch whose per-sector timestamps give
cycles per iteration; every index against the oracle (tolerance 0)."""
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


@pytest.fixture(scope="module")
def batch256():
    clouds = synth.batch_of_objects(256, seed=0)
    cs = [len(p) // 4 for p in clouds]
    want = [oracle.afps(p, c, 8, 32, 0) for p, c in zip(clouds, cs)]
    return clouds, cs, want


def test_one_shot_afps_batched_on_the_batch_of_256(env, batch256):
    torch, B, dev = env
    clouds, cs, want = batch256
    sizes = [len(p) for p in clouds]
    print("afps_batched: 256 clouds, %d points" % sum(sizes), flush=True)
    xyz = torch.from_numpy(np.concatenate(clouds)).to(dev)
    for stream in (None, torch.cuda.Stream(device=dev)):
        if stream is not None:
            stream.wait_stream(torch.cuda.current_stream())
        out = B.batched_oneshot(xyz, sizes, cs, [8] * 256, [32] * 256, [0] * 256, stream=stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        o = 0
        for i, c in enumerate(cs):
            assert np.array_equal(got[o:o + c], want[i]), (stream is not None, i)
            o += c


def test_one_shot_rejects_bad_descriptors_without_launching(env):
    torch, B, dev = env
    xyz = torch.zeros((100, 3), dtype=torch.float32, device=dev)
    out = torch.full((70,), -7, dtype=torch.int32, device=dev)
    with pytest.raises(B.AfpsError) as e:
        B.batched_oneshot(xyz, [50, 50], [10, 60], [1, 1], [None, 4], [0, 0], out_all=out)
    assert e.value.status == -2
    torch.cuda.synchronize()
    assert bool((out == -7).all())


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("explicit_stream", [False, True])
def test_binding_batched_streams(env, batch256, graph, explicit_stream):
    torch, B, dev = env
    clouds, cs, want = batch256
    print("binding.batched graph=%s explicit_stream=%s" % (graph, explicit_stream), flush=True)
    tensors = [torch.from_numpy(p).to(dev) for p in clouds]
    stream = torch.cuda.Stream(device=dev) if explicit_stream else None
    res = B.batched(tensors, cs, [8] * 256, [32] * 256, graph=graph, stream=stream)
    # results are ready on the current stream without a further synchronisation
    host = [r.cpu().numpy() for r in res]
    for i, w in enumerate(want):
        assert np.array_equal(host[i], w), i


def test_stamped_launch_is_exact_and_its_stamps_are_consistent(env, batch256):
    torch, B, dev = env
    clouds, cs, want = batch256
    sizes = [len(p) for p in clouds]
    plan = B.BatchPlan(sizes, cs, [8] * 256, [32] * 256, [0] * 256, device=dev)
    xyz = torch.from_numpy(np.concatenate(clouds)).to(dev)
    print("stamped launch: %d items" % plan.items, flush=True)
    out, stamps = plan.launch_stamped(xyz)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i, w in enumerate(want):
        o = plan.offsets[i]
        assert np.array_equal(got[o:o + cs[i]], w), i
    st = stamps.cpu().numpy()
    pairs = st[:, 5:8].copy().view(np.int32).reshape(-1, 6)   # item, n, c, k, hw_id, xcc_id
    take, loaded, end, take_rt, end_rt = (st[:, j] for j in range(5))
    assert np.array_equal(pairs[:, 0], np.arange(plan.items))          # every item stamped once
    assert sorted(pairs[:, 1].tolist()) == sorted(
        n // 8 + (s < n % 8) for n in sizes for s in range(8))        # its sector's points
    assert np.all(pairs[:, 3] == 32)
    assert np.all(take <= loaded) and np.all(loaded <= end) and np.all(take_rt < end_rt)
    # the shader clock's rate from the two counters: a plausible engine clock
    khz = int(B.lib().afps_wall_clock_khz())
    assert khz > 0
    ghz = (end - take).sum() / (end_rt - take_rt).sum() * khz * 1e-6
    print("shader clock from stamps: %.3f GHz" % ghz, flush=True)
    assert 0.5 < ghz < 3.0
    many = pairs[:, 2] > 1
    cyc = (end - loaded)[many] / (pairs[many, 2] - 1)
    print("cycles per iteration: median %.0f, max %.0f" % (np.median(cyc), cyc.max()), flush=True)
    assert 100 < np.median(cyc) < 5000
    plan.close()


# Pooled launch policies of the launches of several rounds: the built-in one
# (coordinates in LDS records), registers at 8 waves per CU, L2 at 16, and the
# light kernel of two 16-wave workgroups per CU.
ROUND_POLICIES = {"builtin": None, "regs_8": (8, 1), "l2_16": (16, 1), "lite_16x2": (16, 2)}


def _set_round_policy(B, name):
    B.tune_npdu_clear()
    shape = ROUND_POLICIES[name]
    if shape is not None:
        B.set_pool_policy(shape[0], shape[1], True, 3)
        B.tune_npdu(4096, 64, False)
    return shape


@pytest.mark.parametrize("policy", list(ROUND_POLICIES))
def test_rounds_in_one_launch_equal_separate_launches(env, policy):
    """Several rounds of one plan in one pooled launch, alternating two inputs
    of the same layout, every round writing its own output: each round equals
    a separate launch of the plan on that input (and the oracle on samples);
    one round equals afps_plan_launch; a graph capture replays exactly; under
    every pooled policy (placements in LDS, registers and L2, the light
    kernel)."""
    torch, B, dev = env
    shape = _set_round_policy(B, policy)
    try:
        _rounds_case(torch, B, dev, shape)
    finally:
        B.tune_npdu_clear()


def _rounds_case(torch, B, dev, shape):
    sizes = [int(n) for n in np.exp(np.random.default_rng(4).uniform(np.log(1024), np.log(32768), 48)).round()]
    cs = [n // 4 for n in sizes]
    inputs = []
    for seed in (0, 1):
        clouds = [synth.object_cloud(n, seed=1000 * seed + i) for i, n in enumerate(sizes)]
        inputs.append((clouds, torch.from_numpy(np.concatenate(clouds)).to(dev)))
    plan = B.BatchPlan(sizes, cs, [8] * 48, [32] * 48, [0] * 48, device=dev)
    if shape is not None:
        assert (plan.pool_waves, plan.pool_groups) == shape
    want = []
    for clouds, xyz in inputs:
        want.append(plan.launch(xyz).clone())
    torch.cuda.synchronize()
    for i in (0, 17, 47):
        o = plan.offsets[i]
        assert np.array_equal(want[1][o:o + cs[i]].cpu().numpy(), oracle.afps(inputs[1][0][i], cs[i], 8, 32, 0)), i
    for count in (1, 2, 7):
        outs = [torch.full((plan.total_samples,), -7, dtype=torch.int32, device=dev) for _ in range(count)]
        rounds = [(inputs[r % 2][1], outs[r]) for r in range(count)]
        print("rounds: %d" % count, flush=True)
        table = plan.launch_rounds(rounds)
        torch.cuda.synchronize()
        plan.status()
        for r in range(count):
            assert torch.equal(outs[r], want[r % 2]), (count, r)
    # a captured launch of several rounds, replayed with eager work in between
    outs = [torch.full((plan.total_samples,), -7, dtype=torch.int32, device=dev) for _ in range(3)]
    table = plan.round_table([(inputs[r % 2][1], outs[r]) for r in range(3)])
    plan.launch_rounds(table)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.launch_rounds(table, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for o in outs:
            o.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        torch.zeros(1000, device=dev).sum().item()
        for r in range(3):
            assert torch.equal(outs[r], want[r % 2]), ("graph", rep, r)
    plan.close()


@pytest.mark.parametrize("policy", list(ROUND_POLICIES))
def test_rounds_forced_timeouts_fail_whole_sectors(env, policy):
    """A spin limit of 1 in a launch of several rounds: every sector of every
    round is exact or entirely -1, the plan reports the failure, and the next
    launch of several rounds is exact again; under every pooled policy."""
    torch, B, dev = env
    clouds = synth.batch_of_objects(64, seed=9, n_min=2048, n_max=32768)
    sizes, cs = [len(p) for p in clouds], [len(p) // 4 for p in clouds]
    xyz = torch.from_numpy(np.concatenate(clouds)).to(dev)
    shape = _set_round_policy(B, policy)
    try:
        plan = B.BatchPlan(sizes, cs, [8] * 64, [32] * 64, [0] * 64, device=dev)
    finally:
        B.tune_npdu_clear()
    if shape is not None:
        assert (plan.pool_waves, plan.pool_groups) == shape
    want = plan.launch(xyz).clone().cpu().numpy()
    outs = [torch.full((plan.total_samples,), -7, dtype=torch.int32, device=dev) for _ in range(3)]
    table = plan.round_table([(xyz, o) for o in outs])
    B.clear_device_status()
    B.set_spin_limit(1)
    try:
        plan.launch_rounds(table)
        torch.cuda.synchronize()
    finally:
        B.set_spin_limit(1 << 22)
    failed = 0
    for o in outs:
        got = o.cpu().numpy()
        failed += int((got == -1).sum())
        for i, c in enumerate(cs):
            base = plan.offsets[i]
            for s_ in range(8):
                lo = base + s_ * (c // 8) + min(s_, c % 8)
                cc = c // 8 + (s_ < c % 8)
                sector = got[lo:lo + cc]
                assert np.array_equal(sector, want[lo:lo + cc]) or np.all(sector == -1), (i, s_)
    if failed:
        with pytest.raises(B.AfpsError):
            plan.status()
    B.clear_device_status()
    plan.launch_rounds(table)
    torch.cuda.synchronize()
    plan.status()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), want)
    plan.close()
