"""GPU parity: every kernel path, index for index against the CPU oracle.

Squared distances use the same fp32 operation order on both sides with
contraction off, and argmax ties go to the lowest index, so the sampled
indices must be identical (tolerance 0).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2208_08795_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def B():
    from paper_2208_08795_amd import binding
    binding.lib()
    return binding


def _run(B, torch, xyz_t, c, m, k, start, variant=None, flags=0):
    if k is None and m == 1 and variant is None:
        out = B.fps(xyz_t, c, start)
    elif k is None:
        out = B.afps(xyz_t, c, m, start, variant=variant)
    else:
        out = B.afps_npdu(xyz_t, c, m, k, start, variant=variant, flags=flags)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(B, torch, dev, pts, c, m, k, start, variant=None, label="", flags=0):
    print("case %s n=%d c=%d m=%d k=%s start=%d variant=%s flags=%d" % (label, len(pts), c, m, k, start,
                                                                       variant, flags), flush=True)
    xyz = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).to(dev)
    got = _run(B, torch, xyz, c, m, k, start, variant, flags)
    want = oracle.afps(pts, c, m, k, start, flags=flags)
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError("%s: %d mismatches, first at %d: got %d want %d" %
                             (label, bad.size, bad[0], got[bad[0]], want[bad[0]]))


def test_hand_examples(B, torch_dev):
    torch, dev = torch_dev
    with open(GOLDEN) as f:
        for case in json.load(f)["cases"]:
            pts = np.array(case["points"], dtype=np.float32)
            xyz = torch.from_numpy(pts).to(dev)
            got = _run(B, torch, xyz, case["c"], case["m"], case["k"], case["start"], flags=case.get("flags", 0))
            assert got.tolist() == case["expected"], case["name"]


@pytest.mark.parametrize("kind", ["uniform", "grid", "sorted", "object"])
def test_random_small_cases(B, torch_dev, kind):
    torch, dev = torch_dev
    rng = np.random.default_rng(2024)
    for it in range(40):
        n = int(rng.integers(1, 5000))
        if kind == "uniform":
            pts = rng.random((n, 3), dtype=np.float32)
        elif kind == "grid":         # exact ties everywhere
            pts = rng.integers(0, 4, (n, 3)).astype(np.float32)
        elif kind == "sorted":
            pts = synth.uniform_cube(n, int(rng.integers(0, 1 << 30)))
        else:
            pts = synth.object_cloud(max(n, 1), int(rng.integers(0, 1 << 30)))
        c = int(rng.integers(1, min(n, 700) + 1))
        m = int(rng.integers(1, min(c, 40) + 1))
        k = [None, None, 0, 1, 7, 32, 64, 129, 4 * n][int(rng.integers(0, 9))]
        start = int(rng.integers(0, n))
        _check(B, torch, dev, pts, c, m, k, start, label="%s-%d" % (kind, it))


def test_edge_cases(B, torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(5)
    one = rng.random((1, 3), dtype=np.float32)
    for k in (None, 0, 5):
        _check(B, torch, dev, one, 1, 1, k, 0, label="single-point")
    pts = rng.random((300, 3), dtype=np.float32)
    for c, m, k, start in [(300, 1, None, 299), (300, 300, None, 17), (300, 300, 3, 17), (1, 1, None, 5),
                           (300, 7, 0, 0), (300, 1, 0, 150), (299, 13, 1 << 30, 2)]:
        _check(B, torch, dev, pts, c, m, k, start, label="edge")
    dup = np.repeat(rng.random((40, 3), dtype=np.float32), 5, axis=0)   # duplicate points
    for k in (None, 3):
        _check(B, torch, dev, dup, 150, 3, k, 7, label="duplicates")


def test_every_full_variant_agrees(B, torch_dev):
    """All (waves, slots) variants give the oracle's indices (also exercises
    the cross-wave LDS reduction at every wave count)."""
    torch, dev = torch_dev
    for waves in (1, 2, 4, 8, 16):
        for slots in (1, 2, 4, 8, 12, 16, 24, 32):
            cap = 64 * waves * slots
            n = max(2, cap - 37)          # ragged last slot
            pts = synth.object_cloud(n, seed=waves * 100 + slots)
            _check(B, torch, dev, pts, min(n, 300), 1, None, n // 3, variant=(waves, slots),
                   label="variant")
            if cap >= 128:
                _check(B, torch, dev, pts, min(n, 300), 3, None, 1, variant=(waves, slots),
                       label="variant-m3")


@pytest.mark.parametrize("q", [1, 2, 4, 8])
def test_every_npdu_variant_agrees(B, torch_dev, q):
    torch, dev = torch_dev
    n = 4096 * q - 101
    pts = synth.object_cloud(n, seed=q)
    for k, m, start in [(8, 1, 0), (64, 1, n // 2), (33, 2, 5), (200, 1, 17)]:
        ns = -(-n // m)
        if ns > 4096 * q:
            continue
        _check(B, torch, dev, pts, min(n // 4, 2000), m, k, start, variant=(1, q), label="npdu-q%d" % q)


def test_npdu_narrow_window_edges(B, torch_dev):
    """One-wave NPDU for windows of at most two blocks (k <= 64): sectors of
    exactly 4096 points (the window's second block is past the last lane),
    windows touching either end, exact ties, every point sampled, k on both
    sides of 64, and sectors of one or two blocks."""
    torch, dev = torch_dev
    rng = np.random.default_rng(77)
    full = synth.object_cloud(4096, seed=11)
    ties = rng.integers(0, 3, (4096, 3)).astype(np.float32)
    for pts, c, m, k, start in [(full, 4096, 1, 64, 4095), (full, 1500, 1, 63, 4095),
                                (full, 1500, 1, 65, 4095), (full, 2000, 1, 1, 0),
                                (full, 2000, 1, 0, 2048), (full, 4096, 1, 2, 0),
                                (ties, 4096, 1, 64, 4000), (ties, 3000, 1, 31, 64),
                                (full, 4096, 2, 64, 4095)]:
        _check(B, torch, dev, pts, c, m, k, start, variant=(1, 1) if m == 1 else None,
               label="narrow")
    for n in (1, 2, 63, 64, 65, 127, 128, 129):
        pts = rng.random((n, 3), dtype=np.float32)
        for k in (0, 1, 64):
            _check(B, torch, dev, pts, n, 1, k, n - 1, label="narrow-small")


def test_npdu_windows_up_to_32(B, torch_dev):
    """k <= 32 on sectors up to 4096 points: sizes around 32- and 64-point
    boundaries, windows in the last block and at both ends, k = 0 to 32,
    every reading, ties, every point sampled, several sectors."""
    torch, dev = torch_dev
    rng = np.random.default_rng(88)
    for n in (1, 2, 31, 32, 33, 63, 64, 65, 95, 96, 97, 2047, 4063, 4064, 4065, 4095, 4096):
        pts = synth.object_cloud(n, seed=n) if n > 8 else rng.random((n, 3), dtype=np.float32)
        for k, flags, start in [(0, 0, 0), (1, 0, n - 1), (2, 2, n // 2), (31, 0, n - 1), (32, 0, 0),
                                (32, 1, n // 3), (17, 3, n - 1), (32, 2, n - 2 if n > 1 else 0)]:
            _check(B, torch, dev, pts, n if n <= 1024 else 1024, 1, k, start, variant=(1, 1),
                   label="k32-%d" % n, flags=flags)
    ties = rng.integers(0, 3, (4096, 3)).astype(np.float32)
    for k in (8, 32):
        _check(B, torch, dev, ties, 4096, 1, k, 4095, variant=(1, 1), label="k32-ties")
    cloud = synth.object_cloud(20000, seed=3)
    for m, k in [(5, 32), (8, 16), (16, 1)]:
        _check(B, torch, dev, cloud, 20000 // 4, m, k, 12345, label="k32-sectors")


@pytest.mark.parametrize("q", [1, 2, 4, 8])
def test_npdu_wide_windows(B, torch_dev, q):
    """Windows wider than two blocks (re-reduced two blocks at a time): an
    even and an odd number of window blocks, windows reaching the padding
    block past the last point and the last register, windows covering the
    whole sector, both edge readings, exact ties."""
    torch, dev = torch_dev
    rng = np.random.default_rng(900 + q)
    for n in (4096 * q, 4096 * q - 37):
        pts = synth.object_cloud(n, seed=n)
        ties = rng.integers(0, 3, (n, 3)).astype(np.float32)
        for p, k, flags, start in [(pts, 65, 0, n - 1), (pts, 128, 0, 0), (pts, 191, 2, n // 2),
                                   (pts, 256, 0, n - 1), (pts, 700, 1, 3), (pts, 1000, 3, n - 5),
                                   (ties, 200, 0, n // 3), (pts, 2 * n, 0, 7)]:
            _check(B, torch, dev, p, min(n, 1200), 1, k, start, variant=(1, q), label="wide-q%d" % q,
                   flags=flags)


@pytest.mark.parametrize("q", [4, 8])
def test_npdu_large_sectors(B, torch_dev, q):
    """Sectors whose coordinates stay in L2 (more than 8192 points), narrow
    windows: the first sweep through untouched points and the jumps after it,
    windows at both ends, exact ties, every point sampled, both edge readings
    and the full first update, one and two sectors."""
    torch, dev = torch_dev
    rng = np.random.default_rng(1300 + q)
    for n in (4096 * q, 4096 * q - 37, 4096 * q // 2 + 1):
        pts = synth.lidar_scan(-(-n // 64), seed=n, n=n)
        ties = rng.integers(0, 3, (n, 3)).astype(np.float32)
        for p, c, k, flags, start in [(pts, 2000, 64, 0, 0), (pts, 2000, 32, 0, n - 1), (pts, 1500, 63, 2, n // 2),
                                      (pts, 1200, 1, 0, 5), (pts, 1200, 0, 0, n - 3), (pts, 900, 2, 1, 0),
                                      (pts, 900, 64, 3, n - 1), (ties, 1500, 64, 0, n // 3), (ties, 700, 17, 2, 0)]:
            _check(B, torch, dev, p, c, 1, k, start, variant=(1, q), label="large-q%d" % q, flags=flags)
    n = 4096 * q // 2 + 77
    pts = synth.object_cloud(n, seed=q)
    _check(B, torch, dev, pts, n, 1, 64, 0, variant=(1, q), label="large-every-point")
    big = synth.lidar_scan(-(-(2 * n) // 64), seed=5, n=2 * n)
    for k in (8, 33, 64):
        _check(B, torch, dev, big, 2 * n // 8, 2, k, int(rng.integers(0, 2 * n)), label="large-m2")


READING_FLAGS = (1, 2, 3, 4, 5, 6, 7)   # full first update, shifted windows, k counting the sample


def test_npdu_readings_random(B, torch_dev):
    """The alternative NPDU readings on random clouds: both window paths
    (k <= 64 and wider), ragged sectors, every flag combination."""
    torch, dev = torch_dev
    rng = np.random.default_rng(606)
    for it in range(70):
        n = int(rng.integers(1, 6000))
        pts = synth.object_cloud(n, int(rng.integers(0, 1 << 30))) if it % 2 else rng.random((n, 3), dtype=np.float32)
        c = int(rng.integers(1, min(n, 600) + 1))
        m = int(rng.integers(1, min(c, 24) + 1))
        k = [1, 2, 7, 32, 63, 64, 65, 129, 3 * n][int(rng.integers(0, 9))]
        flags = READING_FLAGS[it % len(READING_FLAGS)]
        start = int(rng.integers(0, n))
        _check(B, torch, dev, pts, c, m, k, start, label="readings-%d" % it, flags=flags)


@pytest.mark.parametrize("q", [1, 2, 4, 8])
def test_npdu_readings_every_variant(B, torch_dev, q):
    torch, dev = torch_dev
    n = 4096 * q - 101
    pts = synth.object_cloud(n, seed=40 + q)
    for k, flags, start in [(8, 1, 0), (64, 2, n - 1), (33, 3, 17), (200, 7, n // 2), (64, 4, 5)]:
        _check(B, torch, dev, pts, min(n // 4, 1500), 1, k, start, variant=(1, q), label="readings-q%d" % q,
               flags=flags)


def test_npdu_readings_edges(B, torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(607)
    full = synth.object_cloud(4096, seed=12)
    for c, k, flags, start in [(1, 5, 1, 9), (2, 5, 1, 9), (4096, 64, 2, 4095), (3000, 63, 3, 4000),
                               (2000, 64, 6, 0), (4096, 2, 7, 2048)]:
        _check(B, torch, dev, full, c, 1, k, start, variant=(1, 1), label="readings-4096", flags=flags)
    one = rng.random((1, 3), dtype=np.float32)
    for flags in READING_FLAGS:
        _check(B, torch, dev, one, 1, 1, 3, 0, label="readings-one", flags=flags)
    pts = rng.random((300, 3), dtype=np.float32)
    for flags in READING_FLAGS:
        _check(B, torch, dev, pts, 300, 7, 1000, 250, label="readings-wide", flags=flags)


def test_npdu_readings_batched(B, torch_dev):
    torch, dev = torch_dev
    clouds = synth.batch_of_objects(40, seed=21, n_min=1024, n_max=32768)
    cs = [len(p) // 4 for p in clouds]
    _batch_case(B, torch, dev, clouds, cs, [8] * len(clouds), [32 if i % 3 else 64 for i in range(len(clouds))],
                [i % 5 for i in range(len(clouds))], graph_replays=2,
                flags=[((0,) + READING_FLAGS)[i % 8] for i in range(len(clouds))])


def test_cube_2048_plain_fps(B, torch_dev):
    torch, dev = torch_dev
    pts = synth.uniform_cube(2048, 0)
    _check(B, torch, dev, pts, 512, 1, None, 0, label="cube-fps")
    _check(B, torch, dev, pts, 512, 1, None, 0, variant=(4, 8), label="cube-afps-m1")


def test_object_8192_sweep(B, torch_dev):
    torch, dev = torch_dev
    pts = synth.object_cloud(8192, 0)
    for m in (1, 2, 4, 8, 16, 32):
        for k in (None, 8, 32, 128):
            _check(B, torch, dev, pts, 2048, m, k, 0, label="object-8192")


def test_lidar_32768(B, torch_dev):
    torch, dev = torch_dev
    pts = synth.lidar_scan(512, 0)
    _check(B, torch, dev, pts, 8192, 16, 64, 0, label="lidar-npdu")
    _check(B, torch, dev, pts, 8192, 16, None, 0, label="lidar-afps")
    _check(B, torch, dev, pts, 8192, 1, None, 0, label="lidar-fps")


@pytest.mark.parametrize("n,c", [(40000, 600), (131072, 1024), (70001, 3000)])
def test_grid_fps_large_clouds(B, torch_dev, n, c):
    torch, dev = torch_dev
    pts = synth.lidar_scan(-(-n // 64), seed=n, n=n)
    _check(B, torch, dev, pts, c, 1, None, n // 7, label="grid-fps")


def _batch_case(B, torch, dev, clouds, cs, ms, ks, starts, graph_replays=0, flags=None):
    sizes = [len(p) for p in clouds]
    print("batch clouds=%d points=%d ks=%s graph=%d flags=%s" % (len(clouds), sum(sizes), sorted(set(map(str, ks))),
                                                               graph_replays, flags is not None), flush=True)
    plan = B.BatchPlan(sizes, cs, ms, ks, starts, device=dev, flags=flags)
    xyz_all = torch.from_numpy(np.concatenate(clouds).astype(np.float32)).to(dev)
    out = plan.launch(xyz_all)
    torch.cuda.synchronize()
    eager = out.cpu().numpy().copy()
    for i, p in enumerate(clouds):
        o = plan.descs[i].out_offset
        want = oracle.afps(p, cs[i], ms[i], ks[i], starts[i], flags=0 if flags is None else flags[i])
        assert np.array_equal(eager[o:o + cs[i]], want), "cloud %d" % i
    for r in range(graph_replays):
        out.fill_(-7)
        plan.launch(xyz_all, out_all=out, graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), "graph replay %d" % r
        torch.zeros(1000, device=dev).sum().item()   # eager work between replays
    plan.close()
    return plan


def test_batched_uneven_npdu_and_graph(B, torch_dev):
    torch, dev = torch_dev
    clouds = synth.batch_of_objects(48, seed=3, n_min=1024, n_max=32768)
    cs = [len(p) // 4 for p in clouds]
    _batch_case(B, torch, dev, clouds, cs, [8] * len(clouds), [32] * len(clouds), [0] * len(clouds),
                graph_replays=3)


def test_batched_large_sectors_in_the_pool(B, torch_dev):
    """NPDU sectors of every block-register count in one pooled launch: up to
    4096 points (coordinates in LDS), up to 8192, and sectors whose
    coordinates stay in L2 (up to 16 384 and 32 768 points), ragged sizes,
    windows inside two blocks and wider, starts at both ends, the alternative
    readings, graph replays."""
    torch, dev = torch_dev
    sizes = [32768, 20001, 16384, 12345, 9000, 8192, 5000, 3001, 32700, 16383]
    ms = [1, 1, 1, 1, 2, 1, 1, 1, 2, 3]
    ks = [64, 17, 200, 64, 33, 130, 64, 80, 8, 64]
    cs = [900, 700, 500, 800, 600, 400, 700, 300, 1000, 600]
    starts = [0, 20000, 5, 12344, 8999, 0, 4000, 3000, 16000, 1]
    flags = [0, 0, 0, 2, 0, 1, 3, 0, 0, 2]
    clouds = [synth.lidar_scan(-(-n // 64), seed=i, n=n) if i % 2 == 0 else synth.object_cloud(n, seed=i)
              for i, n in enumerate(sizes)]
    _batch_case(B, torch, dev, clouds, cs, ms, ks, starts, graph_replays=2, flags=flags)


def test_plan_first_launched_on_a_side_stream(B, torch_dev):
    """Two plans of the same clouds, the first replayed on the current stream
    (plain FPS, several milliseconds), the second first launched from a graph
    on a side stream that does not wait for the current one: its workspace
    upload is ordered on the side stream, so both results are exact."""
    torch, dev = torch_dev
    clouds = [synth.object_cloud(n, seed=n) for n in (32768, 3000, 1024)]
    sizes, cs = [len(p) for p in clouds], [4096, 750, 256]
    xyz = torch.from_numpy(np.concatenate(clouds)).to(dev)
    print("side-stream plans sizes=%s" % sizes, flush=True)
    busy = B.BatchPlan(sizes, cs, [1] * 3, [None] * 3, [0] * 3, device=dev)
    late = B.BatchPlan(sizes, cs, [1] * 3, [None] * 3, [0] * 3, device=dev)
    side = torch.cuda.Stream(device=dev)
    out_busy = busy.launch(xyz, graph=True)
    out_late = torch.empty(late.total_samples, dtype=torch.int32, device=dev)
    late.launch(xyz, out_all=out_late, stream=side, graph=True)
    torch.cuda.synchronize()
    for out in (out_busy, out_late):
        got = out.cpu().numpy()
        for i, p in enumerate(clouds):
            assert np.array_equal(got[busy.offsets[i]:busy.offsets[i] + cs[i]], oracle.afps(p, cs[i], 1, None, 0)), i
    busy.close()
    late.close()


@pytest.mark.parametrize("occupancy", [0.0, 1.0, 2.0, 4.0])
def test_batch_of_256_every_cloud(B, torch_dev, occupancy):
    """The timed batch at its full size (256 object clouds, N log-uniform in
    [1024, 32768], C = N/4, AFPS M = 8, NPDU k = 32, the same seed), every
    cloud against the oracle, under each plan occupancy the tuner can pick."""
    torch, dev = torch_dev
    clouds = synth.batch_of_objects(256, seed=0)
    cs = [len(p) // 4 for p in clouds]
    B.set_plan_occupancy(occupancy)
    try:
        plan = _batch_case(B, torch, dev, clouds, cs, [8] * 256, [32] * 256, [0] * 256, graph_replays=2)
    finally:
        B.set_plan_occupancy(0.0)
    # one wave per SIMD: one workgroup of four per CU; two per SIMD: every
    # sector of this batch fits half a CU's pages, so two workgroups of four
    if occupancy == 1.0:
        assert (plan.pool_waves, plan.pool_groups) == (4, 1)
    elif occupancy >= 2.0:
        assert (plan.pool_waves, plan.pool_groups) == (4, 2)


@pytest.mark.parametrize("n,groups", [(4928, 2), (4929, 1), (19904, 2), (19905, 1)])
def test_split_pool_at_the_half_boundary(B, torch_dev, n, groups):
    """At two waves per SIMD the plan splits each CU into two workgroups when
    its largest sector fits one of them: a CU's 158 pages less the second
    workgroup's static LDS leave 78 each.  4928 points of 16-byte records take
    78 pages (77 blocks and the padding block), 4929 take 79; 19904 points of
    distance-only records take 78 (312 blocks of 256 bytes), 19905 take 79.
    Either way every index is exact."""
    torch, dev = torch_dev
    clouds = [synth.object_cloud(n, seed=n), synth.object_cloud(3000, seed=1), synth.object_cloud(700, seed=2)]
    sizes, cs = [len(p) for p in clouds], [600, 500, 175]
    B.set_plan_occupancy(4.0)
    try:
        plan = _batch_case(B, torch, dev, clouds, cs, [1, 1, 1], [64, 32, 17], [n - 1, 0, 5], graph_replays=1)
    finally:
        B.set_plan_occupancy(0.0)
    assert (plan.pool_waves, plan.pool_groups) == (4 if groups == 2 else 8, groups)


def test_pipelined_steps_on_two_streams(B, torch_dev):
    """Consecutive steps alternating over two streams, each with its own plan
    (split pool: two workgroups per CU) and output, several replays each in
    flight together: every output equals the oracle."""
    torch, dev = torch_dev
    clouds = synth.batch_of_objects(64, seed=12, n_min=1024, n_max=32768)
    sizes, cs = [len(p) for p in clouds], [len(p) // 4 for p in clouds]
    xyz = torch.from_numpy(np.concatenate(clouds)).to(dev)
    print("pipelined plans clouds=%d points=%d" % (len(clouds), sum(sizes)), flush=True)
    B.set_plan_occupancy(4.0)
    try:
        plans = [B.BatchPlan(sizes, cs, [8] * 64, [32] * 64, [0] * 64, device=dev) for _ in range(2)]
    finally:
        B.set_plan_occupancy(0.0)
    assert all(p.pool_groups == 2 for p in plans)
    streams = [torch.cuda.current_stream(), torch.cuda.Stream(device=dev)]
    outs = [torch.full((plans[0].total_samples,), -7, dtype=torch.int32, device=dev) for _ in range(2)]
    for i in range(10):
        plans[i % 2].launch(xyz, out_all=outs[i % 2], stream=streams[i % 2], graph=i >= 2)
    torch.cuda.synchronize()
    want = [oracle.afps(p, c, 8, 32, 0) for p, c in zip(clouds, cs)]
    for out in outs:
        got = out.cpu().numpy()
        for i, w in enumerate(want):
            assert np.array_equal(got[plans[0].offsets[i]:plans[0].offsets[i] + cs[i]], w), i
    for p in plans:
        p.close()


def test_batched_mixed_variants(B, torch_dev):
    """Plain FPS, AFPS and NPDU clouds of uneven size in one plan (several
    persistent launches on helper streams)."""
    torch, dev = torch_dev
    rng = np.random.default_rng(11)
    clouds, cs, ms, ks, starts = [], [], [], [], []
    for i in range(24):
        n = int(rng.integers(200, 20000))
        clouds.append(synth.object_cloud(n, seed=int(rng.integers(0, 1 << 30))))
        kind = i % 3
        cs.append(max(1, n // 8))
        ms.append(1 if kind == 0 else int(rng.integers(1, 9)))
        ks.append(None if kind < 2 else int(rng.integers(0, 80)))
        starts.append(int(rng.integers(0, n)))
    _batch_case(B, torch, dev, clouds, cs, ms, ks, starts, graph_replays=2)


def test_batched_plain_fps_up_to_32768(B, torch_dev):
    torch, dev = torch_dev
    clouds = [synth.object_cloud(n, seed=n) for n in (32768, 30000, 24577, 1024, 5000)]
    _batch_case(B, torch, dev, clouds, [256] * 5, [1] * 5, [None] * 5, [0, 1, 2, 3, 4])


def test_grid_barrier_timeout_is_bounded(B, torch_dev):
    """A tiny spin limit forces the grid barrier's bounded wait to give up: the
    kernel must still exit and leave -1 in the outputs it did not finish."""
    torch, dev = torch_dev
    pts = synth.lidar_scan(800, seed=1, n=50000)
    xyz = torch.from_numpy(pts).to(dev)
    B.clear_device_status()
    B.set_spin_limit(1)
    try:
        out = B.fps(xyz, 400, 0)
        torch.cuda.synchronize()
    finally:
        B.set_spin_limit(1 << 22)
    got = out.cpu().numpy()
    want = oracle.fps(pts, 400, 0)
    # a finished prefix equal to the oracle's, then -1 from the failed iteration on
    bad = np.flatnonzero(got == -1)
    f = int(bad[0]) if bad.size else len(got)
    assert np.array_equal(got[:f], want[:f])
    assert np.all(got[f:] == -1)
    # the give-up is reported (AFPS_ERR_DEVICE) until cleared; then a normal run is exact and clean
    if bad.size:
        with pytest.raises(B.AfpsError) as e:
            B.device_status()
        assert e.value.status == -7
    B.clear_device_status()
    out = B.fps(xyz, 400, 0)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    B.device_status()


def test_pool_wait_timeout_fails_whole_sectors_and_resets(B, torch_dev):
    """A spin limit of 1 makes waves of the pooled NPDU kernel give up on the
    allocation lock or on pages: every sector must then be either exact or
    entirely -1 (no sector half written), and the next launch of the same plan
    (counters left reset by the failed one) must be exact again."""
    torch, dev = torch_dev
    clouds = synth.batch_of_objects(64, seed=9, n_min=2048, n_max=32768)
    cs = [len(p) // 4 for p in clouds]
    m = [8] * len(clouds)
    plan = B.BatchPlan([len(p) for p in clouds], cs, m, [32] * len(clouds), [0] * len(clouds), device=dev)
    xyz = torch.from_numpy(np.concatenate(clouds)).to(dev)
    want = [oracle.afps(p, c, 8, 32, 0) for p, c in zip(clouds, cs)]
    failed_sectors = 0
    B.clear_device_status()
    try:
        B.set_spin_limit(1)
        out = plan.launch(xyz)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        failed_sectors = int((got == -1).sum())
        for i, (c, w) in enumerate(zip(cs, want)):
            g = got[plan.offsets[i]:plan.offsets[i] + c]
            qn, rn, qc, rc = len(clouds[i]) // 8, len(clouds[i]) % 8, c // 8, c % 8
            for s in range(8):
                o, cc = s * qc + min(s, rc), qc + (s < rc)
                sector = g[o:o + cc]
                assert np.array_equal(sector, w[o:o + cc]) or np.all(sector == -1), (i, s)
    finally:
        B.set_spin_limit(1 << 22)
    # a launch with -1 sectors reports AFPS_ERR_DEVICE, through the plan and the device
    if failed_sectors:
        for check in (plan.status, B.device_status):
            with pytest.raises(B.AfpsError) as e:
                check()
            assert e.value.status == -7
    B.clear_device_status()
    for graph in (False, True):
        out = plan.launch(xyz, graph=graph)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for i, (c, w) in enumerate(zip(cs, want)):
            assert np.array_equal(got[plan.offsets[i]:plan.offsets[i] + c], w), (graph, i)
        plan.status()                 # each launch clears the plan's word
    B.device_status()
    plan.close()


def test_autotuner_choices_stay_exact(B, torch_dev):
    """The autotuner installs its fastest variants; sampling with them still
    gives the oracle's indices (direct launches and batch plans)."""
    torch, dev = torch_dev
    from paper_2208_08795_amd import autotune
    try:
        table = autotune.tune(classes=(256, 3000), reps=1, batch_points=1 << 18, max_iters=64)
        print("autotune", table, flush=True)
        assert len(table["direct"]) == 2 and len(table["batch"]) == 2
        for n in (256, 3000):
            pts = synth.object_cloud(n, seed=n)
            _check(B, torch, dev, pts, n // 4, 1, None, 3, label="tuned-direct")
        clouds = [synth.object_cloud(n, seed=n + 1) for n in (200, 256, 2900, 3000)]
        _batch_case(B, torch, dev, clouds, [50, 64, 700, 750], [1] * 4, [None] * 4, [0, 1, 2, 3])
    finally:
        B.tune_reset()


@pytest.mark.parametrize("shape", [(8, 1), (16, 1)])
@pytest.mark.parametrize("placement", ["all_out", "out_up_to_2048", "out_above_2048", "all_lds"])
def test_pooled_sectors_with_tuned_coordinate_placement(B, torch_dev, placement, shape):
    """NPDU sectors whose coordinates the tuning table keeps out of LDS (only
    the distances in LDS; the coordinates in registers up to 4096 points with
    k <= 64 in launches of at most 8 waves per workgroup, else read from L2)
    in one pooled launch with sectors that keep them in LDS: sizes on both
    sides of every threshold, every reading, windows inside two blocks and
    wider, a 16-wave shape (no register sets: L2 instead); every index
    against the oracle, graph replays."""
    torch, dev = torch_dev
    B.tune_reset()
    try:
        B.set_pool_policy(shape[0], shape[1], True, 3)
        if placement == "all_out":
            B.tune_npdu(8192, 1 << 30, False)
        elif placement == "out_up_to_2048":
            B.tune_npdu(2048, 1 << 30, False)
            B.tune_npdu(8192, 1 << 30, True)
        elif placement == "out_above_2048":
            B.tune_npdu(2048, 1 << 30, True)
            B.tune_npdu(8192, 1 << 30, False)
        else:
            B.tune_npdu(8192, 1 << 30, True)
        assert B.npdu_xyz_in_lds(1000, 32) == (placement in ("out_above_2048", "all_lds"))
        assert B.npdu_xyz_in_lds(5000, 32) == (placement in ("out_up_to_2048", "all_lds"))
        sizes = [4096, 4097, 2048, 2049, 8192, 777, 65, 1, 3000, 6000, 12000, 1500]
        ms = [1, 1, 1, 1, 1, 1, 1, 1, 2, 3, 2, 1]
        ks = [32, 64, 8, 100, 32, 0, 65, 0, 200, 17, 33, 64]
        cs = [max(m, n // 5) for n, m in zip(sizes, ms)]
        starts = [0, 4096, 7, 2048, 8191, 3, 64, 0, 2999, 5, 11999, 700]
        flags = [0, 1, 2, 3, 0, 2, 0, 0, 1, 0, 2, 3]
        clouds = [synth.object_cloud(n, seed=i) if i % 2 and n >= 64 else synth.uniform_cube(n, seed=i)
                  for i, n in enumerate(sizes)]
        _batch_case(B, torch, dev, clouds, cs, ms, ks, starts, graph_replays=2, flags=flags)
    finally:
        B.tune_reset()


@pytest.mark.parametrize("shape", [(16, 1), (12, 2)])
def test_l2_window_update_edges(B, torch_dev, shape):
    """The narrow loop with coordinates from L2 (D alone in LDS): windows of
    at most 64 points update the 64 points from the window's first on and
    read the two blocks holding it back from LDS, k = 64 updates the two
    blocks in place.  Ragged sectors around 64-point blocks up to 4096
    points, so that windows start at every offset of a block and run into
    the sector's ends, k from 1 to 64, every reading, the 16-wave kernel and
    the light one, graph replays: every index against the oracle."""
    torch, dev = torch_dev
    rng = np.random.default_rng(77)
    sizes = [1, 2, 63, 64, 65, 127, 129, 191, 700, 1023, 2049, 4031, 4095, 4096, 3000, 257]
    ks = [1, 2, 31, 32, 33, 62, 63, 64, 7, 16, 40, 63, 64, 32, 1, 64]
    flags = [i % 8 for i in range(len(sizes))]
    cs = [max(1, n // 3) for n in sizes]
    starts = [int(rng.integers(0, n)) for n in sizes]
    clouds = [synth.object_cloud(n, seed=100 + i) if n >= 64 else synth.uniform_cube(n, seed=100 + i)
              for i, n in enumerate(sizes)]
    B.tune_reset()
    try:
        B.set_pool_policy(shape[0], shape[1], False, 0)
        B.tune_npdu(4096, 64, False)   # sectors of at most 4096 points with k <= 64: coordinates from L2
        plan = _batch_case(B, torch, dev, clouds, cs, [1] * len(sizes), ks, starts, graph_replays=2, flags=flags)
        assert (plan.pool_waves, plan.pool_groups) == shape
    finally:
        B.tune_reset()


@pytest.mark.parametrize("shape", [(4, 1), (8, 1), (4, 2), (12, 1), (16, 1), (12, 2), (16, 2)])
@pytest.mark.parametrize("seeding", [(False, 0), (True, 3)])
def test_pool_policies_stay_exact(B, torch_dev, shape, seeding):
    """Every pooled launch shape and seeding policy the tuner can pick, on
    uneven clouds of the batch workload (sectors of at most 4096 points, k =
    32: the two-workgroup 12- and 16-wave shapes run the light kernels), and
    the light shapes once more with every reading on ragged clouds: indices
    equal the oracle's."""
    torch, dev = torch_dev
    clouds = synth.batch_of_objects(40, seed=21, n_min=1024, n_max=32768)
    cs = [len(p) // 4 for p in clouds]
    B.set_pool_policy(shape[0], shape[1], seeding[0], seeding[1])
    if shape[1] == 2 and shape[0] >= 12:   # the light kernels serve sectors with coordinates out of LDS
        B.tune_npdu(4096, 64, False)
    try:
        plan = _batch_case(B, torch, dev, clouds, cs, [8] * 40, [32] * 40, [0] * 40, graph_replays=1)
        assert (plan.pool_waves, plan.pool_groups) == shape
        if shape[1] == 2 and shape[0] >= 12:
            sizes = [4096, 4095, 2049, 777, 65, 1, 300, 3000]
            ks = [64, 32, 63, 0, 64, 0, 7, 33]
            flags = [0, 1, 2, 3, 0, 2, 1, 0]
            cl = [synth.object_cloud(n, seed=i) if n >= 64 else synth.uniform_cube(n, seed=i)
                  for i, n in enumerate(sizes)]
            plan = _batch_case(B, torch, dev, cl, [max(1, n // 3) for n in sizes], [1] * 8, ks,
                               [n // 2 for n in sizes], graph_replays=1, flags=flags)
            assert (plan.pool_waves, plan.pool_groups) == shape
    finally:
        B.tune_reset()


@pytest.mark.parametrize("policy", ["builtin", "l2_16", "lite_12x2", "regs_8", "l2_12"])
def test_pooled_random_batches_every_policy(B, torch_dev, policy):
    """Random batches (seeded) under every pooled policy the tuner can
    install: cloud sizes log-uniform in [1, 32768], 1 to 16 sectors, k from 0
    to 200 or plain AFPS, every reading, random starts and sample counts; one
    eager launch against the oracle, and (NPDU-only plans) a launch of three
    rounds equal to it."""
    torch, dev = torch_dev
    rng = np.random.default_rng(1234 + ["builtin", "l2_16", "lite_12x2", "regs_8", "l2_12"].index(policy))
    lite = policy == "lite_12x2"
    B.tune_reset()
    try:
        if policy == "l2_16":
            B.set_pool_policy(16, 1, False, 0)
            B.tune_npdu(4096, 64, False)
        elif policy == "l2_12":
            B.set_pool_policy(12, 1, True, 3)
            B.tune_npdu(8192, 1 << 30, False)
        elif policy == "lite_12x2":
            B.set_pool_policy(12, 2, False, 0)
            B.tune_npdu(4096, 64, False)
        elif policy == "regs_8":
            B.set_pool_policy(8, 1, True, 3)
            B.tune_npdu(4096, 64, False)
        for trial in range(3):
            sizes, ms, ks, cs, starts, flags = [], [], [], [], [], []
            for _ in range(int(rng.integers(5, 30))):
                n = int(np.exp(rng.uniform(0, np.log(32768))))
                m = int(rng.integers(1, min(16, n) + 1))
                if lite:
                    m = max(m, (n + 4095) // 4096)
                    k = int(rng.choice([0, 1, 7, 31, 32, 33, 63, 64]))
                else:
                    k = [None, 0, 1, 7, 31, 32, 33, 63, 64, 65, 100, 200][int(rng.integers(0, 12))]
                    if k is None and n > 8192:
                        k = 32
                c = int(rng.integers(m, min(n, 4096 if k is None else n) + 1))
                fl = int(rng.integers(0, 8)) if k is not None else 0
                if k == 0:
                    fl &= 3   # k counting the sample needs k >= 1
                sizes.append(n)
                ms.append(m)
                ks.append(k)
                cs.append(c)
                starts.append(int(rng.integers(0, n)))
                flags.append(fl)
            clouds = [synth.object_cloud(n, seed=100 * trial + i) if n >= 64 else synth.uniform_cube(n, seed=100 * trial + i)
                      for i, n in enumerate(sizes)]
            print("policy %s trial %d: %d clouds, %d points" % (policy, trial, len(sizes), sum(sizes)), flush=True)
            plan = B.BatchPlan(sizes, cs, ms, ks, starts, device=dev, flags=flags)
            xyz = torch.from_numpy(np.concatenate(clouds).astype(np.float32)).to(dev)
            out = plan.launch(xyz)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            for i, p in enumerate(clouds):
                o = plan.descs[i].out_offset
                want = oracle.afps(p, cs[i], ms[i], ks[i], starts[i], flags=flags[i])
                assert np.array_equal(got[o:o + cs[i]], want), "trial %d cloud %d" % (trial, i)
            if all(k is not None for k in ks):
                outs = [torch.full_like(out, -7) for _ in range(3)]
                plan.launch_rounds([(xyz, o) for o in outs])
                torch.cuda.synchronize()
                plan.status()
                assert all(torch.equal(o, out) for o in outs)
            plan.close()
    finally:
        B.tune_reset()


def test_npdu_tuner_choices_stay_exact(B, torch_dev):
    """The NPDU tuner times every pooled launch shape, coordinate placement
    and seeding policy on a batch (one launch of several rounds each), checks
    that each gives the same indices, and installs the fastest: a plan built
    afterwards is exact against the oracle."""
    torch, dev = torch_dev
    from paper_2208_08795_amd import autotune
    clouds = synth.batch_of_objects(32, seed=33, n_min=1024, n_max=32768)
    sizes, cs = [len(p) for p in clouds], [len(p) // 4 for p in clouds]
    xyz = torch.from_numpy(np.concatenate(clouds)).to(dev)
    try:
        res = autotune.tune_npdu(xyz, sizes, cs, [8] * 32, [32] * 32, [0] * 32, rounds=3, reps=1)
        print("npdu tuner best", res["best"], "of", len(res["rows"]), flush=True)
        assert len(res["rows"]) >= 3 * len(autotune.REGS_UP_TO)
        plan = _batch_case(B, torch, dev, clouds, cs, [8] * 32, [32] * 32, [0] * 32, graph_replays=1)
        assert (plan.pool_waves, plan.pool_groups) == res["best"][0]
    finally:
        B.tune_reset()
