"""Autotuner for the full-update (FPS / AFPS) sector kernels.

For every sector-size class it times each compiled (waves per workgroup,
point slots per thread) variant that holds the class, on a synthetic object
cloud, in two regimes, and installs the fastest through the library's tuning
table:

* ``direct`` (latency): one sector alone on the GPU, the single-cloud calls;
  time per iteration is set by the per-iteration reduction chain, so fewer
  waves can win even though they do more work per thread;
* ``batch`` (throughput): many sectors of the class in one launch, as inside
  a batch plan; here the variant that keeps the SIMDs busiest wins.

For the pooled NPDU launch of batch plans (one wave per sector, sectors
placed into each CU's LDS pages), ``tune_npdu`` times the caller's own batch
as it runs (one launch of several rounds) under each launch shape (waves per
workgroup and workgroups per CU: the sector-to-CU mapping), each placement of
the sectors' coordinates (registers up to some sector size, which leaves a
quarter of the pages per sector, LDS records above) and each seeding policy,
and installs the fastest.  Results can be written to a cache file that the library reads at
first use (AFPS_TUNE_CACHE).
"""
from __future__ import annotations

import time

import numpy as np

WAVES = (1, 2, 4, 8, 16)
SLOTS = (1, 2, 4, 8, 12, 16, 24, 32)
CLASSES = (64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 24576, 32768)


def candidates(n: int, oversize: int = 4):
    """Variants holding n points without more than `oversize` times the slots needed."""
    out = []
    for w in WAVES:
        for p in SLOTS:
            cap = 64 * w * p
            if cap >= n and cap < oversize * n + 64 * w:
                out.append((w, p))
    return out


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def tune(classes=CLASSES, reps: int = 3, batch_points: int = 1 << 22, max_iters: int = 512,
         install: bool = True, cache_path: str | None = None, seed: int = 0, log=None):
    """Time the candidates of every class; return {"direct": [...], "batch": [...]}
    rows of (n_max, waves, slots, ms) and install them in the library."""
    import torch

    from . import binding, synth
    t0 = time.perf_counter()
    table = {"direct": [], "batch": []}
    for n in classes:
        c = max(1, min(n // 4, max_iters))
        single = torch.from_numpy(synth.object_cloud(n, seed)).cuda()
        sectors = int(np.clip(batch_points // n, 256, 4096))
        many = torch.from_numpy(np.tile(synth.object_cloud(n, seed + 1), (sectors, 1))).cuda()
        out1 = torch.empty(c, dtype=torch.int32, device="cuda")
        outm = torch.empty(c * sectors, dtype=torch.int32, device="cuda")
        best = {"direct": None, "batch": None}
        for w, p in candidates(n):
            try:
                d = _time(lambda: binding.afps(single, c, 1, 0, out=out1, variant=(w, p)), reps)
                b = _time(lambda: binding.afps(many, c * sectors, sectors, 0, out=outm, variant=(w, p)),
                          reps)
            except binding.AfpsError:
                continue
            for kind, ms in (("direct", d), ("batch", b)):
                if best[kind] is None or ms < best[kind][3]:
                    best[kind] = (n, w, p, ms)
        for kind in ("direct", "batch"):
            if best[kind] is not None:
                table[kind].append(best[kind])
                if install:
                    binding.tune_set(n, best[kind][1], best[kind][2],
                                     binding.TUNE_DIRECT if kind == "direct" else binding.TUNE_BATCH)
        if log:
            log("tune n=%d: direct %s batch %s" % (n, best["direct"], best["batch"]))
        del single, many
    if cache_path:
        with open(cache_path, "w") as f:
            for kind in ("direct", "batch"):
                for n, w, p, _ in table[kind]:
                    f.write("%s %d %d %d\n" % (kind, n, w, p))
    table["seconds"] = time.perf_counter() - t0
    return table


def tune_occupancy(xyz_all, sizes, cs, ms, ks, starts, factors=(0.0, 1.0, 2.0, 4.0),
                   reps: int = 5, streams: int = 1, install: bool = True, log=None):
    """Sector-to-CU mapping of batch plans: time the batch's persistent launches
    under several wave budgets (waves per SIMD; 0 = no budget, as many
    workgroups as fit) and keep the fastest.  With streams > 1 the batch is
    timed as it will run, consecutive graph launches alternating over that
    many streams with a plan and output each (ms per launch over
    20 * streams launches); otherwise one launch at a time (median of reps).
    Returns [(factor, ms)], best first."""
    import torch

    from . import binding
    dev = xyz_all.device
    res = []
    for f in factors:
        binding.set_plan_occupancy(f)
        plans = [binding.BatchPlan(sizes, cs, ms, ks, starts, device=dev) for _ in range(streams)]
        outs = [torch.empty(plans[0].total_samples, dtype=torch.int32, device=dev) for _ in range(streams)]
        strs = [torch.cuda.current_stream(dev)] + [torch.cuda.Stream(device=dev) for _ in range(streams - 1)]
        for p, o, st in zip(plans, outs, strs):
            p.launch(xyz_all, out_all=o, graph=True, stream=st)
        torch.cuda.synchronize()
        if streams == 1:
            ms_ = _time(lambda: plans[0].launch(xyz_all, out_all=outs[0], graph=True), reps)
        else:
            n = 20 * streams
            t0 = time.perf_counter()
            for i in range(n):
                plans[i % streams].launch(xyz_all, out_all=outs[i % streams], graph=True, stream=strs[i % streams])
            torch.cuda.synchronize()
            ms_ = (time.perf_counter() - t0) * 1e3 / n
        for p in plans:
            p.close()
        res.append((f, ms_))
        if log:
            log("plan occupancy %.1f waves/SIMD: %.4f ms" % (f, ms_))
    res.sort(key=lambda x: x[1])
    binding.set_plan_occupancy(res[0][0] if install else 0.0)
    return res


# Pooled launch shapes (waves per workgroup, workgroups per CU) and coordinate
# placements (sectors of at most n points hold their coordinates out of LDS:
# in registers where the kernel can, else L2; larger ones in LDS records; 0 =
# every sector in LDS) that tune_npdu tries.
POOL_SHAPES = ((8, 1), (4, 1), (4, 2), (12, 1), (16, 1), (12, 2), (16, 2))
REGS_UP_TO = (4096, 2048, 1024, 0)
SEEDING = ((True, 3), (False, 3), (True, 0), (False, 0))


def _apply_npdu(shape, regs_up_to, seeding, k_max):
    from . import binding
    binding.tune_npdu_clear()
    binding.set_pool_policy(shape[0], shape[1], seeding[0], seeding[1])
    if regs_up_to:
        binding.tune_npdu(regs_up_to, k_max, False)
    binding.tune_npdu(8192, k_max, True)


def tune_npdu(xyz_all, sizes, cs, ms, ks, starts, rounds: int = 20, reps: int = 3, install: bool = True,
              cache_path: str | None = None, log=None):
    """Tune the pooled NPDU launch on the caller's batch: time one launch of
    `rounds` rounds (median of reps, HIP events) for every launch shape x
    coordinate placement, then every seeding policy at the best of those; keep
    the fastest (installed in the library, optionally written to cache_path
    as "pool" and "npdu" lines).  Outputs of every configuration are checked
    equal to the first one's.  Returns {"rows": [(shape, regs_up_to, seeding,
    ms per round)], "best": (...), "seconds": s}."""
    import torch

    from . import binding
    t0 = time.perf_counter()
    dev = xyz_all.device
    k_max = max(k for k in ks if k is not None)
    rows, ref = [], None

    def measure(shape, regs, seeding):
        nonlocal ref
        _apply_npdu(shape, regs, seeding, k_max)
        plan = binding.BatchPlan(sizes, cs, ms, ks, starts, device=dev)
        if (plan.pool_waves, plan.pool_groups) != shape:   # the shape does not fit these sectors
            plan.close()
            return None
        outs = [torch.empty(plan.total_samples, dtype=torch.int32, device=dev) for _ in range(2)]
        table = plan.round_table([(xyz_all, outs[r % 2]) for r in range(rounds)])
        plan.launch_rounds(table)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            plan.launch_rounds(table)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b) / rounds)
        if ref is None:
            ref = outs[0].clone()
        if not (torch.equal(outs[0], ref) and torch.equal(outs[1], ref)):
            raise RuntimeError("tuned NPDU configuration %s/%s/%s changed the indices" % (shape, regs, seeding))
        plan.close()
        ms_ = float(np.median(ts))
        rows.append((shape, regs, seeding, ms_))
        if log:
            log("npdu tune: shape %s, registers up to %d points, seeding %s: %.4f ms per batch" % (shape, regs, seeding, ms_))
        return ms_

    for shape in POOL_SHAPES:
        for regs in REGS_UP_TO:
            measure(shape, regs, SEEDING[0])
    best = min(rows, key=lambda r: r[3])
    for seeding in SEEDING[1:]:
        measure(best[0], best[1], seeding)
    best = min(rows, key=lambda r: r[3])
    if install:
        _apply_npdu(best[0], best[1], best[2], k_max)
    else:
        binding.tune_npdu_clear()
    if cache_path:
        with open(cache_path, "a") as f:
            f.write("pool %d %d %d %d\n" % (best[0][0], best[0][1], int(best[2][0]), best[2][1]))
            if best[1]:
                f.write("npdu %d %d 0\n" % (best[1], k_max))
            f.write("npdu 8192 %d 1\n" % k_max)
    return {"rows": rows, "best": best, "seconds": time.perf_counter() - t0}
