"""Benchmark: batched AFPS-NPDU vs plain FPS on one MI355X.

One step = one pass of the whole sampling path over one batch: 256 object-like
clouds of uneven size (N log-uniform in [1024, 32768], C = N/4), AFPS with
M = 8 sectors and NPDU window k = 32, all 2048 sectors in one persistent
launch (queue reset + persistent kernel, replayed from a hipGraph).  Inputs are
resident in HBM before the timed region.  The same 256 clouds are also sampled
with plain FPS (one workgroup per cloud) for comparison.

Prints ONE JSON line (rank 0, N = 1).  Extra fields: plain-FPS figures, per-step
latency percentiles, single-cloud latencies of the paper-sized configurations,
coverage radius against plain FPS, the roofline of the dominant kernel and the
oracle's CPU baseline.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sampled pts/s + p50/p99 frame latency, AFPS-NPDU vs plain FPS, 1 MI355X"
# MI355X peaks used for the roofline.
HBM_PEAK_GBS = 8000.0
# fp32 VALU without FMA and without packed ops (the method's distance is a
# chain of separately rounded sub/mul/add): 256 CU x 4 SIMD x 16 lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def time_steps(torch, plans, xyz_all, outs, steps, warmup, streams):
    """Warm up, then time exactly `steps` graph launches, nothing else between
    the two synchronisations.  Step i runs on stream i mod S with plan and
    output i mod S (each plan has its own workspace), so a step starts on the
    compute units the previous one has already finished with; every stream's
    output is checked against the first afterwards.  Returns (wall seconds,
    warm-up steps done)."""
    S = len(plans)
    done = max(warmup, S)                   # every plan's graph captured before timing
    for i in range(done):
        plans[i % S].launch(xyz_all, out_all=outs[i % S], graph=True, stream=streams[i % S])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        plans[i % S].launch(xyz_all, out_all=outs[i % S], graph=True, stream=streams[i % S])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for o in outs[1:]:
        if not torch.equal(o, outs[0]):
            raise SystemExit("bench: the pipelined streams' outputs differ")
    return wall, done


def step_latency(torch, plan, xyz_all, out, reps, stream):
    """One step's own latency: graph launches one at a time on one stream,
    HIP events around each."""
    plan.launch(xyz_all, out_all=out, graph=True, stream=stream)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.launch(xyz_all, out_all=out, graph=True, stream=stream)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return ms


def time_kernel(torch, plan, xyz_all, out, reps, stream):
    """Duration of the plan's kernels alone: eager launches (queue reset + the
    persistent launch, no graph), HIP events on the launch stream."""
    plan.launch(xyz_all, out_all=out, graph=False, stream=stream)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.launch(xyz_all, out_all=out, graph=False, stream=stream)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return ms


def npdu_work(sizes, cs, out_np, offsets, m, k):
    """Algorithmic work of AFPS-NPDU, counted from the picks: for every
    iteration of every sector, 9 fp32 ops per distance update of the window
    (3 sub, 3 mul, 2 add, 1 min) and one compare per sector point for the
    argmax the method defines.  Returns (ops, distance updates)."""
    ops = upd = 0
    for n, c, o in zip(sizes, cs, offsets):
        qn, rn, qc, rc = n // m, n % m, c // m, c % m
        for s in range(m):
            ns, b = qn + (s < rn), s * qn + min(s, rn)
            cc, oo = qc + (s < rc), s * qc + min(s, rc)
            cur = out_np[o + oo:o + oo + cc - 1].astype(np.int64) - b
            lo = np.maximum(0, cur - k // 2)
            hi = np.minimum(ns - 1, cur + (k - k // 2))
            u = int((hi - lo + 1).sum())
            upd += u
            ops += 9 * u + (cc - 1) * ns
    return ops, upd


def single_cloud_latency(torch, binding, synth, stream, reps=20):
    """Single-frame latencies of the paper-sized configurations (ms, median of reps)."""
    res = {}
    cases = {
        "cube_n2048_c512_fps": (synth.uniform_cube(2048, 0), dict(kind="fps", c=512)),
        "lidar_n32768_c8192_fps": (synth.lidar_scan(512, 0), dict(kind="fps", c=8192)),
        "lidar_n32768_c8192_npdu_m16_k64": (synth.lidar_scan(512, 0), dict(kind="npdu", c=8192, m=16, k=64)),
        "object_n8192_c2048_afps_m32": (synth.object_cloud(8192, 0), dict(kind="afps", c=2048, m=32)),
        "object_n8192_c2048_npdu_m32_k32": (synth.object_cloud(8192, 0), dict(kind="npdu", c=2048, m=32, k=32)),
        "object_n8192_c2048_fps": (synth.object_cloud(8192, 0), dict(kind="fps", c=2048)),
    }
    for name, (pts, p) in cases.items():
        xyz = torch.from_numpy(pts).cuda()
        out = torch.empty(p["c"], dtype=torch.int32, device="cuda")

        def run():
            if p["kind"] == "fps":
                binding.fps(xyz, p["c"], 0, out=out, stream=stream)
            elif p["kind"] == "afps":
                binding.afps(xyz, p["c"], p["m"], 0, out=out, stream=stream)
            else:
                binding.afps_npdu(xyz, p["c"], p["m"], p["k"], 0, out=out, stream=stream)
        for _ in range(2):
            run()
        torch.cuda.synchronize()
        ts = []
        r = reps if not name.endswith("n32768_c8192_fps") else 3
        for _ in range(r):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            run()
            b.record(stream)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        res[name] = round(float(np.median(ts)), 4)
        log("single %s: %.4f ms" % (name, res[name]))
    return res


CLOCK_GHZ = 2.4   # MI355X peak engine clock (SQ counters measured 2.41 GHz under these kernels)


def _median_ms(torch, run, stream, reps):
    run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def object_sweep(torch, binding, synth, stream, reps=10):
    """Object cloud N=8192, C=2048: plain FPS, AFPS for M in {1..32}, NPDU at
    k in {8, 32, 128}: time per call (median), cycles per iteration of the
    longest sector, coverage radius relative to plain FPS.  Then the
    alternative NPDU readings at k in {8, 32}, M in {1, 8}."""
    from paper_2208_08795_amd.quality import coverage_radius
    pts = synth.object_cloud(8192, 0)
    xyz = torch.from_numpy(pts).cuda()
    out = torch.empty(2048, dtype=torch.int32, device="cuda")
    rows = []
    ref = None
    for m in (1, 2, 4, 8, 16, 32):
        for k in (None, 8, 32, 128):
            def run():
                if k is None:
                    binding.afps(xyz, 2048, m, 0, out=out, stream=stream)
                else:
                    binding.afps_npdu(xyz, 2048, m, k, 0, out=out, stream=stream)
            ms = _median_ms(torch, run, stream, reps)
            r = coverage_radius(pts, out.cpu().numpy())
            if m == 1 and k is None:
                ref = r
            iters = -(-2048 // m) - 1
            rows.append({"m": m, "k": k, "ms": round(ms, 4), "sampled_pts_per_s": 2048 / (ms / 1e3),
                         "cycles_per_iteration": round(ms * 1e-3 * CLOCK_GHZ * 1e9 / iters, 1),
                         "coverage_radius": round(r, 5), "coverage_vs_fps": round(r / ref, 4)})
    log("object sweep: " + ", ".join("M%d/k%s %.3fms r%.2f" % (x["m"], x["k"], x["ms"], x["coverage_vs_fps"])
                                     for x in rows))
    names = {0: "default", binding.NPDU_FIRST_FULL: "first_full", binding.NPDU_SHIFT_EDGES: "shift_edges",
             binding.NPDU_K_WITH_SELF: "k_with_self",
             binding.NPDU_FIRST_FULL | binding.NPDU_SHIFT_EDGES: "first_full+shift_edges"}
    readings = []
    for m in (1, 8):
        for k in (8, 32):
            for flags, name in names.items():
                def run():
                    binding.afps_npdu(xyz, 2048, m, k, 0, out=out, stream=stream, flags=flags)
                ms = _median_ms(torch, run, stream, reps)
                r = coverage_radius(pts, out.cpu().numpy())
                readings.append({"m": m, "k": k, "reading": name, "ms": round(ms, 4),
                                 "coverage_radius": round(r, 5), "coverage_vs_fps": round(r / ref, 4)})
    log("NPDU readings: " + ", ".join("M%d/k%d/%s %.3fms r%.2f" % (x["m"], x["k"], x["reading"], x["ms"],
                                                                   x["coverage_vs_fps"]) for x in readings))
    return rows, readings


def grouping(torch, binding, synth, stream, reps=10):
    """Grouping around the samples (ball query, k = 32): the LiDAR frame of
    32768 points around its 8192 AFPS-NPDU samples (M = 16, k = 64) within
    1 m, and the 8192-point object cloud around its 2048 samples (M = 8,
    k = 32) within 0.1; the exact query and storage windows.  Per window:
    time (ms, median of HIP events), mean neighbours found (at most 32), and
    their total relative to the exact query's (every neighbour a window finds
    lies within the radius; a window can only find fewer)."""
    res = {}
    for name, pts, c, m, k, radius in [("lidar_n32768_c8192", synth.lidar_scan(512, 0), 8192, 16, 64, 1.0),
                                       ("object_n8192_c2048", synth.object_cloud(8192, 0), 2048, 8, 32, 0.1)]:
        xyz = torch.from_numpy(pts).cuda()
        centers = binding.afps_npdu(xyz, c, m, k, 0, stream=stream)
        rows = []
        exact_cnt = None
        for window in (None, 1024, 256, 64):
            idx = torch.empty((c, 32), dtype=torch.int32, device="cuda")
            cnt = torch.empty(c, dtype=torch.int32, device="cuda")
            run = lambda: binding.ball_query(xyz, centers, radius, 32, window, out=idx, counts=cnt, stream=stream)
            run()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                run()
                b.record(stream)
                b.synchronize()
                ts.append(a.elapsed_time(b))
            cn = cnt.cpu().numpy()
            if window is None:
                exact_cnt = cn
            rows.append({"window": window, "ms": round(float(np.median(ts)), 4),
                         "mean_found": round(float(cn.mean()), 2),
                         "found_vs_exact": round(float(cn.sum() / max(1, exact_cnt.sum())), 4)})
        res[name] = {"radius": radius, "k": 32, "centres": "AFPS-NPDU M=%d k=%d, %d samples" % (m, k, c), "rows": rows}
    return res


def sortedness(torch, binding, synth, stream, reps=10):
    """Coverage radius of AFPS relative to plain FPS on the same points stored
    in different orders (the paper's Table II setting, with the coverage radius
    standing in for task accuracy): unsorted, approximately sorted along x
    (bins of 128 points by rank), exactly sorted along x and along z, and
    unsorted then binned on the GPU along x (N/128 value bins).  Plus the
    binning's time at two sizes."""
    from paper_2208_08795_amd.quality import coverage_radius
    rng = np.random.default_rng(7)
    base = synth.object_cloud(8192, 2)
    unsorted = base[rng.permutation(len(base))]
    orders = {"unsorted": unsorted,
              "approx_sorted_x_bin128": synth.approx_sort(unsorted, unsorted[:, 0], 128, 3),
              "sorted_x": synth.approx_sort(unsorted, unsorted[:, 0], 1, 3),
              "sorted_z": synth.approx_sort(unsorted, unsorted[:, 2], 1, 3)}
    xyz_u = torch.from_numpy(unsorted).cuda()
    _, binned = binding.bin_points(xyz_u, 0, len(unsorted) // 128)
    orders["gpu_binned_x_64_bins"] = binned.cpu().numpy()
    out = torch.empty(2048, dtype=torch.int32, device="cuda")
    rows = {}
    for name, pts in orders.items():
        xyz = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
        binding.fps(xyz, 2048, 0, out=out, stream=stream)
        torch.cuda.synchronize()
        ref = coverage_radius(pts, out.cpu().numpy())
        row = {}
        for m in (2, 8, 32):
            binding.afps(xyz, 2048, m, 0, out=out, stream=stream)
            torch.cuda.synchronize()
            row["m%d" % m] = round(coverage_radius(pts, out.cpu().numpy()) / ref, 4)
        rows[name] = row
    times = {}
    for n in (8192, 131072, 1048576):
        pts = synth.lidar_scan(max(1, n // 64), 4, n=n)
        xyz = torch.from_numpy(pts[rng.permutation(len(pts))]).cuda()
        bins = min(8192, n // 128)
        times["n%d_bins%d" % (n, bins)] = round(_median_ms(
            torch, lambda: binding.bin_points(xyz, 0, bins, stream=stream), stream, reps), 4)
    log("sortedness (AFPS coverage / FPS): %s; binning ms %s" % (rows, times))
    return {"coverage_vs_fps": rows, "binning_ms": times,
            "what": "object cloud N=8192, C=2048, start 0; AFPS coverage radius / plain FPS coverage radius "
                    "on the same order; binning: shuffled LiDAR frames, points in binned order written"}


def serving(torch, rates=(50, 200, 800), frames_npdu=160, frames_fps=24, pool=48, seed=1):
    """Open-loop Poisson streams of LiDAR frames (N uniform in [16384, 131072],
    C = N/8, M in {8, 16, 32}, k = 64) through the continuous-batching server,
    AFPS-NPDU and plain FPS, per-frame latency from arrival to completion."""
    from paper_2208_08795_amd import synth
    from paper_2208_08795_amd.serve import GpuExecutor, Request, Scheduler, latency_summary
    rng = np.random.default_rng(seed)
    log("generating %d serving frames" % pool)
    frames = synth.frame_stream(rate=1.0, count=pool, seed=seed)
    pinned = [torch.from_numpy(f.points).pin_memory() for f in frames]
    budget = 256 << 20
    ex = GpuExecutor(budget, streams=4)
    res = {"budget_bytes": budget, "frames": "pool of %d distinct synthetic 64-beam frames, N uniform "
                                                "in [16384, 131072], C = N/8, M in {8,16,32}, k = 64" % pool}

    def stream(method, count, lam):
        gaps = rng.exponential(1.0 / lam, count)
        arr = np.cumsum(gaps) - gaps[0]
        reqs = []
        for i in range(count):
            f = frames[i % pool]
            m, k = (f.m, f.k) if method == "afps_npdu" else (1, None)
            reqs.append(Request(i, f.points.shape[0], f.c, m, k, 0, float(arr[i]), pinned[i % pool]))
        s = Scheduler(ex, budget, max_inflight=8, max_batch=32)
        done = s.run(reqs)
        torch.cuda.synchronize()
        out = latency_summary(done)
        out.update({"offered_fps": lam, "peak_waiting": s.peak_waiting, "peak_arena_bytes": s.peak_bytes})
        return out

    for method, count in (("afps_npdu", frames_npdu), ("plain_fps", frames_fps)):
        stream(method, 6, 1000.0)            # warm-up (plans, kernel attributes)
        res[method] = {}
        for lam in rates:
            r = stream(method, count, float(lam))
            res[method][str(lam)] = r
            log("serve %s @%d/s: p50 %.2f ms p99 %.2f ms, %.3e pts/s, peak queue %d" %
                (method, lam, r["p50_ms"], r["p99_ms"], r["sampled_pts_per_s"] or 0, r["peak_waiting"]))
    return res


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` (the NPDU step) from the committed
    FETCH_SIZE / WRITE_SIZE runs, or None when the kernel sources changed
    since or that kernel was not profiled."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pooled_npdu_kernel_batch256_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = "".join(open(os.path.join(ROOT, s)).read() for s in rec["sources"])
    if hashlib.sha256(src.encode()).hexdigest() != rec["source_sha256"]:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return k["traffic_bytes_per_launch"] if k else None


def shader_clock_mhz():
    """The driver's current shader-clock level (sysfs pp_dpm_sclk, the line
    marked '*'), in MHz, for every GPU that exposes it; None where unreadable."""
    import glob
    out = []
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            with open(path) as f:
                for line in f:
                    if "*" in line:
                        out.append(int("".join(ch for ch in line.split(":", 1)[1] if ch.isdigit())))
        except (OSError, ValueError, IndexError):
            continue
    return out or None


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(clouds, cs, m, k, gpu_out, offsets, budget_s=20.0):
    """The oracle (never tuned) on the host cores: one cloud per task."""
    import oracle
    oracle.load()
    cores = min(16, os.cpu_count() or 1)
    # bounded sample: clouds in order until the estimated single-core work
    # (~ N^2 / (8 m) compare steps) reaches the budget
    est, take = 0.0, 0
    for p, c in zip(clouds, cs):
        est += len(p) * c / m * 2e-9
        take += 1
        if est > budget_s * cores * 0.5:
            break
    idx = list(range(take))

    def one(i):
        t = time.perf_counter()
        o = oracle.afps(clouds[i], cs[i], m, k, 0)
        return o, time.perf_counter() - t
    # whole passes over the sample, the median reported, within the time budget
    dts = []
    with cf.ThreadPoolExecutor(cores) as ex:
        while len(dts) < 5 and sum(dts) < budget_s:
            t0 = time.perf_counter()
            res = list(ex.map(one, idx))
            dts.append(time.perf_counter() - t0)
    dt = float(np.median(dts))
    outs = [o for o, _ in res]
    per_cloud_ms = [1e3 * t for _, t in res]   # each cloud runs on one thread: its latency
    same = all(np.array_equal(outs[j], gpu_out[offsets[i]:offsets[i] + cs[i]]) for j, i in enumerate(idx))
    samples = sum(cs[i] for i in idx)
    return {"value": samples / dt, "unit": "sampled pts/s", "cores": cores, "kind": "oracle",
            "sample": "first %d of the 256 clouds (%d points, %d samples), AFPS M=%d NPDU k=%d, one cloud "
                      "per thread; median of %d passes, %.2f s each" %
                      (take, sum(len(clouds[i]) for i in idx), samples, m, k, len(dts), dt),
            "host_cpu": host_cpu_model(),
            "matches_gpu": bool(same),
            "single_thread_ms_per_cloud": {"p50": float(np.percentile(per_cloud_ms, 50)),
                                           "max": float(np.max(per_cloud_ms)),
                                           "mean_points": float(np.mean([len(clouds[i]) for i in idx]))}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--streams", type=int, default=2,
                    help="streams the timed steps alternate over (each with its own plan and output)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-single", action="store_true", help="skip single-cloud latencies")
    ap.add_argument("--no-fps", action="store_true", help="skip the plain-FPS comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving streams")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (built-in variant rule)")
    ap.add_argument("--occupancy", type=float, default=None,
                    help="plan wave budget in waves per SIMD for the timed batch (skips its tuning; "
                         "0 = the built-in rule, >= 1.5 = two pooled waves per SIMD)")
    args = ap.parse_args()
    if args.streams < 1:
        ap.error("--streams must be at least 1")
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent clouds would shard by request with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2208_08795_amd import binding, synth
    from paper_2208_08795_amd.quality import coverage_radius

    binding.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    M, K = 8, 32
    log("generating 256 clouds")
    clouds = synth.batch_of_objects(256, seed=args.seed)
    sizes = [len(p) for p in clouds]
    cs = [n // 4 for n in sizes]
    xyz_all = torch.from_numpy(np.concatenate(clouds)).to(dev)
    total_samples = sum(cs)

    # A plain device copy of known size: rocprofv3 --pmc runs read its
    # FETCH_SIZE / WRITE_SIZE to calibrate the counters.
    calib = torch.empty(64 << 20, dtype=torch.uint8, device=dev)
    calib2 = torch.empty_like(calib)
    calib2.copy_(calib)

    tuned_occ = args.occupancy is None and not args.no_tune
    if args.occupancy is not None:
        binding.set_plan_occupancy(args.occupancy)
    elif tuned_occ:
        from paper_2208_08795_amd import autotune
        log("autotuning the batch plan's wave budget")
        occ = autotune.tune_occupancy(xyz_all, sizes, cs, [M] * 256, [K] * 256, [0] * 256,
                                      streams=args.streams, log=log)
        res_occ = [[f, round(t, 4)] for f, t in occ]
    S = args.streams
    streams = [stream] + [torch.cuda.Stream(device=dev) for _ in range(S - 1)]
    plans = [binding.BatchPlan(sizes, cs, [M] * 256, [K] * 256, [0] * 256, device=dev) for _ in range(S)]
    outs = [torch.empty(plans[0].total_samples, dtype=torch.int32, device=dev) for _ in range(S)]
    plan, out = plans[0], outs[0]
    log("AFPS-NPDU plan: %d items, %d launch(es), %d stream(s)" % (plan.items, plan.launches, S))
    wall, warm = time_steps(torch, plans, xyz_all, outs, args.steps, args.warmup, streams)
    sclk = shader_clock_mhz()
    ms_per_step = wall * 1e3 / args.steps
    value = total_samples / (wall / args.steps)
    out_np = out.cpu().numpy()
    log("AFPS-NPDU: %.3f ms/step, %.3e sampled pts/s" % (ms_per_step, value))
    ev_ms = step_latency(torch, plan, xyz_all, out, max(20, args.steps), stream)

    res = {"metric": METRIC, "value": value, "unit": "sampled pts/s", "n_gpus": 1, "steps": args.steps,
           "warmup": warm, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256 object-like clouds, N log-uniform [1024, 32768] (%d points), "
                                  "C = N/4 (%d samples), AFPS M=8 with NPDU k=32, one persistent launch "
                                  "per step replayed from a hipGraph; consecutive steps alternate over %d "
                                  "streams, each with its own plan workspace and output"
                                  % (sum(sizes), total_samples, S),
                      "clouds": 256, "m": M, "k": K, "points": sum(sizes), "samples": total_samples,
                      "streams": S}}
    if tuned_occ:
        res["plan_occupancy_tuning"] = {"waves_per_simd_vs_ms": res_occ, "chosen": res_occ[0][0],
                                        "what": "ms per step, timed as the steps are (%d stream(s))" % S}
    elif args.occupancy is not None:
        res["plan_occupancy"] = args.occupancy
    res["sclk_mhz_after_timed_steps"] = sclk
    res["batch_latency"] = {"unit": "ms", "what": "one step alone (whole batch of 256 clouds, graph launches "
                                                  "one at a time on one stream), HIP events",
                            "p50": percentile(ev_ms, 50), "p99": percentile(ev_ms, 99)}

    # Roofline of the dominant kernel (the pooled NPDU kernel is the step).
    pool_label = "pooled_npdu_kernel<%d>" % plan.pool_waves
    if plan.pool_groups > 1:
        pool_label += " x%d per CU" % plan.pool_groups
    ops, upd = npdu_work(sizes, cs, out_np, plan.offsets, M, K)
    kern_ms = time_kernel(torch, plan, xyz_all, out, max(10, args.steps), stream)
    kern_s = float(np.mean(kern_ms)) / 1e3
    hbm_bytes = 12 * sum(sizes) + 4 * total_samples + 40 * plan.items
    res["roofline"] = {"bound": "alu", "achieved": ops / kern_s / 1e12, "peak": VALU_PEAK_TOPS,
                       "unit": "TOPS (fp32 VALU ops)", "frac": ops / kern_s / 1e12 / VALU_PEAK_TOPS,
                       "traffic": counter_traffic(pool_label),
                       "kernel": pool_label,
                       "algorithmic_ops_per_launch": ops, "distance_updates_per_launch": upd,
                       "hbm_bytes_per_launch": hbm_bytes,
                       "hbm_frac": hbm_bytes / kern_s / 1e9 / HBM_PEAK_GBS,
                       "avg_launch_ms": kern_s * 1e3,
                       "avg_launch_what": "queue reset + pooled kernel, eager launches, HIP events on the "
                                          "launch stream (the step's graph replay adds its launch overhead)"}

    if not args.no_tune:
        from paper_2208_08795_amd import autotune
        log("autotuning full-update variants")
        tab = autotune.tune(log=log)
        res["autotune"] = {k: [[int(n), int(w), int(p), round(ms, 4)] for n, w, p, ms in v]
                           for k, v in tab.items() if k != "seconds"}
        res["autotune"]["seconds"] = round(tab["seconds"], 2)

    if not args.no_fps:
        binding.set_plan_occupancy(0.0)      # plain FPS: grids as large as fit
        fplans = [binding.BatchPlan(sizes, cs, [1] * 256, [None] * 256, [0] * 256, device=dev) for _ in range(S)]
        fouts = [torch.empty(fplans[0].total_samples, dtype=torch.int32, device=dev) for _ in range(S)]
        fplan, fout = fplans[0], fouts[0]
        fsteps = max(3, args.steps // 4)
        fwall, _ = time_steps(torch, fplans, xyz_all, fouts, fsteps, 1, streams)
        fvalue = total_samples / (fwall / fsteps)
        fout_np = fout.cpu().numpy()
        fev = step_latency(torch, fplan, xyz_all, fout, 3, stream)
        log("plain FPS: %.3f ms/step, %.3e sampled pts/s" % (fwall * 1e3 / fsteps, fvalue))
        res["plain_fps"] = {"value": fvalue, "unit": "sampled pts/s", "ms_per_step": fwall * 1e3 / fsteps,
                            "steps": fsteps, "launches": fplan.launches, "streams": S,
                            "latency_p50_ms": percentile(fev, 50), "latency_p99_ms": percentile(fev, 99),
                            "afps_npdu_speedup": value / fvalue}
        # quality: coverage radius against plain FPS (fp64, 32 clouds)
        ratios = []
        for i in range(0, 256, 8):
            o = plan.offsets[i]
            r_n = coverage_radius(clouds[i], out_np[o:o + cs[i]])
            r_f = coverage_radius(clouds[i], fout_np[o:o + cs[i]])
            ratios.append(r_n / r_f)
        res["coverage_radius_vs_fps"] = {"mean": float(np.mean(ratios)), "max": float(np.max(ratios)),
                                         "clouds": len(ratios)}
        for p in fplans:
            p.close()

    if not args.no_single:
        single = single_cloud_latency(torch, binding, synth, stream)
        res["single_cloud_ms"] = single
        iters = {"cube_n2048_c512_fps": 511, "lidar_n32768_c8192_fps": 8191, "lidar_n32768_c8192_npdu_m16_k64": 511,
                 "object_n8192_c2048_afps_m32": 63, "object_n8192_c2048_npdu_m32_k32": 63,
                 "object_n8192_c2048_fps": 2047}
        res["cycles_per_iteration"] = {k: round(v * 1e-3 * CLOCK_GHZ * 1e9 / iters[k], 1) for k, v in single.items()}
        res["cycles_per_iteration"]["note"] = "call time x 2.4 GHz / iterations of the longest sector (launch included)"
        res["object_n8192_c2048_sweep"], res["npdu_readings"] = object_sweep(torch, binding, synth, stream)
        res["sortedness"] = sortedness(torch, binding, synth, stream)
        res["grouping_ball_query"] = grouping(torch, binding, synth, stream)

    if not args.no_serve:
        res["serving"] = serving(torch)
        mid = res["serving"]["afps_npdu"]["200"]
        res["latency"] = {"unit": "ms", "what": "per frame, arrival to completion, AFPS-NPDU serving "
                                               "at 200 frames/s", "p50": mid["p50_ms"], "p99": mid["p99_ms"]}

    if not args.no_cpu:
        log("oracle CPU baseline")
        res["cpu_baseline"] = cpu_baseline(clouds, cs, M, K, out_np, plan.offsets)
        log("cpu baseline: %s" % res["cpu_baseline"])
    for p in plans:
        p.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
