"""Benchmark: batched AFPS-NPDU vs plain FPS on one MI355X.

One step = one pass of the whole sampling path over one batch: 256 object-like
clouds of uneven size (N log-uniform in [1024, 32768], C = N/4), AFPS with
M = 8 sectors and NPDU window k = 32 (2048 sectors).  The K timed steps are one
pooled launch of K rounds of that batch (afps_plan_launch_rounds: a stream of
batches processed back to back on the device; the rounds alternate over two
resident copies of the input and each writes its own output), bracketed by
synchronisations; the same launch's HIP-event duration is the roofline's time
basis, so `value` and `roofline` share one clock.  Inputs are resident in HBM
before the timed region, and untimed launches of the same shape run back to
back for --settle-ms right before it (a GPU coming out of idle needs tens of ms
of load to reach its steady clocks).  The same 256 clouds are also sampled with plain FPS.

Prints ONE JSON line (rank 0, N = 1).  Extra fields: one step's own latency,
device-measured cycles per iteration (per-sector timestamps), plain-FPS
figures with their roofline, single-cloud latencies of the paper-sized
configurations, coverage radius against plain FPS, the serving streams with
their p50/p99 and the served launches' roofline, and the oracle's CPU
baseline.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import gc
import hashlib
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sampled pts/s + p50/p99 frame latency, AFPS-NPDU vs plain FPS, 1 MI355X"
# MI355X figures for the rooflines.
HBM_PEAK_GBS = 8000.0
CUS, SIMDS_PER_CU = 256, 4
# fp32 VALU without FMA and without packed ops (the method's distance is a
# chain of separately rounded sub/mul/add): 256 CU x 4 SIMD x 16 lanes x 2.4 GHz.
VALU_PEAK_TOPS = CUS * SIMDS_PER_CU * 16 * 2.4e9 / 1e12
PEAK_CLOCK_GHZ = 2.4
# LDS bytes a CU serves per clock on 128-bit reads, measured with a
# microbenchmark on MI355X (every wave of eight workgroups per CU reading
# conflict-free 1 KB rows; see the LDS section of the design notes).
LDS_BYTES_PER_CLK_PER_CU = 128.0
# A wave64 VALU instruction occupies its SIMD's vector ALU for 4 cycles.
VALU_CYCLES_PER_INST = 4
# Bytes one LDS instruction of the NPDU loop moves, on average over its mix per
# iteration.  Coordinates in LDS records: one broadcast 16-byte read of the
# sample, two 16-byte reads of a window block each, one paired 4-byte write
# of the window's distances (1024 + 2 x 1024 + 512 bytes of lanes in 4
# instructions).  Coordinates in registers: one paired 4-byte read and one
# paired 4-byte write of the window's distances (512 + 512 in 2).
# Coordinates from L2 with windows of at most 64 points: a 4-byte read and
# write of the window's own lanes and a paired 4-byte read of the two blocks
# holding it (256 + 256 + 512 in 3).
LDS_BYTES_PER_INST_RECORDS = (1024 + 2 * 1024 + 512) / 4
LDS_BYTES_PER_INST_REGS = (512 + 512) / 2
LDS_BYTES_PER_INST_L2_WINDOW = (256 + 256 + 512) / 3


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def _event_ms(torch, run, stream, reps):
    """HIP-event durations (ms) of `reps` calls of run() on `stream`, one at a time."""
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run()
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return ms


def npdu_counts(sizes, cs, out_np, offsets, m, k, records_above=None):
    """Work of one pass of AFPS-NPDU over the batch, counted from its picks:
    distance updates (the exact window sizes), iterations, the window and
    block-maximum compares of the argmax (k + 1 + ceil(n_s / 64) per
    iteration) and the compares of an Algorithm-1 scan ((c_s - 1) n_s).
    With records_above, `updates_records` counts the updates of sectors of
    more points, whose coordinates sit in LDS records (the others' only D)."""
    upd = iters = win_cmp = blk_cmp = scan_cmp = upd_rec = 0
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
            if records_above is not None and ns > records_above:
                upd_rec += u
            iters += cc - 1
            win_cmp += (cc - 1) * (k + 1)
            blk_cmp += (cc - 1) * (-(-ns // 64))
            scan_cmp += (cc - 1) * ns
    return {"updates": upd, "iterations": iters, "ops": 9 * upd + win_cmp + blk_cmp,
            "alg1_scan_ops": 9 * upd + scan_cmp, "updates_records": upd_rec}


def fps_ops(sizes, cs):
    """Plain FPS: every point updated and compared once per iteration."""
    upd = sum((c - 1) * n for n, c in zip(sizes, cs))
    return 9 * upd + upd, upd


def counter_record(label):
    """Per-round SQ / traffic counters of the pooled kernel in `label`'s launch
    layout and coordinate placement from the committed rocprofv3 record, or
    None when the kernel or plan sources changed since or that layout was not
    profiled."""
    path = os.path.join(ROOT, "profiles", "pooled_npdu_kernel_batch256_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = "".join(open(os.path.join(ROOT, s)).read() for s in rec["sources"])
    if hashlib.sha256(src.encode()).hexdigest() != rec["source_sha256"]:
        return None
    return rec.get("kernels", {}).get(label)


def stamp_cycles(stamps, wall_khz):
    """Device-measured cycles per iteration from one stamped launch: per
    sector (end - loaded) / (c - 1) on the shader clock, the shader clock's
    rate from the constant-rate counter, and the critical sector."""
    st = stamps.cpu().numpy()
    pairs = st[:, 5:8].copy().view(np.int32).reshape(-1, 6)   # item, n, c, k, hw_id, xcc_id
    take, loaded, end, take_rt, end_rt = (st[:, j].astype(np.float64) for j in range(5))
    n, c = pairs[:, 1], pairs[:, 2]
    ok = c > 1
    cyc = (end - loaded)[ok] / (c[ok] - 1)
    ghz = float((end - take).sum() / (end_rt - take_rt).sum() * wall_khz * 1e-6) if wall_khz else None
    # shader-clock counters differ between XCDs: compare sectors on the
    # constant-rate counter only (the launch's first take to each sector's end)
    crit = int(np.argmax(end_rt))
    return {"median": round(float(np.median(cyc)), 1), "p10": round(float(np.percentile(cyc, 10)), 1),
            "p90": round(float(np.percentile(cyc, 90)), 1),
            "critical_sector": {"points": int(n[crit]), "samples": int(c[crit]),
                                "cycles_per_iteration": round(float((end[crit] - loaded[crit]) / max(1, c[crit] - 1)), 1),
                                "load_us": round(float((loaded[crit] - take[crit]) / (ghz * 1e3)), 2) if ghz else None,
                                "ends_at_us": round(float((end_rt[crit] - take_rt.min()) / (wall_khz * 1e-3)), 1)
                                if wall_khz else None},
            "by_points": {label: round(float(np.median(cyc[(n[ok] > lo) & (n[ok] <= hi)])), 1)
                          for label, lo, hi in (("<=1024", 0, 1024), ("1025-2048", 1024, 2048),
                                                ("2049-4096", 2048, 4096))
                          if ((n[ok] > lo) & (n[ok] <= hi)).any()},
            "sclk_ghz": round(ghz, 4) if ghz else None,
            "what": "shader-clock cycles per iteration of each NPDU sector of one pass, from s_memtime stamps "
                    "when the sector was in LDS and when its last pick was written; clock rate from "
                    "s_memrealtime"}


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


def object_sweep(torch, binding, synth, stream, clock_ghz, reps=10):
    """Object cloud N=8192, C=2048: plain FPS, AFPS for M in {1..32}, NPDU at
    k in {8, 32, 128}: time per call (median), cycles per iteration of the
    longest sector (call time at the measured shader clock, launch included),
    coverage radius relative to plain FPS.  Then the
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
                         "cycles_per_iteration": round(ms * 1e-3 * clock_ghz * 1e9 / iters, 1),
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




def serving(torch, ops_fn, rates=(50, 200, 800), seconds=10.0, max_frames=2000, pool=48, seed=1):
    """Open-loop Poisson streams of LiDAR frames (N uniform in [16384, 131072],
    C = N/8, M in {8, 16, 32}, k = 64) through the continuous-batching server:
    AFPS-NPDU for min(2000 frames, 10 s of arrivals) per rate, plain FPS for a
    fixed 10 s window per rate (what completed, and the queue left at the
    end).  Per-frame latency from arrival to completion, the indices back on
    the host.  The served launches' roofline: algorithmic ops of each batch
    (from its picks) over its launches' HIP-event time."""
    from paper_2208_08795_amd import synth
    from paper_2208_08795_amd.serve import GpuExecutor, Request, Scheduler, latency_summary
    rng = np.random.default_rng(seed)
    log("generating %d serving frames" % pool)
    frames = synth.frame_stream(rate=1.0, count=pool, seed=seed)
    pinned = [torch.from_numpy(f.points).pin_memory() for f in frames]
    budget = 256 << 20
    ex = GpuExecutor(budget, streams=4, keep_results=True, timing=True)
    res = {"budget_bytes": budget,
           "frames": "pool of %d distinct synthetic 64-beam frames, N uniform in [16384, 131072], C = N/8, "
                     "M in {8,16,32}, k = 64; indices copied back to pinned host memory per frame" % pool,
           "length": "AFPS-NPDU: min(%d frames, %.0f s of arrivals) per rate; plain FPS: a %.0f s window per rate"
                     % (max_frames, seconds, seconds)}

    def stream(method, count, lam, window=None):
        gaps = rng.exponential(1.0 / lam, count)
        arr = np.cumsum(gaps) - gaps[0]
        reqs = []
        for i in range(count):
            f = frames[i % pool]
            m, k = (f.m, f.k) if method == "afps_npdu" else (1, None)
            reqs.append(Request(i, f.points.shape[0], f.c, m, k, 0, float(arr[i]), pinned[i % pool]))
        s = Scheduler(ex, budget, max_inflight=8, max_batch=32)
        # a serving loop keeps the collector out of its frames' latency
        gc.collect()
        gc.disable()
        try:
            done = s.run(reqs, window=window)
            torch.cuda.synchronize()
        finally:
            gc.enable()
        out = latency_summary(done)
        out.update({"offered_fps": lam, "offered_frames": count, "peak_waiting": s.peak_waiting,
                    "peak_arena_bytes": s.peak_bytes})
        if window is not None:
            out.update({"window_s": window, "left_waiting": s.left_waiting,
                        "oldest_wait_ms": s.oldest_wait_s * 1e3})
        ops = ms = 0.0
        per_launch = []
        for b in s.batch_log:
            if b.kernel_ms is None or b.kernel_ms <= 0:
                continue
            o = sum(ops_fn(r) for r in b.requests if r.state == "done")
            ops += o
            ms += b.kernel_ms
            per_launch.append(o / (b.kernel_ms * 1e-3) / 1e12)
        if per_launch:
            out["roofline"] = {"bound": "alu", "unit": "TOPS (fp32 VALU lane-ops)", "peak": VALU_PEAK_TOPS,
                               "achieved_mean_per_launch": float(np.mean(per_launch)),
                               "frac": float(np.mean(per_launch)) / VALU_PEAK_TOPS,
                               "launches": len(per_launch), "mean_launch_ms": ms / len(per_launch),
                               "what": "per batch: its algorithmic ops over its sampling launches' HIP-event "
                                       "time (batches on four streams overlap), mean over batches"}
        return out

    for method in ("afps_npdu", "plain_fps"):
        stream(method, 6, 1000.0)            # warm-up (plans, kernel attributes)
        res[method] = {}
        for lam in rates:
            if method == "afps_npdu":
                r = stream(method, int(min(max_frames, math.ceil(seconds * lam))), float(lam))
            else:
                r = stream(method, int(math.ceil(seconds * lam)), float(lam), window=seconds)
            res[method][str(lam)] = r
            log("serve %s @%d/s: %d frames, p50 %.2f ms p99 %.2f ms, %.3e pts/s, left waiting %s" %
                (method, lam, r.get("frames", 0), r.get("p50_ms") or 0, r.get("p99_ms") or 0,
                 r.get("sampled_pts_per_s") or 0, r.get("left_waiting", 0)))
    return res


def served_ops(req):
    """Algorithmic ops of one served frame from its picks (NPDU: 9 per window
    update + the argmax compares; plain FPS: 10 per point per iteration)."""
    if req.result is None:
        return 0.0
    out = req.result.numpy()
    if req.k is None and req.m == 1:
        return 10.0 * (req.c - 1) * req.n
    return float(npdu_counts([req.n], [req.c], out, [0], req.m, req.k)["ops"])




def lscpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return host_cpu_model()


def cpu_baseline(clouds, cs, m, k, gpu_out, offsets, budget_s=20.0):
    """The oracle (never tuned) on the host: single-thread latency per cloud,
    and throughput with one cloud per task on every host core the process may
    use, capped at the 16 threads a one-GPU machine grants a job.  Median of up to
    five whole passes over a bounded sample, input generation untimed."""
    import oracle
    oracle.load()
    nproc = os.cpu_count() or 1
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else nproc
    threads = max(1, min(16, allowed))
    # bounded sample: clouds in order until the estimated single-core work
    # (~ N C / m x 2 ns) reaches the budget
    est, take = 0.0, 0
    for p, c in zip(clouds, cs):
        est += len(p) * c / m * 2e-9
        take += 1
        if est > budget_s * threads * 0.5:
            break
    idx = list(range(take))

    def one(i):
        t = time.perf_counter()
        o = oracle.afps(clouds[i], cs[i], m, k, 0)
        return o, time.perf_counter() - t

    # latency leg: one thread, every cloud of the sample once (the first 64 at most)
    lat_idx = idx[:64]
    lat = [one(i)[1] * 1e3 for i in lat_idx]
    # throughput leg: whole passes on `threads` threads
    dts = []
    with cf.ThreadPoolExecutor(threads) as ex:
        while len(dts) < 5 and sum(dts) < budget_s:
            t0 = time.perf_counter()
            res = list(ex.map(one, idx))
            dts.append(time.perf_counter() - t0)
    dt = float(np.median(dts))
    outs = [o for o, _ in res]
    same = all(np.array_equal(outs[j], gpu_out[offsets[i]:offsets[i] + cs[i]]) for j, i in enumerate(idx))
    samples = sum(cs[i] for i in idx)
    return {"value": samples / dt, "unit": "sampled pts/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of the 256 clouds (%d points, %d samples), AFPS M=%d NPDU k=%d, one cloud "
                      "per task on %d threads; median of %d passes, %.2f s each" %
                      (take, sum(len(clouds[i]) for i in idx), samples, m, k, threads, len(dts), dt),
            "host": {"nproc": nproc, "affinity_cpus": allowed, "threads_used": threads,
                     "thread_cap": "16 threads: a one-GPU box's share of host CPUs",
                     "cpu_model": lscpu_model()},
            "matches_gpu": bool(same),
            "single_thread_latency_ms_per_cloud": {"p50": float(np.percentile(lat, 50)),
                                                    "p99": float(np.percentile(lat, 99)),
                                                    "clouds": len(lat),
                                                    "mean_points": float(np.mean([len(clouds[i]) for i in lat_idx]))}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-single", action="store_true", help="skip single-cloud latencies and sweeps")
    ap.add_argument("--no-fps", action="store_true", help="skip the plain-FPS comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving streams")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuners (built-in rules)")
    ap.add_argument("--pool", type=str, default=None,
                    help="pooled launch policy 'waves,groups[,seed_sleep,seed_priority]' for the timed batch "
                         "(skips its tuning; seeding defaults to 1,3)")
    ap.add_argument("--regs-up-to", type=int, default=None,
                    help="NPDU sectors of at most this many points hold their coordinates out of LDS "
                         "(registers), larger ones in LDS (with --pool; 0 = all in LDS)")
    ap.add_argument("--settle-ms", type=float, default=50.0,
                    help="untimed launches of the timed launch's shape, back to back right before it, for at "
                         "least this long (0: none)")
    ap.add_argument("--only-timed", action="store_true",
                    help="stop after the timed launch (for profiler runs: warm-up and timed launches only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent clouds would shard by request with no exchange)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.steps > 4096 or args.warmup < 0 or args.settle_ms < 0:
        ap.error("--steps must be in [1, 4096] (rounds of one launch), --warmup and --settle-ms >= 0")

    import torch
    from paper_2208_08795_amd import autotune, binding, synth
    from paper_2208_08795_amd.quality import coverage_radius

    L = binding.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    M, K = 8, 32
    log("generating 256 clouds")
    clouds = synth.batch_of_objects(256, seed=args.seed)
    sizes = [len(p) for p in clouds]
    cs = [n // 4 for n in sizes]
    xyz_all = torch.from_numpy(np.concatenate(clouds)).to(dev)
    xyz_copy = xyz_all.clone()                  # the rounds alternate over two resident inputs
    total_samples = sum(cs)

    # A plain device copy of known size: rocprofv3 --pmc runs read its
    # FETCH_SIZE / WRITE_SIZE to calibrate the counters.
    calib = torch.empty(64 << 20, dtype=torch.uint8, device=dev)
    calib2 = torch.empty_like(calib)
    calib2.copy_(calib)

    res_tune = None
    if args.pool is not None:
        pol = [int(x) for x in args.pool.split(",")]
        if len(pol) not in (2, 4):
            ap.error("--pool takes waves,groups or waves,groups,seed_sleep,seed_priority")
        w, g = pol[:2]
        sleep, prio = (pol[2], pol[3]) if len(pol) == 4 else (1, 3)
        binding.set_pool_policy(w, g, bool(sleep), prio)
        if args.regs_up_to is not None:
            if args.regs_up_to:
                binding.tune_npdu(args.regs_up_to, K, False)
            binding.tune_npdu(8192, K, True)
    elif not args.no_tune:
        log("tuning the pooled NPDU launch on the batch")
        res_tune = autotune.tune_npdu(xyz_all, sizes, cs, [M] * 256, [K] * 256, [0] * 256, rounds=20, log=log)
    plan = binding.BatchPlan(sizes, cs, [M] * 256, [K] * 256, [0] * 256, device=dev)
    label = "pooled_npdu_kernel<%d>" % plan.pool_waves
    if plan.pool_groups > 1:
        label += " x%d per CU" % plan.pool_groups
    regs_up_to = max((n for n in range(64, 8193, 64) if not binding.npdu_xyz_in_lds(n, K)), default=0)
    log("AFPS-NPDU plan: %d sectors, %s, coordinates out of LDS up to %d points" % (plan.items, label, regs_up_to))

    # ---- the timed steps: one launch of K rounds, each round its own output;
    # the warm-up launch (W rounds) writes a reference of its own
    steps, warm = args.steps, args.warmup
    outs = torch.full((steps, plan.total_samples), -7, dtype=torch.int32, device=dev)
    inputs = (xyz_all, xyz_copy)
    table = plan.round_table([(inputs[r % 2], outs[r]) for r in range(steps)])
    wouts = torch.full((max(1, warm), plan.total_samples), -7, dtype=torch.int32, device=dev)
    wtable = plan.round_table([(inputs[r % 2], wouts[r]) for r in range(max(1, warm))])
    plan.launch_rounds(wtable, stream=stream)
    torch.cuda.synchronize()
    ref = wouts[0].clone()
    out_np = ref.cpu().numpy()          # checked against the oracle by cpu_baseline
    if not bool((wouts == ref.unsqueeze(0)).all()):
        raise SystemExit("bench: the warm-up rounds' indices differ")
    if not args.only_timed:             # and against a separate single pass
        single = plan.launch(xyz_all, stream=stream)
        torch.cuda.synchronize()
        if not torch.equal(single, ref):
            raise SystemExit("bench: a round's indices differ from a single pass")
    # The GPU's clocks settle only after tens of ms of continuous load (a
    # launch that starts from idle runs its first ~20 ms up to 10% slower), so
    # launches of the timed launch's own shape (K rounds, their own outputs)
    # run back to back, untimed, right before it: the timed launch then
    # measures the steady state of a stream of batches.
    settle = None
    if args.settle_ms > 0:
        souts = torch.full((steps, plan.total_samples), -7, dtype=torch.int32, device=dev)
        stable = plan.round_table([(inputs[r % 2], souts[r]) for r in range(steps)])
        torch.cuda.synchronize()
        ts, n_settle = time.perf_counter(), 0
        while n_settle == 0 or time.perf_counter() - ts < args.settle_ms / 1e3:
            plan.launch_rounds(stable, stream=stream)
            torch.cuda.synchronize()
            n_settle += 1
        settle = {"launches": n_settle, "rounds": n_settle * steps,
                  "ms": round((time.perf_counter() - ts) * 1e3, 2),
                  "what": "untimed launches of K rounds (the timed launch's shape, outputs of their own, checked "
                          "after the timed launch), back to back right before it, so that the timed launch starts "
                          "at the clocks of continuous load"}
    # The events' first record creates them (about 40 us of host time):
    # done before the timed region, which then holds only the launch.
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev_a.record(stream)
    ev_b.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev_a.record(stream)
    plan.launch_rounds(table, stream=stream)
    ev_b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = ev_a.elapsed_time(ev_b)
    sclk = shader_clock_mhz()
    plan.status(stream=stream)
    if not bool((outs == ref.unsqueeze(0)).all()):
        raise SystemExit("bench: a timed round's indices differ from the warm-up's")
    if settle is not None:
        if not bool((souts == ref.unsqueeze(0)).all()):
            raise SystemExit("bench: a settling round's indices differ from the warm-up's")
        del souts, stable
    ms_per_step = wall * 1e3 / steps
    value = total_samples * steps / wall
    log("AFPS-NPDU: %d rounds in one launch, %.4f ms/step (launch %.3f ms), %.3e sampled pts/s" %
        (steps, ms_per_step, launch_ms, value))

    res = {"metric": METRIC, "value": value, "unit": "sampled pts/s", "n_gpus": 1, "steps": steps,
           "warmup": warm, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256 object-like clouds, N log-uniform [1024, 32768] (%d points), "
                                  "C = N/4 (%d samples), AFPS M=8 with NPDU k=32; the K timed steps are one "
                                  "pooled launch of K rounds of the batch (alternating two resident inputs, "
                                  "one output per round)" % (sum(sizes), total_samples),
                      "clouds": 256, "m": M, "k": K, "points": sum(sizes), "samples": total_samples,
                      "pool_launch": label, "coordinates_out_of_lds_up_to_points": regs_up_to}}
    if res_tune is not None:
        res["npdu_tuning"] = {"best": {"shape": list(res_tune["best"][0]), "regs_up_to": res_tune["best"][1],
                                       "seed_sleep": res_tune["best"][2][0], "seed_priority": res_tune["best"][2][1],
                                       "ms_per_step": round(res_tune["best"][3], 4)},
                              "rows": [[list(r[0]), r[1], list(r[2]), round(r[3], 4)] for r in res_tune["rows"]],
                              "seconds": round(res_tune["seconds"], 2),
                              "what": "ms per batch in one launch of 20 rounds, per pooled launch shape "
                                      "(waves, workgroups per CU), bound of coordinates out of LDS and seeding (sleep, priority)"}
    res["settle"] = settle
    res["sclk_mhz_after_timed_steps"] = sclk

    # ---- roofline of the dominant kernel, on the timed launch's own time
    cnt = npdu_counts(sizes, cs, out_np, plan.offsets, M, K, records_above=regs_up_to)
    stamps = None
    wall_khz = int(L.afps_wall_clock_khz())
    if not args.only_timed:
        _, stamps = plan.launch_stamped(xyz_all, stream=stream)
        torch.cuda.synchronize()
    cyc = stamp_cycles(stamps, wall_khz) if stamps is not None else None
    clock_ghz = (cyc or {}).get("sclk_ghz") or PEAK_CLOCK_GHZ
    launch_s = launch_ms / 1e3
    round_s = launch_s / steps
    ops_launch = cnt["ops"] * steps
    hbm_round = 12 * sum(sizes) + 4 * total_samples + 40 * plan.items
    # per update: 16 B read (x, y, z, D) + 4 B written with LDS records, 4 + 4 B
    # (D only) with the coordinates in registers
    lds_round = 20 * cnt["updates_records"] + 8 * (cnt["updates"] - cnt["updates_records"])
    lds_peak_tbs = CUS * LDS_BYTES_PER_CLK_PER_CU * clock_ghz * 1e9 / 1e12
    rec = counter_record("%s, coordinates out of LDS up to %d" % (label, regs_up_to))
    roof = {"bound": "alu", "kernel": label, "achieved": ops_launch / launch_s / 1e12, "peak": VALU_PEAK_TOPS,
            "unit": "TOPS (fp32 VALU lane-ops)", "frac": ops_launch / launch_s / 1e12 / VALU_PEAK_TOPS,
            "traffic": (int(rec["traffic_bytes_per_round"] * steps) if rec and rec.get("traffic_bytes_per_round")
                        else None),
            "time_basis": "the timed launch of %d rounds (the K steps), HIP events on its stream; `value` "
                          "divides the same launch's samples by its synchronised wall time" % steps,
            "avg_launch_ms": launch_ms, "rounds_per_launch": steps, "launches_timed": 1,
            "algorithmic_ops_per_launch": ops_launch,
            "ops_count": "9 per window distance update (3 sub, 3 mul, 2 add, 1 min) + (k+1) window compares + "
                         "ceil(n_s/64) block-maximum compares per iteration",
            "alg1_scan_ops_per_launch": cnt["alg1_scan_ops"] * steps,
            "alg1_scan_frac": cnt["alg1_scan_ops"] * steps / launch_s / 1e12 / VALU_PEAK_TOPS,
            "distance_updates_per_launch": cnt["updates"] * steps, "iterations_per_round": cnt["iterations"],
            "hbm_bytes_per_launch": hbm_round * steps, "hbm_frac": hbm_round / round_s / 1e9 / HBM_PEAK_GBS,
            "lds": {"algorithmic_bytes_per_launch": lds_round * steps,
                    "achieved_tbs": lds_round / round_s / 1e12, "peak_tbs": lds_peak_tbs,
                    "frac": lds_round / round_s / 1e12 / lds_peak_tbs,
                    "peak_basis": "%d CUs x %.0f B/clk (measured, 128-bit reads) x %.3f GHz (measured)" %
                                  (CUS, LDS_BYTES_PER_CLK_PER_CU, clock_ghz)},
            "clock_ghz": clock_ghz}
    if rec:
        valu = rec["SQ_INSTS_VALU_per_round"]
        roof["valu_issue_frac"] = valu * VALU_CYCLES_PER_INST / (CUS * SIMDS_PER_CU * round_s * clock_ghz * 1e9)
        if cnt["updates_records"]:
            per_inst = LDS_BYTES_PER_INST_RECORDS
        else:   # the 4- and 8-wave kernels hold coordinates out of LDS in registers, the others read L2
            per_inst = LDS_BYTES_PER_INST_REGS if plan.pool_waves <= 8 or K > 63 else LDS_BYTES_PER_INST_L2_WINDOW
        kb = rec["SQ_INSTS_LDS_per_round"] * per_inst
        roof["lds"].update({"kernel_bytes_per_launch": kb * steps, "kernel_frac": kb / round_s / 1e12 / lds_peak_tbs})
        roof["counters_per_round"] = {k: v for k, v in rec.items() if k.endswith("_per_round")}
        roof["counters_note"] = ("SQ and traffic counters per round from the committed rocprofv3 record of this "
                                 "launch layout (kernel sources unchanged since); VALU issue = SQ_INSTS_VALU x "
                                 "%d cycles over %d SIMDs x the round's cycles" % (VALU_CYCLES_PER_INST,
                                                                                 CUS * SIMDS_PER_CU))
    else:
        roof["valu_issue_frac"] = None
        roof["counters_note"] = "no rocprofv3 counter record matches the current kernel sources and layout"
    res["roofline"] = roof
    if cyc is not None:
        res["cycles_per_iteration_device"] = cyc
    if args.only_timed:
        print(json.dumps(res), flush=True)
        return

    # ---- one step's own latency (one pass at a time, graph replays): the
    # throughput-tuned plan, then the built-in policy (coordinates in LDS
    # records: the shortest single launch), which the rest of the run (serving
    # included) keeps as the latency operating point
    reps = max(20, min(steps, 100))
    plan.launch(xyz_all, out_all=ref, graph=True, stream=stream)
    torch.cuda.synchronize()
    ev_tuned = _event_ms(torch, lambda: plan.launch(xyz_all, out_all=ref, graph=True, stream=stream), stream, reps)
    binding.tune_npdu_clear()
    binding.set_pool_policy(0, 0, True, 3)
    lplan = binding.BatchPlan(sizes, cs, [M] * 256, [K] * 256, [0] * 256, device=dev)
    lout = lplan.launch(xyz_all, stream=stream, graph=True)
    torch.cuda.synchronize()
    if not torch.equal(lout, ref):
        raise SystemExit("bench: the built-in policy's indices differ from the tuned plan's")
    ev_ms = _event_ms(torch, lambda: lplan.launch(xyz_all, out_all=lout, graph=True, stream=stream), stream, reps)
    res["batch_latency"] = {"unit": "ms", "what": "one step alone (the whole batch of 256 clouds, one pooled "
                                                  "launch per step, graph replays one at a time), HIP events, "
                                                  "built-in policy (pooled_npdu_kernel<%d>, coordinates in LDS "
                                                  "records): the latency operating point, kept for the rest of "
                                                  "the run" % lplan.pool_waves,
                            "p50": percentile(ev_ms, 50), "p99": percentile(ev_ms, 99),
                            "throughput_policy": {"kernel": label, "p50": percentile(ev_tuned, 50),
                                                  "p99": percentile(ev_tuned, 99)}}
    lplan.close()

    if not args.no_tune:
        log("autotuning full-update variants")
        tab = autotune.tune(log=log)
        res["autotune"] = {k: [[int(n), int(w), int(p), round(ms, 4)] for n, w, p, ms in v]
                           for k, v in tab.items() if k != "seconds"}
        res["autotune"]["seconds"] = round(tab["seconds"], 2)

    if not args.no_fps:
        fplan = binding.BatchPlan(sizes, cs, [1] * 256, [None] * 256, [0] * 256, device=dev)
        fout = fplan.launch(xyz_all, stream=stream, graph=True)
        torch.cuda.synchronize()
        fsteps = max(3, min(steps // 10, 20))
        fev = _event_ms(torch, lambda: fplan.launch(xyz_all, out_all=fout, graph=True, stream=stream), stream,
                        fsteps)
        fms = float(np.mean(fev))
        fops, fupd = fps_ops(sizes, cs)
        fvalue = total_samples / (fms / 1e3)
        fout_np = fout.cpu().numpy()
        log("plain FPS: %.3f ms/step, %.3e sampled pts/s" % (fms, fvalue))
        fhbm = 12 * sum(sizes) + 4 * total_samples + 40 * fplan.items
        res["plain_fps"] = {"value": fvalue, "unit": "sampled pts/s", "ms_per_step": fms, "steps": fsteps,
                            "launches": fplan.launches,
                            "latency_p50_ms": percentile(fev, 50), "latency_p99_ms": percentile(fev, 99),
                            "afps_npdu_speedup": value / fvalue,
                            "roofline": {"bound": "alu", "achieved": fops / (fms / 1e3) / 1e12,
                                         "peak": VALU_PEAK_TOPS, "unit": "TOPS (fp32 VALU lane-ops)",
                                         "frac": fops / (fms / 1e3) / 1e12 / VALU_PEAK_TOPS,
                                         "algorithmic_ops_per_launch": fops, "distance_updates_per_launch": fupd,
                                         "hbm_bytes_per_launch": fhbm,
                                         "hbm_frac": fhbm / (fms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                         "avg_launch_ms": fms,
                                         "time_basis": "one step (the plan's persistent launches, one workgroup "
                                                       "per cloud), HIP events, steps one at a time",
                                         "ops_count": "10 per point per iteration (9 for its distance update, 1 "
                                                      "argmax compare)"}}
        ratios = []
        for i in range(0, 256, 8):
            o = plan.offsets[i]
            ratios.append(coverage_radius(clouds[i], out_np[o:o + cs[i]]) /
                          coverage_radius(clouds[i], fout_np[o:o + cs[i]]))
        res["coverage_radius_vs_fps"] = {"mean": float(np.mean(ratios)), "max": float(np.max(ratios)),
                                         "clouds": len(ratios)}
        fplan.close()

    if not args.no_single:
        single = single_cloud_latency(torch, binding, synth, stream)
        res["single_cloud_ms"] = single
        iters = {"cube_n2048_c512_fps": 511, "lidar_n32768_c8192_fps": 8191, "lidar_n32768_c8192_npdu_m16_k64": 511,
                 "object_n8192_c2048_afps_m32": 63, "object_n8192_c2048_npdu_m32_k32": 63,
                 "object_n8192_c2048_fps": 2047}
        res["cycles_per_iteration"] = {k: round(v * 1e-3 * clock_ghz * 1e9 / iters[k], 1) for k, v in single.items()}
        res["cycles_per_iteration"]["note"] = ("call time x the measured shader clock (%.3f GHz) / iterations of the "
                                               "longest sector (launch included)" % clock_ghz)
        res["object_n8192_c2048_sweep"], res["npdu_readings"] = object_sweep(torch, binding, synth, stream, clock_ghz)
        res["sortedness"] = sortedness(torch, binding, synth, stream)
        res["grouping_ball_query"] = grouping(torch, binding, synth, stream)

    if not args.no_serve:
        res["serving"] = serving(torch, served_ops)
        mid = res["serving"]["afps_npdu"]["200"]
        res["latency"] = {"unit": "ms", "what": "per frame, arrival to completion (indices back on the host), "
                                               "AFPS-NPDU serving at 200 frames/s", "p50": mid["p50_ms"],
                          "p99": mid["p99_ms"]}

    if not args.no_cpu:
        log("oracle CPU baseline")
        res["cpu_baseline"] = cpu_baseline(clouds, cs, M, K, out_np, plan.offsets)
        log("cpu baseline: %s" % res["cpu_baseline"])
    plan.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
