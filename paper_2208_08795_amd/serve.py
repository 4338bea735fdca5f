"""Serving loop: continuous batching of point-cloud frames on one GPU.

Frames arrive over time (e.g. LiDAR sweeps).  The scheduler admits a waiting
frame when its HBM footprint fits in a fixed device arena (points, output
indices and its share of the batch workspace) and a launch slot is free; all
frames admitted in one tick form one batch (frames of different sizes and
sector counts), which the executor copies into the arena and samples with one
batch-plan launch on one of several streams.  Batches launched while others
are still running overlap on the device.  When a batch's completion event has
fired, its frames are done (latency = completion - arrival, host clock) and
their arena blocks are freed for the next admissions.  A frame's indices come
back to the host with it (an asynchronous copy into a pinned mirror of the
arena, ordered before the completion event); a frame whose indices hold -1
(a kernel gave up a bounded wait, see afps_set_spin_limit) is "failed".

The scheduler (admission, arena, bookkeeping) is plain host logic; the
executor is the only part that touches the GPU, so the policy can be checked
with a fake executor and a fake clock.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np

ALIGN = 768          # lcm(256, 12): a block offset is both 256-byte and point aligned


class Arena:
    """First-fit allocator over [0, size) bytes, blocks aligned to ALIGN."""

    def __init__(self, size: int):
        self.size = size - size % ALIGN
        self.free_list = [(0, self.size)]      # (offset, length), sorted, coalesced
        self.used = {}

    def alloc(self, nbytes: int):
        need = -(-max(nbytes, 1) // ALIGN) * ALIGN
        for i, (off, ln) in enumerate(self.free_list):
            if ln >= need:
                if ln == need:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + need, ln - need)
                self.used[off] = need
                return off
        return None

    def free(self, off: int):
        ln = self.used.pop(off)
        fl = self.free_list
        fl.append((off, ln))
        fl.sort()
        merged = []
        for o, l in fl:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((o, l))
        self.free_list = merged

    @property
    def bytes_used(self) -> int:
        return sum(self.used.values())


@dataclass
class Request:
    rid: int
    n: int
    c: int
    m: int
    k: int | None                 # None: no NPDU (m == 1 and None is plain FPS)
    start: int
    arrival: float
    points: object = None         # host points (pinned torch tensor or numpy)
    state: str = "pending"        # pending -> waiting -> running -> done | failed | rejected
    admitted: float = None
    done: float = None
    pts_off: int = None
    out_off: int = None
    result: object = None
    error: str = None

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


def footprint(req: Request) -> tuple[int, int]:
    """(points bytes, output bytes) a frame needs on the device."""
    return 12 * req.n, 4 * req.c


def library_workspace_bytes(items: int) -> int:
    """Workspace of a batch plan with `items` sectors, as the library sizes it."""
    from . import binding
    return binding.workspace_bytes_for_items(items)


@dataclass
class Batch:
    requests: list
    ws_off: int = None
    ws_bytes: int = 0          # size of the arena block reserved for the plan's workspace
    handle: object = None
    launched: float = None
    kernel_ms: float = None    # the sampling launches' own time (HIP events), when the executor times them


class Scheduler:
    """Admission by HBM footprint, continuous batching, bounded launches in flight."""

    def __init__(self, executor, arena_bytes: int, max_inflight: int = 8, max_batch: int = 64,
                 clock=time.perf_counter, workspace_bytes=library_workspace_bytes):
        self.ex = executor
        self.workspace_bytes = workspace_bytes   # items -> bytes of a plan's workspace
        self.arena = Arena(arena_bytes)
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.clock = clock
        self.waiting = []
        self.inflight = []
        self.finished = []
        self.peak_bytes = 0
        self.peak_waiting = 0
        self.batch_log = []            # completed batches, in completion order
        self.left_waiting = 0          # frames still waiting when a time window closed
        self.oldest_wait_s = 0.0       # how long the oldest of them had waited then

    def _fits_ever(self, req) -> bool:
        p, o = footprint(req)
        w = self.workspace_bytes(req.m)
        blocks = sum(-(-x // ALIGN) * ALIGN for x in (p, o, w))
        return blocks <= self.arena.size

    def submit(self, req: Request):
        if not self._fits_ever(req):
            req.state = "rejected"
            req.error = "frame footprint exceeds the device budget"
            self.finished.append(req)
            return
        req.state = "waiting"
        self.waiting.append(req)
        self.peak_waiting = max(self.peak_waiting, len(self.waiting))

    def _admit(self, now):
        if len(self.inflight) >= self.max_inflight or not self.waiting:
            return None
        batch, taken, items = [], 0, 0
        for req in self.waiting:                     # FIFO: stop at the first that does not fit
            if len(batch) >= self.max_batch:
                break
            p, o = footprint(req)
            po = self.arena.alloc(p)
            if po is None:
                break
            oo = self.arena.alloc(o)
            if oo is None:
                self.arena.free(po)
                break
            req.pts_off, req.out_off = po, oo
            batch.append(req)
            items += req.m
            taken += 1
        if not batch:
            return None
        # The plan's workspace (queue counters + one work item per sector),
        # sized exactly as the library sizes it.
        ws_need = self.workspace_bytes(items)
        ws = self.arena.alloc(ws_need)
        while ws is None:                             # give the last frame back and retry smaller
            last = batch.pop()
            self.arena.free(last.pts_off)
            self.arena.free(last.out_off)
            last.pts_off = last.out_off = None
            items -= last.m
            taken -= 1
            if not batch:
                return None
            ws_need = self.workspace_bytes(items)
            ws = self.arena.alloc(ws_need)
        del self.waiting[:taken]
        for req in batch:
            req.state, req.admitted = "running", now
        self.peak_bytes = max(self.peak_bytes, self.arena.bytes_used)
        return Batch(batch, ws, self.arena.used[ws])

    def _release(self, batch: Batch):
        for req in batch.requests:
            if req.pts_off is not None:
                self.arena.free(req.pts_off)
                self.arena.free(req.out_off)
        self.arena.free(batch.ws_off)

    def _complete(self):
        """Finish the batches whose completion event has fired; True if any did."""
        moved = False
        for batch in list(self.inflight):
            if self.ex.done(batch.handle):
                t = self.clock()
                failed = self.ex.finish(batch) or {}
                for req in batch.requests:
                    req.done = t
                    if req.rid in failed:
                        req.state, req.error = "failed", failed[req.rid]
                    else:
                        req.state = "done"
                    self.finished.append(req)
                self._release(batch)
                self.inflight.remove(batch)
                self.batch_log.append(batch)
                moved = True
        return moved

    def step(self):
        """Complete finished batches, then admit and launch. Returns True if anything moved."""
        now = self.clock()
        moved = self._complete()
        while True:
            batch = self._admit(now)
            if batch is None:
                break
            try:
                batch.handle = self.ex.launch(batch)
                batch.launched = now
                self.inflight.append(batch)
            except Exception as e:                     # a failed launch fails its frames only
                for req in batch.requests:
                    req.state, req.error = "failed", str(e)
                    self.finished.append(req)
                self._release(batch)
            moved = True
        return moved

    def run(self, requests, idle_sleep: float = 0.0, window: float | None = None):
        """Feed requests at their arrival times (seconds after the start) until
        all finish, or, with `window`, until that many seconds have passed:
        then frames not yet arrived are dropped, frames still waiting stay in
        self.waiting (counted in left_waiting, the longest wait in
        oldest_wait_s) and the batches on the device complete."""
        pending = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in pending:
            r.arrival += t0
        i = 0
        while i < len(pending) or self.waiting or self.inflight:
            now = self.clock()
            if window is not None and now - t0 >= window:
                self.left_waiting = len(self.waiting)
                self.oldest_wait_s = max((now - r.arrival for r in self.waiting), default=0.0)
                while self.inflight:
                    self.clock()
                    if not self._complete() and idle_sleep:
                        time.sleep(idle_sleep)
                break
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            if not self.step() and idle_sleep:
                time.sleep(idle_sleep)
        return self.finished


class GpuExecutor:
    """Copies a batch's frames into the device arena and samples them in one
    batch-plan launch (NPDU-AFPS / AFPS) or one launch per frame (plain FPS),
    on one of `streams` HIP streams, then copies each frame's indices into a
    pinned host mirror of the arena; completion is an event.  `on_launch`, if
    given, is called with (stream, batch) right after the sampling launches
    (e.g. to record timing events around them)."""

    def __init__(self, arena_bytes: int, streams: int = 4, keep_results: bool = False,
                 device="cuda", on_launch=None, timing: bool = False):
        import torch

        from . import binding
        self.torch, self.B = torch, binding
        self.L = binding.lib()
        self.buf = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        self.base = self.buf.data_ptr()
        self.host = torch.empty(arena_bytes, dtype=torch.uint8, pin_memory=True)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(streams)]
        self.next = 0
        self.keep = keep_results
        self.on_launch = on_launch
        self.timing = timing           # HIP events around each batch's sampling launches

    def _points_view(self, req):
        t = self.torch
        return self.buf[req.pts_off:req.pts_off + 12 * req.n].view(t.float32).view(req.n, 3)

    def _out_view(self, req):
        return self.buf[req.out_off:req.out_off + 4 * req.c].view(self.torch.int32)

    def launch(self, batch: Batch):
        torch, B = self.torch, self.B
        s = self.streams[self.next]
        self.next = (self.next + 1) % len(self.streams)
        reqs = batch.requests
        plan = None
        with torch.cuda.stream(s):
            for req in reqs:
                self._points_view(req).copy_(req.points, non_blocking=True)
            fps = [r for r in reqs if r.m == 1 and r.k is None]
            rest = [r for r in reqs if not (r.m == 1 and r.k is None)]
            ev0 = ev1 = None
            if self.timing:
                ev0 = torch.cuda.Event(enable_timing=True)
                ev0.record(s)
            sh = ctypes.c_void_p(s.cuda_stream)
            if rest:
                descs = (B.CloudDesc * len(rest))()
                for i, r in enumerate(rest):
                    descs[i] = B.CloudDesc(r.pts_off // 12, r.out_off // 4, r.n, r.c, r.m,
                                           -1 if r.k is None else r.k, r.start, 0)
                h = ctypes.c_void_p()
                B._check(self.L.afps_plan_create(ctypes.cast(descs, ctypes.c_void_p), len(rest),
                                                 ctypes.byref(h)))
                plan = h
                ws = ctypes.c_void_p(self.base + batch.ws_off)
                # the true size of the reserved block: the library refuses a
                # plan whose workspace would not fit in it
                B._check(self.L.afps_plan_upload(h, ws, batch.ws_bytes, sh))
                B._check(self.L.afps_plan_launch(h, ctypes.c_void_p(self.base),
                                                 ctypes.c_void_p(self.base), ws, sh))
            for r in fps:
                B._check(self.L.afps_fps_plain(ctypes.c_void_p(self.base + r.pts_off), r.n, r.c,
                                               r.start, ctypes.c_void_p(self.base + r.out_off), sh))
            if self.timing:
                ev1 = torch.cuda.Event(enable_timing=True)
                ev1.record(s)
            if self.on_launch is not None:
                self.on_launch(s, batch)
            for r in reqs:
                self._host_view(r).copy_(self._out_view(r), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, plan, ev0, ev1)

    def _host_view(self, req):
        return self.host[req.out_off:req.out_off + 4 * req.c].view(self.torch.int32)

    def done(self, handle) -> bool:
        return handle[0].query()

    def finish(self, batch: Batch):
        """The batch's event has fired: destroy its plan and return
        {rid: error} for the frames whose indices hold -1."""
        ev, plan, ev0, ev1 = batch.handle
        if ev0 is not None:
            batch.kernel_ms = ev0.elapsed_time(ev1)
        failed = {}
        for r in batch.requests:
            v = self._host_view(r).numpy()
            if v.size and int(v.min()) < 0:
                failed[r.rid] = "device-side failure: %d of %d indices are -1" % (int((v < 0).sum()), v.size)
            if self.keep:
                r.result = self.torch.from_numpy(v.copy())
        if plan is not None:
            self.L.afps_plan_destroy(plan)
        return failed


def latency_summary(finished):
    lat = np.array([r.latency for r in finished if r.state == "done"])
    if lat.size == 0:
        return {}
    done = [r for r in finished if r.state == "done"]
    span = max(r.done for r in done) - min(r.arrival for r in done)
    return {"frames": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3),
            "sampled_pts_per_s": float(sum(r.c for r in done) / span) if span > 0 else None,
            "frames_per_s": float(len(done) / span) if span > 0 else None,
            "rejected": sum(r.state == "rejected" for r in finished),
            "failed": sum(r.state == "failed" for r in finished)}
