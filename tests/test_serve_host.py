"""Serving scheduler on the CPU: a fake executor and a fake clock check
admission by footprint, FIFO order, slot reuse, rejection and launch failure."""
import random

from paper_2208_08795_amd.serve import ALIGN, Arena, Request, Scheduler, footprint, library_workspace_bytes


class FakeClock:
    def __init__(self, dt=1e-4):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


class FakeExecutor:
    """A batch takes 1 ms per frame; launches of frames in fail_ids raise;
    frames in device_fail_ids complete with a device-side failure."""

    def __init__(self, clock, fail_ids=(), device_fail_ids=()):
        self.clock, self.fail_ids = clock, set(fail_ids)
        self.device_fail_ids = set(device_fail_ids)
        self.launched = []
        self.live_bytes = []

    def launch(self, batch):
        if any(r.rid in self.fail_ids for r in batch.requests):
            raise RuntimeError("forced launch failure")
        # the reserved workspace block holds the plan the library would build
        items = sum(r.m for r in batch.requests)
        assert batch.ws_bytes >= library_workspace_bytes(items), (batch.ws_bytes, items)
        self.launched.append([r.rid for r in batch.requests])
        return self.clock.t + 1e-3 * len(batch.requests)

    def done(self, handle):
        return self.clock.t >= handle

    def finish(self, batch):
        return {r.rid: "device-side failure: -1 indices" for r in batch.requests if r.rid in self.device_fail_ids}


def _req(i, n, arrival, m=8, k=64):
    return Request(rid=i, n=n, c=n // 8, m=m, k=k, start=0, arrival=arrival)


def test_arena_first_fit_and_coalescing():
    a = Arena(10 * ALIGN)
    x = a.alloc(1)
    y = a.alloc(2 * ALIGN)
    z = a.alloc(ALIGN + 1)
    assert (x, y, z) == (0, ALIGN, 3 * ALIGN)
    assert a.alloc(6 * ALIGN) is None and a.alloc(5 * ALIGN) == 5 * ALIGN
    a.free(y)
    a.free(x)
    assert a.free_list[0] == (0, 3 * ALIGN)        # coalesced
    a.free(z)
    assert a.free_list[0] == (0, 5 * ALIGN)
    assert all(off % 12 == 0 and off % 256 == 0 for off in (x, y, z))


def test_admission_never_exceeds_budget_and_all_finish():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    budget = 3 * 1024 * 1024
    s = Scheduler(ex, budget, max_inflight=3, max_batch=4, clock=clock)
    rng = random.Random(0)
    reqs = [_req(i, rng.randint(16384, 131072), 0.0005 * i) for i in range(60)]
    done = s.run(reqs)
    assert len(done) == 60 and all(r.state == "done" for r in done)
    assert s.peak_bytes <= s.arena.size
    assert s.arena.bytes_used == 0 and s.arena.free_list == [(0, s.arena.size)]
    # FIFO: admission order equals arrival order
    order = [rid for b in ex.launched for rid in b]
    assert order == sorted(order)
    # continuous batching: some batch held more than one frame, and work overlapped
    assert max(len(b) for b in ex.launched) > 1
    assert all(r.latency > 0 for r in done)


def test_oversized_frame_is_rejected_and_loop_continues():
    clock = FakeClock()
    s = Scheduler(FakeExecutor(clock), 1 << 20, clock=clock)
    reqs = [_req(0, 20000, 0.0), _req(1, 200000, 0.0), _req(2, 30000, 0.001)]
    done = {r.rid: r for r in s.run(reqs)}
    assert done[1].state == "rejected" and "budget" in done[1].error
    assert done[0].state == "done" and done[2].state == "done"


def test_launch_failure_frees_memory_and_others_complete():
    clock = FakeClock()
    s = Scheduler(FakeExecutor(clock, fail_ids={3}), 8 << 20, max_batch=1, clock=clock)
    reqs = [_req(i, 50000, 0.0002 * i) for i in range(8)]
    done = {r.rid: r for r in s.run(reqs)}
    assert done[3].state == "failed" and "forced" in done[3].error
    assert all(done[i].state == "done" for i in range(8) if i != 3)
    assert s.arena.bytes_used == 0


def test_slots_are_reused_under_a_small_budget():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    blocks = list(footprint(_req(0, 60000, 0))) + [library_workspace_bytes(8)]
    one = sum(-(-x // ALIGN) * ALIGN for x in blocks)
    s = Scheduler(ex, one + ALIGN, max_inflight=4, clock=clock)   # room for one frame at a time
    reqs = [_req(i, 60000, 0.0) for i in range(5)]
    done = s.run(reqs)
    assert all(r.state == "done" for r in done)
    assert all(len(b) == 1 for b in ex.launched) and len(ex.launched) == 5
    assert s.peak_waiting >= 4


def test_workspace_block_covers_large_batches():
    """Regression: the workspace block reserved for a batch must hold the
    library's item table (40-byte items) for every sector of every frame,
    also for batches of many 32-sector frames."""
    clock = FakeClock()
    ex = FakeExecutor(clock)
    s = Scheduler(ex, 64 << 20, max_inflight=2, max_batch=32, clock=clock)
    reqs = [_req(i, 20000, 0.0, m=32) for i in range(64)]
    done = s.run(reqs)
    assert all(r.state == "done" for r in done)
    assert max(len(b) for b in ex.launched) >= 16
    assert library_workspace_bytes(32 * 16) > 256 + 32 * 32 * 16     # 40 bytes per sector


def test_device_side_failure_marks_only_its_frames_failed():
    clock = FakeClock()
    s = Scheduler(FakeExecutor(clock, device_fail_ids={2, 5}), 16 << 20, max_batch=3, clock=clock)
    reqs = [_req(i, 40000, 0.0003 * i) for i in range(9)]
    done = {r.rid: r for r in s.run(reqs)}
    assert {i for i, r in done.items() if r.state == "failed"} == {2, 5}
    assert all("-1" in done[i].error for i in (2, 5))
    assert all(done[i].state == "done" for i in range(9) if i not in (2, 5))
    assert s.arena.bytes_used == 0
    from paper_2208_08795_amd.serve import latency_summary
    summ = latency_summary(list(done.values()))
    assert summ["failed"] == 2 and summ["frames"] == 7


def test_time_window_stops_admission_and_reports_the_queue():
    """A window shorter than the stream: frames still waiting are reported
    (count and the oldest one's wait), frames on the device complete, frames
    that had not arrived are dropped."""
    clock = FakeClock(dt=1e-4)
    ex = FakeExecutor(clock)
    s = Scheduler(ex, 4 << 20, max_inflight=1, max_batch=1, clock=clock)
    reqs = [_req(i, 60000, 0.0005 * i) for i in range(200)]     # 1 ms of work each, arriving every 0.5 ms
    done = s.run(reqs, window=0.05)
    assert all(r.state == "done" for r in done)
    assert 20 <= len(done) <= 60
    assert s.left_waiting > 10 and s.oldest_wait_s > 0.01
    assert not s.inflight and len(s.waiting) == s.left_waiting
