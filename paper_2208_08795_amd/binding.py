"""Thin Python binding of libafps.so (include/afps.h): argument marshalling only.

Every function takes torch tensors on a HIP device, checks dtype / device /
shape / contiguity, and passes raw pointers and the current torch stream to
the C ABI.  All sampling runs in the library's kernels; there is no other
code path, and a missing library is an error.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafps.so")

_lock = threading.Lock()
_lib = None


class AfpsError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__("afps error %d (%s): %s" % (status, status_string(status), detail))
        self.status = status


class CloudDesc(ctypes.Structure):
    _fields_ = [("xyz_offset", ctypes.c_int64), ("out_offset", ctypes.c_int64),
                ("n", ctypes.c_int32), ("c", ctypes.c_int32), ("m", ctypes.c_int32),
                ("k", ctypes.c_int32), ("start", ctypes.c_int32), ("flags", ctypes.c_int32)]


def library_path() -> str:
    return LIB_PATH


def lib():
    """Load libafps.so (built in-tree by the package's build step)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libafps.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        # torch carries its own HIP runtime with the same soname as the
        # system one; loading torch first makes the library bind to that one
        # runtime, so tensors' device pointers and torch streams are valid in
        # both.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        i32, vp, sz = ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
        i32p = ctypes.POINTER(ctypes.c_int32)
        sig = {
            "afps_fps_plain": ([vp, i32, i32, i32, vp, vp], ctypes.c_int),
            "afps_afps": ([vp, i32, i32, i32, i32, vp, vp], ctypes.c_int),
            "afps_afps_npdu": ([vp, i32, i32, i32, i32, i32, vp, vp], ctypes.c_int),
            "afps_afps_npdu_ex": ([vp, i32, i32, i32, i32, i32, i32, vp, vp], ctypes.c_int),
            "afps_afps_variant": ([vp, i32, i32, i32, i32, i32, i32, vp, i32, i32, vp], ctypes.c_int),
            "afps_max_sector_points": ([], i32),
            "afps_plan_create": ([vp, i32, ctypes.POINTER(vp)], ctypes.c_int),
            "afps_plan_workspace_bytes": ([vp], sz),
            "afps_workspace_bytes_for_items": ([i32], sz),
            "afps_plan_upload": ([vp, vp, sz, vp], ctypes.c_int),
            "afps_plan_launch": ([vp, vp, vp, vp, vp], ctypes.c_int),
            "afps_plan_graph_launch": ([vp, vp, vp, vp, vp], ctypes.c_int),
            "afps_plan_launch_noalloc": ([vp, vp, vp, vp], ctypes.c_int),
            "afps_plan_launch_stamped": ([vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
            "afps_plan_status": ([vp, vp, vp], ctypes.c_int),
            "afps_device_status": ([vp, i32], ctypes.c_int),
            "afps_init": ([], ctypes.c_int),
            "afps_wall_clock_khz": ([], i32),
            "afps_tune_npdu": ([i32, i32, i32], ctypes.c_int),
            "afps_plan_rounds_workspace_bytes": ([vp, i32], sz),
            "afps_plan_launch_rounds": ([vp, vp, i32, vp, sz, vp], ctypes.c_int),
            "afps_npdu_xyz_in_lds": ([i32, i32], ctypes.c_int),
            "afps_tune_npdu_clear": ([], None),
            "afps_set_pool_policy": ([i32, i32, i32, i32], ctypes.c_int),
            "afps_noalloc_max_items": ([], i32),
            "afps_plan_items": ([vp], i32),
            "afps_plan_launches": ([vp], i32),
            "afps_plan_pool_waves": ([vp], i32),
            "afps_plan_pool_groups_per_cu": ([vp], i32),
            "afps_plan_destroy": ([vp], None),
            "afps_batched_workspace_bytes": ([vp, i32], sz),
            "afps_batched": ([vp, vp, i32, vp, vp, sz, vp], ctypes.c_int),
            "afps_tune_get": ([i32, i32, i32p, i32p], ctypes.c_int),
            "afps_tune_set": ([i32, i32, i32, i32], ctypes.c_int),
            "afps_tune_reset": ([], None),
            "afps_set_spin_limit": ([ctypes.c_uint32], ctypes.c_int),
            "afps_check_points": ([vp, ctypes.c_int64, vp], ctypes.c_int),
            "afps_bin_workspace_bytes": ([i32, i32], ctypes.c_size_t),
            "afps_bin_points": ([vp, i32, i32, i32, vp, vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
            "afps_set_checking": ([i32], ctypes.c_int),
            "afps_ball_query": ([vp, i32, vp, i32, ctypes.c_float, i32, i32, vp, vp, vp], ctypes.c_int),
            "afps_set_plan_occupancy": ([ctypes.c_float], ctypes.c_int),
            "afps_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "afps_last_error": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
        return L


def status_string(status: int) -> str:
    return lib().afps_status_string(status).decode()


def _check(status: int):
    if status != 0:
        raise AfpsError(status, lib().afps_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_points(xyz):
    torch = _torch()
    if not isinstance(xyz, torch.Tensor) or xyz.device.type != "cuda":
        raise TypeError("xyz must be a torch tensor on a HIP device")
    if xyz.dtype != torch.float32 or xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
        raise TypeError("xyz must be a contiguous float32 (N, 3) tensor")


def _used_on(stream, *tensors):
    """Tensors that the library's kernels read or write on an explicitly given
    stream: the caching allocator must not hand their memory to another tensor
    before that stream's queued work is done, even if the caller drops them
    first (they were allocated on, and are freed to, the current stream)."""
    if stream is None:
        return
    for t in tensors:
        if t is not None and t.is_cuda:
            t.record_stream(stream)


def _out(xyz, c, out):
    torch = _torch()
    if out is None:
        return torch.empty(c, dtype=torch.int32, device=xyz.device)
    if out.dtype != torch.int32 or out.device != xyz.device or not out.is_contiguous() or out.numel() < c:
        raise TypeError("out must be a contiguous int32 tensor of >= c entries on xyz's device")
    return out


def fps(xyz, c: int, start: int = 0, out=None, stream=None):
    """Plain FPS (Algorithm 1) -> int32 indices."""
    _check_points(xyz)
    out = _out(xyz, c, out)
    _used_on(stream, xyz, out)
    _check(lib().afps_fps_plain(ctypes.c_void_p(xyz.data_ptr()), xyz.shape[0], c, start,
                                ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def afps(xyz, c: int, m: int, start: int = 0, out=None, stream=None, variant=None):
    """AFPS with m sectors (Sec. III-B) -> int32 indices, sector-major.

    ``variant=(waves, slots)`` forces a kernel variant (autotuner, tests).
    """
    _check_points(xyz)
    out = _out(xyz, c, out)
    _used_on(stream, xyz, out)
    if variant is None:
        rc = lib().afps_afps(ctypes.c_void_p(xyz.data_ptr()), xyz.shape[0], c, m, start,
                             ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    else:
        rc = lib().afps_afps_variant(ctypes.c_void_p(xyz.data_ptr()), xyz.shape[0], c, m, -1, start, 0,
                                     ctypes.c_void_p(out.data_ptr()), variant[0], variant[1],
                                     _stream_handle(stream))
    _check(rc)
    return out


# NPDU readings other than the default (AFPS_NPDU_* in include/afps.h).
NPDU_FIRST_FULL, NPDU_SHIFT_EDGES, NPDU_K_WITH_SELF = 1, 2, 4


def afps_npdu(xyz, c: int, m: int, k: int, start: int = 0, out=None, stream=None, variant=None,
              flags: int = 0):
    """AFPS with NPDU window k (Sec. III-C) -> int32 indices, sector-major.
    ``flags`` selects the alternative readings (NPDU_*)."""
    _check_points(xyz)
    out = _out(xyz, c, out)
    _used_on(stream, xyz, out)
    if variant is None:
        rc = lib().afps_afps_npdu_ex(ctypes.c_void_p(xyz.data_ptr()), xyz.shape[0], c, m, k, start, flags,
                                     ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    else:
        rc = lib().afps_afps_variant(ctypes.c_void_p(xyz.data_ptr()), xyz.shape[0], c, m, k, start, flags,
                                     ctypes.c_void_p(out.data_ptr()), variant[0], variant[1],
                                     _stream_handle(stream))
    _check(rc)
    return out


def descriptors(sizes, cs, ms, ks, starts, flags=None):
    """Host descriptor array for clouds packed back to back (points and outputs)."""
    n = len(sizes)
    arr = (CloudDesc * n)()
    xo = oo = 0
    for i in range(n):
        arr[i] = CloudDesc(xo, oo, int(sizes[i]), int(cs[i]), int(ms[i]),
                           -1 if ks[i] is None else int(ks[i]), int(starts[i]),
                           0 if flags is None else int(flags[i]))
        xo += int(sizes[i])
        oo += int(cs[i])
    return arr, xo, oo


class BatchPlan:
    """A batch of clouds packed back to back in one (sum N, 3) tensor.

    Owns the device workspace (a torch tensor) and the library's plan.
    """

    def __init__(self, sizes, cs, ms, ks, starts, device="cuda", flags=None):
        torch = _torch()
        self.descs, self.total_points, self.total_samples = descriptors(sizes, cs, ms, ks, starts, flags)
        h = ctypes.c_void_p()
        _check(lib().afps_plan_create(ctypes.cast(self.descs, ctypes.c_void_p), len(sizes), ctypes.byref(h)))
        self._plan = h
        self.workspace_bytes = int(lib().afps_plan_workspace_bytes(h))
        self.items = int(lib().afps_plan_items(h))
        self.launches = int(lib().afps_plan_launches(h))
        self.pool_waves = int(lib().afps_plan_pool_waves(h))   # waves per workgroup of the NPDU launch
        self.pool_groups = int(lib().afps_plan_pool_groups_per_cu(h))   # its workgroups per CU
        self.workspace = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=device)
        self.offsets = [d.out_offset for d in self.descs]
        self._uploaded = False

    def upload(self, stream=None):
        _used_on(stream, self.workspace)
        _check(lib().afps_plan_upload(self._plan, ctypes.c_void_p(self.workspace.data_ptr()),
                                      self.workspace.numel(), _stream_handle(stream)))
        self._uploaded = True

    def _args(self, xyz_all, out_all, stream):
        _check_points(xyz_all)
        if xyz_all.shape[0] < self.total_points:
            raise ValueError("xyz_all holds fewer points than the plan's clouds")
        out_all = _out(xyz_all, self.total_samples, out_all)
        if not self._uploaded:
            # on the launch stream: a stream that does not wait for the current
            # one would otherwise read the workspace before the copy lands
            self.upload(stream)
        return out_all

    def launch(self, xyz_all, out_all=None, stream=None, graph=False):
        out_all = self._args(xyz_all, out_all, stream)
        _used_on(stream, xyz_all, out_all, self.workspace)
        f = lib().afps_plan_graph_launch if graph else lib().afps_plan_launch
        _check(f(self._plan, ctypes.c_void_p(xyz_all.data_ptr()), ctypes.c_void_p(out_all.data_ptr()),
                 ctypes.c_void_p(self.workspace.data_ptr()), _stream_handle(stream)))
        return out_all

    def launch_stamped(self, xyz_all, out_all=None, stream=None):
        """Eager launch that also records each NPDU sector's timestamps
        (afps_plan_launch_stamped); returns (out_all, stamps) with stamps an
        int64 (items, 8) tensor: take, loaded, end (shader clock), take_rt,
        end_rt (constant-rate clock), then (item, n) (c, k) (hw_id, xcc_id) as
        pairs of int32 packed in the last three columns."""
        torch = _torch()
        out_all = self._args(xyz_all, out_all, stream)
        stamps = torch.zeros((max(self.items, 1), 8), dtype=torch.int64, device=xyz_all.device)
        _used_on(stream, xyz_all, out_all, self.workspace, stamps)
        _check(lib().afps_plan_launch_stamped(self._plan, ctypes.c_void_p(xyz_all.data_ptr()),
                                              ctypes.c_void_p(out_all.data_ptr()),
                                              ctypes.c_void_p(self.workspace.data_ptr()),
                                              ctypes.c_void_p(stamps.data_ptr()), stamps.numel() * 8,
                                              _stream_handle(stream)))
        return out_all, stamps

    def round_table(self, rounds):
        """DEVICE table (int64 pairs) of the rounds' (xyz_all, out_all) for
        launch_rounds; the caller keeps the tensors alive while it is in use."""
        torch = _torch()
        rows = []
        for xyz_all, out_all in rounds:
            _check_points(xyz_all)
            if xyz_all.shape[0] < self.total_points:
                raise ValueError("a round's xyz_all holds fewer points than the plan's clouds")
            _out(xyz_all, self.total_samples, out_all)
            rows.append([xyz_all.data_ptr(), out_all.data_ptr()])
        return torch.tensor(rows, dtype=torch.int64).to(self.workspace.device)

    def launch_rounds(self, rounds, stream=None):
        """Run the batch once per round in one pooled launch
        (afps_plan_launch_rounds): `rounds` is a list of (xyz_all, out_all)
        pairs or a table from round_table()."""
        torch = _torch()
        table = rounds if isinstance(rounds, torch.Tensor) else self.round_table(rounds)
        count = int(table.shape[0])
        need = int(lib().afps_plan_rounds_workspace_bytes(self._plan, count))
        if need == 0:
            raise AfpsError(-2, "round count %d outside [1, 4096] or an empty plan" % count)
        if self.workspace.numel() < need:
            self.workspace = torch.empty(need, dtype=torch.uint8, device=self.workspace.device)
            self._uploaded = False
        if not self._uploaded:
            self.upload(stream)
        _used_on(stream, self.workspace, table)
        _check(lib().afps_plan_launch_rounds(self._plan, ctypes.c_void_p(table.data_ptr()), count,
                                             ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                             _stream_handle(stream)))
        return table

    def status(self, stream=None):
        """Raise AfpsError (AFPS_ERR_DEVICE) if a wave of the last launch gave
        up a bounded wait; waits for the stream."""
        _check(lib().afps_plan_status(self._plan, ctypes.c_void_p(self.workspace.data_ptr()),
                                      _stream_handle(stream)))

    def launch_noalloc(self, xyz_all, out_all=None, stream=None):
        """Launch with the library's static per-GPU workspace instead of the
        plan's own (afps_plan_launch_noalloc): no device allocation by the
        library; calls that overlap on one GPU race on that workspace."""
        _check_points(xyz_all)
        if xyz_all.shape[0] < self.total_points:
            raise ValueError("xyz_all holds fewer points than the plan's clouds")
        out_all = _out(xyz_all, self.total_samples, out_all)
        _used_on(stream, xyz_all, out_all)
        _check(lib().afps_plan_launch_noalloc(self._plan, ctypes.c_void_p(xyz_all.data_ptr()),
                                              ctypes.c_void_p(out_all.data_ptr()), _stream_handle(stream)))
        return out_all

    def split(self, out_all):
        """Per-cloud views of the packed output."""
        return [out_all[self.descs[i].out_offset:self.descs[i].out_offset + self.descs[i].c]
                for i in range(len(self.descs))]

    def close(self):
        if getattr(self, "_plan", None):
            lib().afps_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batched(clouds, cs, ms, ks, starts=None, graph=False, stream=None):
    """Sample a list of (N_i, 3) device tensors in one batch plan; returns
    per-cloud indices, ready on the current stream.  With `stream`, the launch
    runs there after the current stream's pending work (the packed input is
    written on the current stream)."""
    torch = _torch()
    starts = starts or [0] * len(clouds)
    plan = BatchPlan([c.shape[0] for c in clouds], cs, ms, ks, starts, device=clouds[0].device)
    xyz_all = torch.cat(list(clouds), dim=0).contiguous()
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream())
    out = plan.launch(xyz_all, stream=stream, graph=graph)
    if stream is not None:
        torch.cuda.current_stream().wait_stream(stream)
    res = [o.clone() for o in plan.split(out)]
    # the plan's graph and events may still be in use on the launch stream
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()
    plan.close()
    return res


def batched_oneshot(xyz_all, sizes, cs, ms, ks, starts, out_all=None, stream=None, flags=None):
    """afps_batched: plan, upload and launch in one call on host descriptors
    for clouds packed back to back in xyz_all; returns the packed indices."""
    torch = _torch()
    _check_points(xyz_all)
    descs, total_points, total_samples = descriptors(sizes, cs, ms, ks, starts, flags)
    if xyz_all.shape[0] < total_points:
        raise ValueError("xyz_all holds fewer points than the clouds")
    out_all = _out(xyz_all, total_samples, out_all)
    need = int(lib().afps_batched_workspace_bytes(ctypes.cast(descs, ctypes.c_void_p), len(sizes)))
    if need == 0 and len(sizes) > 0:
        raise AfpsError(-2, lib().afps_last_error().decode())
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=xyz_all.device)
    _used_on(stream, xyz_all, out_all, ws)
    _check(lib().afps_batched(ctypes.c_void_p(xyz_all.data_ptr()), ctypes.cast(descs, ctypes.c_void_p), len(sizes),
                              ctypes.c_void_p(out_all.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                              _stream_handle(stream)))
    return out_all


def device_status(stream=None):
    """Raise AfpsError (AFPS_ERR_DEVICE) if a kernel on the current device has
    given up a bounded wait since the record was last cleared."""
    _check(lib().afps_device_status(_stream_handle(stream), 0))


def clear_device_status(stream=None) -> bool:
    """Clear the device's failure record; True if a failure was recorded."""
    rc = lib().afps_device_status(_stream_handle(stream), 1)
    if rc not in (0, -7):
        _check(rc)
    return rc == -7


def init():
    """Set up the library's state on the current device."""
    _check(lib().afps_init())


def workspace_bytes_for_items(items: int) -> int:
    """Device workspace of a batch plan with `items` sectors in total."""
    return int(lib().afps_workspace_bytes_for_items(items))


def set_plan_occupancy(waves_per_simd: float):
    _check(lib().afps_set_plan_occupancy(waves_per_simd))


def set_spin_limit(polls: int):
    _check(lib().afps_set_spin_limit(polls))


def check_points(xyz, stream=None):
    """Input check of one cloud (waits for the stream): raises AfpsError
    (AFPS_ERR_DATA) if a coordinate is not finite or the squared bounding-box
    diagonal is not below 1e10."""
    _check_points(xyz)
    _check(lib().afps_check_points(ctypes.c_void_p(xyz.data_ptr()), xyz.shape[0], _stream_handle(stream)))


def bin_points(xyz, axis: int, bins: int, with_points: bool = True, stream=None):
    """Binning along one axis (Sec. III-A): returns (perm, binned points or
    None); perm[i] is the storage index of the i-th point in binned order."""
    torch = _torch()
    _check_points(xyz)
    n = xyz.shape[0]
    need = int(lib().afps_bin_workspace_bytes(n, bins))
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=xyz.device)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=xyz.device)
    out = torch.empty_like(xyz) if with_points else None
    _used_on(stream, xyz, ws, perm, out)
    _check(lib().afps_bin_points(ctypes.c_void_p(xyz.data_ptr()), n, axis, bins, ctypes.c_void_p(perm.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()) if out is not None else None,
                                 ctypes.c_void_p(ws.data_ptr()), need, _stream_handle(stream)))
    return perm[:n], out


def ball_query(xyz, centers, radius: float, k: int, window: int | None = None, out=None, counts=None,
               stream=None):
    """Grouping around the samples (ball query; see afps_ball_query): returns
    (idx int32 (C, k), count int32 (C,)) for the int32 centre indices
    ``centers``; ``window`` bounds the candidates to storage positions within
    ``window`` of each centre (None: the whole cloud)."""
    torch = _torch()
    _check_points(xyz)
    if centers.dtype != torch.int32 or not centers.is_contiguous() or centers.device != xyz.device:
        raise ValueError("centers must be a contiguous int32 tensor on the points' device")
    c = centers.shape[0]
    if out is None:
        out = torch.empty((c, k), dtype=torch.int32, device=xyz.device)
    if counts is None:
        counts = torch.empty(c, dtype=torch.int32, device=xyz.device)
    if out.shape != (c, k) or out.dtype != torch.int32 or not out.is_contiguous() or out.device != xyz.device:
        raise ValueError("out must be a contiguous int32 (C, k) tensor on the points' device")
    if (counts.shape != (c,) or counts.dtype != torch.int32 or not counts.is_contiguous()
            or counts.device != xyz.device):
        raise ValueError("counts must be a contiguous int32 (C,) tensor on the points' device")
    _used_on(stream, xyz, centers, out, counts)
    _check(lib().afps_ball_query(ctypes.c_void_p(xyz.data_ptr()), xyz.shape[0], ctypes.c_void_p(centers.data_ptr()),
                                 c, float(radius), int(k), -1 if window is None else int(window),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(counts.data_ptr()),
                                 _stream_handle(stream)))
    return out, counts


def set_checking(on: bool):
    """Check every cloud's preconditions before each sampling call."""
    _check(lib().afps_set_checking(1 if on else 0))


TUNE_DIRECT, TUNE_NPDU, TUNE_BATCH = 0, 1, 2


def tune_get(n_s: int, kind: int = TUNE_DIRECT):
    w, s = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().afps_tune_get(n_s, kind, ctypes.byref(w), ctypes.byref(s)))
    return w.value, s.value


def tune_set(n_s_max: int, waves: int, slots: int, kind: int = TUNE_DIRECT):
    _check(lib().afps_tune_set(n_s_max, kind, waves, slots))


def tune_reset():
    lib().afps_tune_reset()


def tune_npdu(n_s_max: int, k_max: int, xyz_in_lds: bool):
    """Coordinates of NPDU sectors of at most n_s_max points (windows k <= k_max)
    in LDS or read from L2, for batch plans created afterwards."""
    _check(lib().afps_tune_npdu(n_s_max, k_max, 1 if xyz_in_lds else 0))


def tune_npdu_clear():
    """Forget the NPDU placement and pool policy (full-update tuning stays)."""
    lib().afps_tune_npdu_clear()


def npdu_xyz_in_lds(n_s: int, k: int) -> bool:
    return bool(lib().afps_npdu_xyz_in_lds(n_s, k))


def set_pool_policy(waves: int = 0, groups: int = 0, seed_sleep: bool = True, seed_priority: int = 3):
    """Shape and seeding of the pooled NPDU launch of batch plans created afterwards."""
    _check(lib().afps_set_pool_policy(waves, groups, 1 if seed_sleep else 0, seed_priority))
