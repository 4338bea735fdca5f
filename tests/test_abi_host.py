"""The C-ABI library loads, exports every function include/afps.h declares, and
rejects bad arguments on the host before touching a GPU (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afps.h")


@pytest.fixture(scope="module")
def L():
    from paper_2208_08795_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2208_08795_amd import build_lib
        build_lib.build()
    return binding.lib()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(afps_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_function(L):
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name


def test_status_strings(L):
    from paper_2208_08795_amd import binding
    for st in range(0, -9, -1):
        assert binding.status_string(st) not in ("", "unknown status")
    assert binding.status_string(-99) == "unknown status"


def test_host_validation_without_gpu(L):
    from paper_2208_08795_amd import binding
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: validation rejects first
    assert L.afps_afps(None, 10, 5, 1, 0, dummy, None) == -1
    assert L.afps_afps(dummy, 10, 5, 1, 0, None, None) == -1
    assert L.afps_afps(dummy, 10, 11, 1, 0, dummy, None) == -2     # c > n
    assert L.afps_afps(dummy, 10, 5, 6, 0, dummy, None) == -2      # m > c
    assert L.afps_afps(dummy, 10, 5, 0, 0, dummy, None) == -2      # m < 1
    assert L.afps_afps(dummy, 10, 5, 2, 10, dummy, None) == -3     # start >= n
    assert L.afps_afps(dummy, 10, 5, 2, -1, dummy, None) == -3
    assert L.afps_afps_npdu(dummy, 10, 5, 2, -1, 0, dummy, None) == -2   # k < 0
    assert L.afps_fps_plain(dummy, 0, 0, 0, dummy, None) == -2
    assert "1 <= m <= c <= n" in L.afps_last_error().decode()
    assert L.afps_set_spin_limit(0) == -2
    assert L.afps_check_points(None, 10, None) == -1
    assert L.afps_check_points(dummy, -1, None) == -2
    assert L.afps_check_points(dummy, 0, None) == 0          # empty cloud: nothing to read
    assert L.afps_set_checking(0) == 0
    # binning: sizes and arguments checked on the host
    assert L.afps_bin_workspace_bytes(0, 16) == 0 and L.afps_bin_workspace_bytes(10, 0) == 0
    assert L.afps_bin_workspace_bytes(10, 8193) == 0
    assert L.afps_bin_workspace_bytes(8192, 1024) == 256 + 1024 * 4 + 8 * 1024 * 4   # 8 chunks of 1024 points
    assert L.afps_bin_points(None, 10, 0, 4, dummy, None, dummy, 1 << 20, None) == -1
    assert L.afps_bin_points(dummy, 10, 3, 4, dummy, None, dummy, 1 << 20, None) == -2
    assert L.afps_bin_points(dummy, 10, 0, 9000, dummy, None, dummy, 1 << 20, None) == -2
    assert L.afps_bin_points(dummy, 10, 0, 4, dummy, dummy, dummy, 1 << 20, None) == -2   # xyz_out == xyz
    assert L.afps_bin_points(dummy, 10, 0, 4, dummy, None, dummy, 100, None) == -4
    # NPDU reading flags: unknown bits, k counting the sample with k = 0
    assert L.afps_afps_npdu_ex(dummy, 10, 5, 1, 3, 0, 8, dummy, None) == -2
    assert L.afps_afps_npdu_ex(dummy, 10, 5, 1, 0, 0, 4, dummy, None) == -2
    assert "counts the sample" in L.afps_last_error().decode()
    fl, _, _ = binding.descriptors([100, 50], [10, 20], [2, 1], [4, None], [0, 0], flags=[1, 2])
    fplan = ctypes.c_void_p()
    assert L.afps_plan_create(ctypes.cast(fl, ctypes.c_void_p), 2, ctypes.byref(fplan)) == -2
    assert "descriptor 1" in L.afps_last_error().decode()
    # bad descriptors are rejected before any device work
    descs, _, _ = binding.descriptors([100, 50], [10, 60], [2, 1], [None, 4], [0, 0])
    plan = ctypes.c_void_p()
    assert L.afps_plan_create(ctypes.cast(descs, ctypes.c_void_p), 2, ctypes.byref(plan)) == -2
    assert "descriptor 1" in L.afps_last_error().decode()
    assert L.afps_tune_set(100, 0, 3, 5) == -2   # no such variant
    assert L.afps_tune_set(100, 1, 1, 1) == -2   # NPDU is not tuned
    assert L.afps_tune_set(100, 0, 1, 1) == -2   # 64 points: too small for 100
    assert L.afps_max_sector_points() == 32768
    # plan calls without a plan, stamps or workspace are rejected on the host
    assert L.afps_plan_launch_noalloc(None, dummy, dummy, None) == -1
    assert L.afps_plan_status(None, dummy, None) == -1
    assert L.afps_plan_launch_stamped(None, dummy, dummy, dummy, dummy, 64, None) == -1
    # the no-alloc entry point takes plans whose workspace fits its 1 MiB scratch:
    # 256 B of counters, 512 pooled workgroups (8 B each) and their seeds (16
    # waves of 8 B), then 40 B per work item and at most one 16 B queue per item
    header = 256 + 512 * 8 + 512 * 16 * 8
    L.afps_workspace_bytes_for_items.restype = ctypes.c_size_t
    L.afps_workspace_bytes_for_items.argtypes = [ctypes.c_int32]
    assert L.afps_workspace_bytes_for_items(1) == (header + 40 + 8 + 16 + 255) // 256 * 256
    cap = L.afps_noalloc_max_items()
    assert L.afps_workspace_bytes_for_items(cap) <= 1 << 20 < L.afps_workspace_bytes_for_items(cap + 1)
    assert cap == ((1 << 20) - header) // 56
    # grouping: arguments checked on the host; no centres launches nothing
    assert L.afps_ball_query(None, 10, dummy, 4, 1.0, 8, -1, dummy, None, None) == -1
    assert L.afps_ball_query(dummy, 10, None, 4, 1.0, 8, -1, dummy, None, None) == -1
    assert L.afps_ball_query(dummy, 0, dummy, 4, 1.0, 8, -1, dummy, None, None) == -2
    assert L.afps_ball_query(dummy, 10, dummy, 4, 1.0, 0, -1, dummy, None, None) == -2
    assert L.afps_ball_query(dummy, 10, dummy, 4, -1.0, 8, -1, dummy, None, None) == -2
    assert L.afps_ball_query(dummy, 10, dummy, 4, float("nan"), 8, -1, dummy, None, None) == -2
    assert L.afps_ball_query(dummy, 10, dummy, -1, 1.0, 8, -1, dummy, None, None) == -2
    assert L.afps_ball_query(dummy, 10, dummy, 0, 1.0, 8, -1, dummy, None, None) == 0


def test_descriptor_layout():
    from paper_2208_08795_amd import binding
    assert ctypes.sizeof(binding.CloudDesc) == 40
    arr, tp, ts = binding.descriptors([5, 7], [2, 3], [1, 1], [None, 2], [0, 1])
    assert (arr[1].xyz_offset, arr[1].out_offset, arr[0].k, arr[1].k) == (5, 2, -1, 2)
    assert (tp, ts) == (12, 5)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2208_08795_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        binding.lib()


def test_tune_tables_round_trip(L):
    from paper_2208_08795_amd import binding
    binding.tune_reset()
    rule = binding.tune_get(3000, binding.TUNE_DIRECT)
    assert 64 * rule[0] * rule[1] >= 3000
    binding.tune_set(4096, 16, 4, binding.TUNE_DIRECT)
    binding.tune_set(4096, 2, 32, binding.TUNE_BATCH)
    assert binding.tune_get(3000, binding.TUNE_DIRECT) == (16, 4)
    assert binding.tune_get(3000, binding.TUNE_BATCH) == (2, 32)
    assert binding.tune_get(5000, binding.TUNE_DIRECT) == binding.tune_get(5000, binding.TUNE_DIRECT)
    assert binding.tune_get(3000, binding.TUNE_NPDU) == (1, 1)
    binding.tune_reset()
    assert binding.tune_get(3000, binding.TUNE_DIRECT) == rule


def test_autotune_candidates_hold_the_class():
    from paper_2208_08795_amd.autotune import CLASSES, candidates
    for n in CLASSES:
        cands = candidates(n)
        assert cands, n
        assert all(64 * w * p >= n for w, p in cands)
    assert (1, 1) in candidates(64) and (16, 32) in candidates(32768)
