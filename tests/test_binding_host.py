"""Host logic of the Python binding that needs no GPU: which stream a batch
plan's workspace upload is ordered on (a recording stand-in replaces the
library; nothing is launched)."""
import ctypes
import types

import pytest
import torch

from paper_2208_08795_amd import binding


class _RecordingLib:
    def __init__(self):
        self.calls = []

    def afps_plan_create(self, descs, n, handle):
        return 0

    def afps_plan_workspace_bytes(self, h):
        return 4096

    def afps_plan_items(self, h):
        return 1

    def afps_plan_launches(self, h):
        return 1

    def afps_plan_pool_waves(self, h):
        return 4

    def afps_plan_pool_groups_per_cu(self, h):
        return 1

    def afps_plan_upload(self, h, ws, nbytes, stream):
        self.calls.append(("upload", stream.value))
        return 0

    def afps_plan_launch(self, h, xyz, out, ws, stream):
        self.calls.append(("launch", stream.value))
        return 0

    def afps_plan_graph_launch(self, h, xyz, out, ws, stream):
        self.calls.append(("graph", stream.value))
        return 0

    def afps_plan_destroy(self, h):
        return None


@pytest.fixture
def fake(monkeypatch):
    rec = _RecordingLib()
    monkeypatch.setattr(binding, "lib", lambda: rec)
    monkeypatch.setattr(binding, "_check_points", lambda xyz: None)
    return rec


@pytest.mark.parametrize("graph", [False, True])
def test_first_launch_uploads_on_its_own_stream(fake, graph):
    """The first launch uploads the workspace on the launch stream, so a
    stream that does not wait for the current one never reads it early;
    later launches, on any stream, do not upload again."""
    plan = binding.BatchPlan([10], [4], [1], [None], [0], device="cpu")
    xyz = torch.zeros(10, 3)
    out = torch.empty(4, dtype=torch.int32)
    side, other = types.SimpleNamespace(cuda_stream=0x5100), types.SimpleNamespace(cuda_stream=0x5200)
    plan.launch(xyz, out_all=out, stream=side, graph=graph)
    plan.launch(xyz, out_all=out, stream=other, graph=graph)
    kind = "graph" if graph else "launch"
    assert fake.calls == [("upload", 0x5100), (kind, 0x5100), (kind, 0x5200)]
    plan.close()


def test_explicit_upload_is_not_repeated(fake):
    plan = binding.BatchPlan([10], [4], [1], [None], [0], device="cpu")
    side = types.SimpleNamespace(cuda_stream=0x5300)
    plan.upload(side)
    plan.launch(torch.zeros(10, 3), out_all=torch.empty(4, dtype=torch.int32), stream=side)
    assert fake.calls == [("upload", 0x5300), ("launch", 0x5300)]
    plan.close()


def test_ball_query_rejects_mis_sized_outputs(monkeypatch):
    """Caller-supplied outputs of the wrong shape, type or device are refused
    before anything is launched (a short counts tensor would be written past
    its end)."""
    monkeypatch.setattr(binding, "_check_points", lambda xyz: None)
    monkeypatch.setattr(binding, "lib", lambda: pytest.fail("nothing may reach the library"))
    xyz = torch.zeros(10, 3)
    centers = torch.zeros(4, dtype=torch.int32)
    good_out, good_cnt = torch.empty(4, 8, dtype=torch.int32), torch.empty(4, dtype=torch.int32)
    for out, cnt in [(torch.empty(4, 7, dtype=torch.int32), good_cnt),
                     (torch.empty(4, 8, dtype=torch.int64), good_cnt),
                     (good_out, torch.empty(3, dtype=torch.int32)),
                     (good_out, torch.empty(4, dtype=torch.float32)),
                     (good_out, torch.empty(8, dtype=torch.int32)[::2])]:
        with pytest.raises(ValueError):
            binding.ball_query(xyz, centers, 0.5, 8, out=out, counts=cnt)
