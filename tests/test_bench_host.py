"""Host logic of bench.py that needs no GPU: the algorithmic counts behind the
roofline (pinned on hand cases), the counter record used only while the
kernel sources still match the hash it was taken with, the device-stamp
reduction, and the host and clock readers."""
import hashlib
import json
import os

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORD = os.path.join(ROOT, "profiles", "pooled_npdu_kernel_batch256_counters.json")


def test_npdu_counts_by_hand():
    # one sector of 10 points, k = 2 (window [cur-1, cur+1]), picks 0, 2, 4, 9
    # (the first pick is the start): the updates of iterations 1..3 use the
    # windows of picks 0, 2 and 4: [0,1] (2 points), [1,3] (3), [3,5] (3)
    out = np.array([0, 2, 4, 9], dtype=np.int32)
    c = bench.npdu_counts([10], [4], out, [0], 1, 2)
    assert c["updates"] == 8 and c["iterations"] == 3
    assert c["ops"] == 9 * 8 + 3 * (2 + 1) + 3 * 1           # window + one 64-point block per iteration
    assert c["alg1_scan_ops"] == 9 * 8 + 3 * 10
    # LDS-record updates: sectors of more points than the register bound
    assert bench.npdu_counts([10], [4], out, [0], 1, 2, records_above=9)["updates_records"] == 8
    assert bench.npdu_counts([10], [4], out, [0], 1, 2, records_above=10)["updates_records"] == 0
    assert c["updates_records"] == 0
    # two sectors of 70 and 69 points (M = 2, N = 139), two samples each: one
    # iteration per sector, two blocks in the first, two in the second
    out = np.array([0, 35, 70, 100], dtype=np.int32)
    c = bench.npdu_counts([139], [4], out, [0], 2, 4)
    assert c["iterations"] == 2 and c["updates"] == 3 + 3      # windows [0,2] and [0,2] (local)
    assert c["ops"] == 9 * 6 + 2 * 5 + 2 + 2


def test_fps_ops():
    ops, upd = bench.fps_ops([100, 10], [5, 1])
    assert upd == 4 * 100 and ops == 10 * 400


def test_counter_record_follows_the_source_hash():
    if not os.path.exists(RECORD):
        assert bench.counter_record("pooled_npdu_kernel<16>, coordinates out of LDS up to 4096") is None
        return
    with open(RECORD) as f:
        rec = json.load(f)
    src = "".join(open(os.path.join(ROOT, s)).read() for s in rec["sources"])
    current = hashlib.sha256(src.encode()).hexdigest() == rec["source_sha256"]
    for name, entry in rec["kernels"].items():
        got = bench.counter_record(name)
        assert (got == entry) if current else got is None, name
        want = (entry["fetch_kib_per_round"] * entry["fetch_scale"] +
                entry["write_kib_per_round"] * entry["write_scale"]) * 1024
        assert abs(entry["traffic_bytes_per_round"] - want) <= 0.002 * want + 2048, name
    assert bench.counter_record("no such kernel") is None


def test_stamp_cycles_reduction():
    import torch
    # two sectors: 101 samples over 10 000 cycles after load, and 11 over 2 000;
    # constant-rate counter at 100 MHz advancing 1/20 as fast (a 2 GHz clock)
    rows = []
    for item, (n, c, take, loaded, end) in enumerate([(4096, 101, 0, 600, 10600), (1000, 11, 100, 300, 2300)]):
        pairs = np.array([item, n, c, 32, 0, 0], dtype=np.int32).view(np.int64)
        rows.append([take, loaded, end, take // 20, end // 20] + list(pairs))
    # the second sector ran on another XCD whose shader clock reads far ahead
    rows[1][:3] = [v + 10 ** 9 for v in rows[1][:3]]
    st = torch.tensor(rows, dtype=torch.int64)
    r = bench.stamp_cycles(st, 100000)
    assert r["median"] == 150.0 and r["sclk_ghz"] == 2.0
    assert r["critical_sector"]["points"] == 4096 and r["critical_sector"]["cycles_per_iteration"] == 100.0
    assert r["critical_sector"]["load_us"] == 0.3
    assert r["critical_sector"]["ends_at_us"] == 5.3     # on the constant-rate counter: 530 ticks at 100 MHz


def test_host_readers_return_plain_values():
    model = bench.host_cpu_model()
    assert model is None or (isinstance(model, str) and model)
    model = bench.lscpu_model()
    assert model is None or (isinstance(model, str) and model)
    clocks = bench.shader_clock_mhz()
    assert clocks is None or all(isinstance(c, int) and c > 0 for c in clocks)
