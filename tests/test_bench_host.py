"""Host logic of bench.py that needs no GPU: the HBM traffic record is used
only while the kernel and plan sources still match the hash it was taken
with, and the host and clock readers return plain values."""
import hashlib
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORD = os.path.join(ROOT, "profiles", "pooled_npdu_kernel_batch256_traffic.json")


def test_traffic_record_follows_the_source_hash():
    with open(RECORD) as f:
        rec = json.load(f)
    src = "".join(open(os.path.join(ROOT, s)).read() for s in rec["sources"])
    current = hashlib.sha256(src.encode()).hexdigest() == rec["source_sha256"]
    for name, entry in rec["kernels"].items():
        got = bench.counter_traffic(name)
        assert got == (entry["traffic_bytes_per_launch"] if current else None), name
        # scaled FETCH + WRITE bytes, as the record states them
        want = (entry["fetch_kib_per_launch"] * entry["fetch_scale"] +
                entry["write_kib_per_launch"] * entry["write_scale"]) * 1024
        assert abs(entry["traffic_bytes_per_launch"] - want) <= 0.002 * want + 2048, name
    assert bench.counter_traffic("no such kernel") is None


def test_host_readers_return_plain_values():
    model = bench.host_cpu_model()
    assert model is None or (isinstance(model, str) and model)
    clocks = bench.shader_clock_mhz()
    assert clocks is None or all(isinstance(c, int) and c > 0 for c in clocks)
