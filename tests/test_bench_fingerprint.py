"""The walk's HBM traffic in the bench line comes from committed counter runs; it is
reported only while the walk kernel is the one those runs measured, identified by
its source and its compile flags."""

import bench
from paper_1106_1900_amd import build


def test_fingerprint_follows_source_and_flags(monkeypatch):
    h0 = bench.walk_source_hash()
    assert len(h0) == 16
    flags = dict(build.SOURCE_FLAGS)
    flags["walk.hip"] = list(flags.get("walk.hip", ())) + ["-DSOME_OTHER_SETTING=1"]
    monkeypatch.setattr(build, "SOURCE_FLAGS", flags)
    assert bench.walk_source_hash() != h0


def test_traffic_is_dropped_for_another_kernel(monkeypatch, tmp_path):
    # a counter file taken on another kernel version gives no traffic figure
    f = tmp_path / "traffic.json"
    f.write_text('{"walk_source_sha256_16": "0000000000000000", "bytes_per_launch": 123}')
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() is None
    f.write_text('{"walk_source_sha256_16": "%s", "bytes_per_launch": 123}' % bench.walk_source_hash())
    assert bench.measured_traffic() == 123
