"""Host-side accounting of bench.py: algorithmic bytes and the counter-based traffic."""
import bench


def test_algorithmic_bytes_per_site():
    # per site of the doubled lattice: FP64 384 B per RHS + 576 shared, FP32 192 + 256, BF16 links 192 + 208,
    # plus half a per-RHS figure for every extra epilogue vector
    assert bench.algorithmic_bytes(0, 1, 1, 1) == 960
    assert bench.algorithmic_bytes(1, 1, 1, 1) == 448
    assert bench.algorithmic_bytes(2, 1, 1, 1) == 400
    assert bench.algorithmic_bytes(2, 10, 1, 4, 8) == 10 * (192 * 4 + 208 + 96 * 8)
    # shared bytes count once per launch
    assert bench.algorithmic_bytes(1, 1, 2, 8) == 192 * 8 + 2 * 256


def test_measured_traffic_reads_the_launch_and_checks_the_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.md"
    f.write_text("text\n```\nsource_sha256: %s\ntraffic bf16 16 1600\ntraffic bf16 12 1200\n"
                 "traffic fp64 12 5000\n```\n" % bench.apply_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(f))
    assert bench.measured_traffic("bf16", 16) == 1600
    assert bench.measured_traffic("bf16", 12) == 1200
    assert bench.measured_traffic("bf16", 14) is None  # no line for this launch width
    assert bench.measured_traffic("fp32", 12) is None
    f.write_text("source_sha256: 0000000000000000\ntraffic bf16 16 1600\n")
    assert bench.measured_traffic("bf16", 16) is None  # counters taken on other kernel sources
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("bf16", 16) is None
