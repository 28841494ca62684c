"""Host-side checks of the benchmark's contract (no GPU): the one-GPU rule,
the roofline constants, and the traffic records it reports."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_fp32_lane_peak_from_unit_counts():
    # 256 compute units x 4 SIMDs x 16 lanes x 2.4 GHz, in T op/s
    assert bench.VALU_PEAK_TOPS == pytest.approx(39.3216)
    # eq. (1): 3 adds, 3 medians, 3 scalings per PE (sign products are
    # bitwise and not counted against the FP32 lanes)
    assert bench.OPS_PER_PE == 9


def test_every_traffic_record_names_existing_sources():
    for name, (record, srcs) in bench.TRAFFIC_RECORDS.items():
        assert record.startswith("traffic_") and record.endswith(".txt")
        for src in srcs:
            assert os.path.isfile(src), (name, src)


def test_traffic_is_reported_only_while_the_sources_match(tmp_path,
                                                          monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel v1\n")
    rec = tmp_path / "traffic_test.txt"
    monkeypatch.setitem(bench.TRAFFIC_RECORDS, "t", (str(rec), [str(src)]))
    digest = bench.source_digest([str(src)])
    rec.write_text(f"# summary\n@source_sha256_16 = {digest}\n"
                   "@frames_per_launch = 64\n"
                   "@traffic_bytes_per_launch = 12345\n")
    assert bench.measured_traffic("t") == 12345.0
    assert bench.measured_traffic("t", 64) == 12345.0
    # counted at another batch size: not this launch's traffic
    assert bench.measured_traffic("t", 65) is None
    src.write_text("// kernel v2\n")
    assert bench.measured_traffic("t") is None
    rec.unlink()
    assert bench.measured_traffic("t") is None


def test_committed_records_parse():
    """Each committed record carries the machine-read lines bench.py needs
    (whether its digest still matches the sources is a property of the tree
    at measurement time, not checked here)."""
    for name, (record, _) in bench.TRAFFIC_RECORDS.items():
        path = os.path.join(ROOT, "profiles", record)
        if not os.path.exists(path):
            continue
        keys = {ln[1:].split("=", 1)[0].strip()
                for ln in open(path) if ln.startswith("@")}
        assert {"source_sha256_16", "traffic_bytes_per_launch",
                "fetch_scale", "write_scale"} <= keys, name


def test_committed_records_match_the_kernel_sources():
    """Each traffic record was counted on the kernel sources as they stand,
    so the benchmark line carries it (a kernel change needs a new count)."""
    for name, (record, srcs) in bench.TRAFFIC_RECORDS.items():
        path = os.path.join(ROOT, "profiles", record)
        assert os.path.exists(path), name
        lines = {ln[1:].split("=", 1)[0].strip(): ln.split("=", 1)[1].strip()
                 for ln in open(path) if ln.startswith("@")}
        assert lines["source_sha256_16"] == bench.source_digest(srcs), name
        frames = int(lines["frames_per_launch"])
        assert bench.measured_traffic(name, frames) == float(
            lines["traffic_bytes_per_launch"]), name
