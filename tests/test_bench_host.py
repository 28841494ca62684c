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
    # eq. (1): three distinct min-sum terms (sign product, magnitude
    # minimum, scaling) and three additions per PE
    assert bench.OPS_PER_PE == 12
    # one round-trip pass computes two outputs: two terms and two additions
    assert bench.OPS_PER_PE_PASS == 8
    # SC: m N / 2 evaluations each of f and g, two operations each
    assert bench.sc_ops_per_frame(1024) == 20480


def test_record_readers(tmp_path, monkeypatch):
    """Trace and counter records give the kernel time and the VALU issue
    fraction only while their sources and frame count match."""
    src = tmp_path / "k.hip"
    src.write_text("kernel")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    rec = tmp_path / "profiles" / "t.md"
    monkeypatch.setitem(bench.TRACE_RECORDS, "t", ("t.md", [str(src)]))
    monkeypatch.setitem(bench.COUNTER_RECORDS, "t", ("t.md", [str(src)]))
    digest = bench.source_digest([str(src)])
    rec.write_text(f"@source_sha256_16 = {digest}\n@frames_per_launch = 100\n"
                   "@avg_ns[k<1>] = 2500000\n"
                   "@sq_insts_valu_per_launch[k<1>] = 1228800000\n")
    assert bench.traced_kernel_ms("t", "k<1>", 100) == pytest.approx(2.5)
    assert bench.traced_kernel_ms("t", "k<1>", 99) is None
    assert bench.traced_kernel_ms("t", "k<2>", 100) is None
    # 1.2288e9 instructions x 64 lanes in 2.5 ms over 39.3216e12 lane-op/s
    assert bench.valu_issue("t", "k<1>", 100, 2.5) == pytest.approx(0.8)
    src.write_text("changed kernel")
    assert bench.traced_kernel_ms("t", "k<1>", 100) is None
    assert bench.valu_issue("t", "k<1>", 100, 2.5) is None


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


def test_committed_traces_and_counters_match_the_kernel_sources():
    """Each kernel-trace and counter record was taken on the kernel sources
    as they stand, so the benchmark lines carry the traced kernel time and
    the VALU issue fraction (a kernel change needs a new trace)."""
    for table in (bench.TRACE_RECORDS, bench.COUNTER_RECORDS):
        for name, (record, srcs) in table.items():
            path = os.path.join(ROOT, "profiles", record)
            assert os.path.exists(path), (name, record)
            lines = {ln[1:].split("=", 1)[0].strip(): ln.split("=", 1)[1].strip()
                     for ln in open(path) if ln.startswith("@")}
            assert lines["source_sha256_16"] == bench.source_digest(srcs), (name, record)
            assert int(lines["frames_per_launch"]) > 0, (name, record)
    assert bench.traced_kernel_ms("n1024", bench.KERNEL, 1000000) > 0
    assert bench.valu_issue("n1024", bench.KERNEL, 1000000, 63.0) > 0
    assert bench.valu_issue("unrolled", "unrolled_backward_kernel<10>", 4096, 1.4) > 0
