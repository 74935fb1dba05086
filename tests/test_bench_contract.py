"""The benchmark's host-side contract (no GPU needed): the one-GPU refusal and
the rule that counted HBM traffic is reported only for the kernel sources it
was measured on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _summary(path, digest, traffic):
    with open(path, "w") as f:
        f.write("# HBM traffic\n\n")
        f.write(f"kernel_source_sha256: {digest}\n")
        f.write(f"traffic_bytes_per_launch: {traffic}\n")


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    path = str(tmp_path / "traffic.md")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", path)
    # no summary: nothing to report
    assert bench.measured_traffic("fv2048") is None
    # a summary of the current sources is read back
    _summary(path, bench.kernel_source_digest(), 58583286.4)
    assert bench.measured_traffic("fv2048") == 58583286.4
    # it covers the FV 2048^2 workload only
    assert bench.measured_traffic("fv8192") is None
    # a summary of other sources (a changed kernel) is not used
    _summary(path, "0" * 64, 58583286.4)
    assert bench.measured_traffic("fv2048") is None


def test_source_digest_covers_the_product_sources():
    csrc = os.path.join(ROOT, "paper_2508_17517_amd", "csrc")
    for f in bench.TRAFFIC_SOURCES:
        assert os.path.exists(os.path.join(csrc, f)), f
    assert "spmv.hip" in bench.TRAFFIC_SOURCES and "order.hip" in bench.TRAFFIC_SOURCES
    d = bench.kernel_source_digest()
    assert len(d) == 64 and d == bench.kernel_source_digest()
