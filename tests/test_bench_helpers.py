"""The measurement helpers of bench.py that need no GPU: the HBM traffic is
taken from a counter summary only while it matches the kernel source, the
insertion scan and the single-block loop split the up-moves' algorithmic
bytes, and the roofline divides algorithmic bytes by measured time."""
import sys

import pytest

sys.path.insert(0, __file__.rsplit("/tests/", 1)[0])
import bench  # noqa: E402


def test_traffic_only_for_the_current_source(tmp_path):
    p = tmp_path / "summary.txt"
    p.write_text(f"hbm_bytes_per_launch: 1234.5\nkernel_source_sha256_16: {bench.source_digest()}\n")
    assert bench.measured_traffic(str(p)) == 1234.5
    p.write_text("hbm_bytes_per_launch: 1234.5\nkernel_source_sha256_16: 0000000000000000\n")
    assert bench.measured_traffic(str(p)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt")) is None


def test_kernel_bytes_split():
    s = {"alg_bytes_up": 1000, "alg_bytes_up_loop": 150}
    assert bench.kernel_bytes("ins_scan", s) == 850
    assert bench.kernel_bytes("ins_loop", s) == 150
    assert bench.kernel_bytes("jmp_scan", s) == 1000


def test_roofline():
    r = bench.roofline({"launches": 10, "timed_ms": 0.1, "alg_bytes": 8e6}, "ins_scan")
    assert r["kernel"] == "k_ins_scan" and r["avg_launch_us"] == pytest.approx(10.0)
    assert r["achieved"] == pytest.approx(8e5 / 1e-5 / 1e9, rel=1e-3)       # 80 GB/s
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, rel=1e-2)
    assert bench.roofline({"launches": 0, "timed_ms": 0.0, "alg_bytes": 0}, "ins_scan") is None
