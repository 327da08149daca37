"""Host-side pieces of bench.py (no GPU): the dominant-kernel roofline entry,
the counter-traffic lookup and its source digest guard, the compression rate
from the library's own sizes, and the kernel-family names."""
import pytest

import bench

T = pytest.importorskip("paper_2407_00769_amd._tnc", reason="libtnc.so not built")


def _fam(ms, flops, nbytes, launches=4):
    return {"ms": ms, "flops": flops, "bytes": nbytes, "launches": launches}


def test_roofline_entry_takes_the_family_with_most_time():
    fam = {"gemm_dma_8w": _fam(100.0, 1.2e17, 1e11), "permute": _fam(40.0, 0.0, 2e11, 10),
           "gemm_skinny": _fam(20.0, 1e13, 9e10, 50)}
    r = bench.roofline_entry(fam, "f16")
    assert r["kernel"] == "gemm_dma_8w" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(1.2e17 / 0.1 / 1e12, rel=1e-6)
    assert r["frac"] == pytest.approx(r["achieved"] / 2516.6, rel=1e-3)
    assert r["avg_launch_us"] == pytest.approx(25000.0)
    assert r["share_of_device_time"] == pytest.approx(100 / 160, rel=1e-3)


def test_roofline_entry_hbm_bound_below_the_ridge():
    fam = {"gemm_skinny": _fam(10.0, 1e12, 5e10), "permute": _fam(1.0, 0.0, 1e9)}
    r = bench.roofline_entry(fam, "f16")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(5e10 / 0.01 / 1e9, rel=1e-6)
    assert bench.roofline_entry({"permute": _fam(2.0, 0.0, 1e10)}, "f16")["bound"] == "hbm"


def test_traffic_lookup_is_guarded_by_the_source_digest(monkeypatch):
    val = bench.measured_traffic("gemm_dma_8w", "53q_f16_4m")
    if val is not None:
        assert val > 0
    assert bench.measured_traffic("no_such_kernel", "53q_f16_4m") is None
    assert bench.measured_traffic("gemm_dma_8w", "no_such_workload") is None
    monkeypatch.setattr(bench, "gemm_source_digest", lambda: "changed")
    assert bench.measured_traffic("gemm_dma_8w", "53q_f16_4m") is None


def test_compression_rate_from_library_sizes():
    n = 1 << 20
    assert bench.compression_rate(T, "half", n) == pytest.approx(0.5, abs=1e-5)
    assert bench.compression_rate(T, "int8", n) == pytest.approx(0.25, abs=1e-5)
    assert bench.compression_rate(T, "int4", n) == pytest.approx(0.125 + 8 / 512, abs=1e-6)


def test_every_kernel_id_has_a_family_name():
    names = [bench.kernel_family(i) for i in range(16)]
    assert len(set(names)) == 16
    assert all(not n[len("gemm_"):].isdigit() for n in names)
