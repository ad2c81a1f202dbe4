"""Host-side checks of bench.py's report plumbing (no GPU): the HBM traffic it attaches to a
roofline comes from the committed counter summary only while the kernel's sources are unchanged."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SUMMARY = """# HBM traffic per launch

Sources: `svd.hip`: `{svd}`, `sketch.hip`: `{sketch}`

| kernel | launches | FETCH_SIZE KiB | WRITE_SIZE KiB | fetched MB | written MB | algorithmic MB | traffic / algorithmic |
|---|---:|---:|---:|---:|---:|---:|---:|
| `nsk::sparse_kernel<float, double, 8, 16>` | 5 | 449722 | 24307 | 921.0 | 24.9 | 805.3 | 1.175 |
| `nsk::svd_jacobi_coop_kernel<4>` | 5 | 27463 | 63292 | 56.2 | 64.8 |  |  |
"""


@pytest.fixture
def summary(tmp_path, monkeypatch):
    path = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(path))
    return path


def test_traffic_is_fetched_plus_written_of_the_kernel_row(summary):
    summary.write_text(SUMMARY.format(svd=bench.kernel_source_hash("svd.hip"),
                                      sketch=bench.kernel_source_hash("sketch.hip")))
    assert bench.measured_traffic("svd_jacobi_coop_kernel") == pytest.approx((56.2 + 64.8) * 1e6)
    assert bench.measured_traffic("sparse_kernel") == pytest.approx((921.0 + 24.9) * 1e6)
    assert bench.measured_traffic("residual_kernel") is None  # not listed


def test_traffic_is_null_once_the_kernels_sources_changed(summary):
    summary.write_text(SUMMARY.format(svd="0" * 16, sketch=bench.kernel_source_hash("sketch.hip")))
    assert bench.measured_traffic("svd_jacobi_coop_kernel") is None
    assert bench.measured_traffic("sparse_kernel") is not None


def test_source_digest_covers_the_unit_and_the_headers():
    a, b = bench.kernel_source_hash("svd.hip"), bench.kernel_source_hash("sketch.hip")
    assert len(a) == 16 and a != b
