"""Host logic of bench.py that decides what the JSON line reports: the
committed rocprofv3 traffic summaries are used only while the kernel's
sources are the ones they were taken from, the roofline picks the longer
of the two ideal times, and the committed summaries parse."""
import os

import pytest

import bench


def _summary(tmp_path, digest, hbm=123456.0):
    p = tmp_path / "s.txt"
    p.write_text("# a comment = not a value\nlaunches = 3\nhbm_bytes_per_launch = %r\nsource_sha256 = %s\n"
                 % (hbm, digest))
    return str(p)


def test_traffic_needs_the_same_sources(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    path = _summary(tmp_path, bench.source_digest([str(src)]))
    assert bench.pmc_traffic(path, [str(src)]) == 123456.0
    src.write_text("kernel v2\n")  # the kernel changed since the counters were taken
    assert bench.pmc_traffic(path, [str(src)]) is None


def test_traffic_missing_summary_or_value(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("x")
    assert bench.pmc_traffic(str(tmp_path / "none.txt"), [str(src)]) is None
    p = tmp_path / "s.txt"
    p.write_text("source_sha256 = %s\n" % bench.source_digest([str(src)]))
    assert bench.pmc_traffic(str(p), [str(src)]) is None


def test_digest_depends_on_order_and_content(tmp_path):
    a, b = tmp_path / "a", tmp_path / "b"
    a.write_text("1")
    b.write_text("2")
    assert bench.source_digest([str(a), str(b)]) != bench.source_digest([str(b), str(a)])


def test_roofline_bound_is_the_longer_ideal_time():
    # 8 GB at 8 TB/s = 1 ms; 1 GFLOP at 78.6 TF ~ 13 us: HBM-bound
    r = bench.roofline(8e9, 1e9, 2e-3, bench.FP64_MFMA_PEAK_TFLOPS, "k")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0) and r["frac"] == pytest.approx(0.5)
    # 1 MB and 1 TFLOP: MFMA-bound
    r = bench.roofline(1e6, 1e12, 1.0, bench.FP64_MFMA_PEAK_TFLOPS, "k", traffic=5.0)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["traffic"] == 5.0
    assert r["frac"] == pytest.approx(1.0 / bench.FP64_MFMA_PEAK_TFLOPS)


def test_committed_summaries_parse():
    for path in (bench.PMC_SUMMARY, bench.BATCH_PMC_SUMMARY):
        assert os.path.exists(path)
        vals = {}
        for line in open(path):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
        assert float(vals["hbm_bytes_per_launch"]) > 0
        assert len(vals["source_sha256"]) == 64


def test_lr_model_counts_each_core_once():
    import numpy as np
    x = [np.zeros((1, 3, 2)), np.zeros((2, 4, 5)), np.zeros((5, 2, 1))]
    b, f = bench.lr_model(x, 7)
    assert b == 8 * (6 + 40 + 10) + 8 * 7 * (2 + 5 + 1)
    assert f == 2 * 7 * (6 + 40 + 10)


def test_committed_summaries_match_the_sources():
    # the bench line reports traffic only from counters taken on the current kernel sources
    assert bench.pmc_traffic(bench.PMC_SUMMARY, bench.PC_SOURCES) is not None
    assert bench.pmc_traffic(bench.BATCH_PMC_SUMMARY, bench.BATCH_SOURCES) is not None
