"""bench.py's host-side helpers (no GPU): the counter figures it reports
beside the roofline come from the committed rocprofv3 summaries, and only
while those were taken on the current kernel source (its hash recorded in
the summary)."""
import os
import re
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("cfg,storage,engine,flags,kernel", [
    (2, "f16", "fft", 0, "ols_fft"),
    (5, "f16", "fft", 1, "ols_fft"),
    (4, "f16", "gemm", 0, "ols_gemm"),
    (4, "bf16", "gemm", 0, "ols_gemm"),
])
def test_counters_read_from_profiles(cfg, storage, engine, flags, kernel, monkeypatch):
    key = bench.workload_key(cfg, storage, engine, flags=flags)
    text = open(os.path.join(bench.PROFILE_DIR, f"{kernel}_{key}_pmc.md")).read()
    taken_on = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text).group(1)
    monkeypatch.setattr(bench, "kernel_hash", lambda engine: taken_on)   # as if the source were unchanged
    traffic, busy = bench.counters_from_profile(kernel, key, engine)
    assert traffic is not None and traffic > 1e9
    assert 0.0 < busy["valu_busy"] <= 1.0
    if engine == "gemm":
        assert 0.0 < busy["mfma_busy"] <= 1.0
    else:
        assert "mfma_busy" not in busy


def test_counters_ignored_for_another_kernel_source(tmp_path, monkeypatch):
    key = bench.workload_key(2, "f16", "fft")
    src = os.path.join(bench.PROFILE_DIR, f"ols_fft_{key}_pmc.md")
    shutil.copy(src, tmp_path / os.path.basename(src))
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    taken_on = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", open(src).read()).group(1)
    monkeypatch.setattr(bench, "kernel_hash", lambda engine: taken_on)
    assert bench.counters_from_profile("ols_fft", key, "fft")[0] is not None
    monkeypatch.setattr(bench, "kernel_hash", lambda engine: "0" * 16)
    assert bench.counters_from_profile("ols_fft", key, "fft") == (None, {})


def test_no_profile_no_counters():
    assert bench.counters_from_profile("ols_fft", "no_such_workload", "fft") == (None, {})
