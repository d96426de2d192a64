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


def test_more_than_one_gpu_exits_with_a_message():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_tune_cache_file_is_a_temporary_copy(tmp_path):
    path, note = bench.tune_cache_file(None)
    try:
        assert path != bench.TUNE_CACHE and os.path.exists(path)
        assert open(path).read() == open(bench.TUNE_CACHE).read()
        assert "tune_mi355x.txt" in note
    finally:
        os.unlink(path)
    assert bench.tune_cache_file("") == (None, "")
    given = str(tmp_path / "t.txt")
    assert bench.tune_cache_file(given)[0] == given
