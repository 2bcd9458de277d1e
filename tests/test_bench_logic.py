"""Host logic of bench.py (no GPU): the choice of the split mode that carries
the 1e-5 comparison, and the use of a committed counter summary only for the
kernel sources and the launch shape it was taken with."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _errs(**worst):
    return {k: {"max_rel_err_gamma_n": v} for k, v in worst.items()}


def test_split_choice_takes_the_fastest_mode_within_half_the_bar(bench):
    errs = _errs(bf16x3=9.9e-6, bf16x6=3.0e-7, fp16x3=3.1e-7)
    ms = {"bf16x3": 6.5, "bf16x6": 7.5, "fp16x3": 12.8}
    tflops = {"bf16x3": 76.4, "bf16x6": 66.6, "fp16x3": 38.8}
    r = bench.split_at_bar(errs, ms, tflops)
    assert r["mode"] == "bf16x6"
    assert r["stage2_ms"] == 7.5 and r["gemm_tflops"] == 66.6 and r["max_rel_err_gamma_n"] == 3.0e-7
    # at half the bar or below a faster mode qualifies
    errs["bf16x3"]["max_rel_err_gamma_n"] = 5.0e-6
    assert bench.split_at_bar(errs, ms, tflops)["mode"] == "bf16x3"
    # modes without a timing are not candidates
    assert bench.split_at_bar(errs, {"bf16x6": 7.5}, {"bf16x6": 66.6})["mode"] == "bf16x6"


def test_split_choice_is_none_when_no_mode_qualifies(bench):
    errs = _errs(bf16x3=9.0e-6, bf16x6=6.0e-6)
    assert bench.split_at_bar(errs, {"bf16x3": 1.0, "bf16x6": 2.0}, {"bf16x3": 1.0, "bf16x6": 1.0}) is None


def test_profiled_traffic_needs_matching_sources_and_launches(bench, tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_scan_field_1m.md").write_text(
        "# summary\n\nkernel-source-sha256: abc123\n\nlaunches-per-step: 16\n\ntraffic-bytes-per-launch: 4.43e+09\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc123")
    assert bench.profiled_traffic(16) == pytest.approx(4.43e9)
    assert bench.profiled_traffic(4) is None                     # another chunking
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "def456")
    assert bench.profiled_traffic(16) is None                    # other kernel sources
    assert bench.profiled_traffic(16, summary="missing.md") is None


def test_kernel_source_hash_is_a_stable_sha256(bench):
    h = bench.kernel_source_hash()
    assert len(h) == 64 and int(h, 16) >= 0
    assert bench.kernel_source_hash() == h


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in (r.stdout + r.stderr)
    assert "{" not in r.stdout  # no bench line
