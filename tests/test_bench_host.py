"""Host logic of bench.py (CPU): the single-GPU refusal, the comment-blind
kernel-source hash that ties a committed profile to the kernels it measured,
the reading of per-step figures from a profile summary, and the regime."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_source_hash_ignores_comments_and_blank_lines_only():
    a = "int f(int x) {\n  // twice\n  return 2 * x; /* doubled */\n}\n"
    b = "int f(int x) {\n\n  return 2 * x;\n}\n"
    c = "int f(int x) {\n  return 3 * x;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
    assert len(bench.kernel_source_hash()) == 16


def test_profile_figure_is_read_only_for_the_current_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    p = tmp_path / "summary.md"
    p.write_text("text\ntraffic_bytes_per_step: 4.110283e+09 sources: %s\n"
                 "valu_instr_per_step: 1.1e9 sources: 0123456789abcdef\n" % h)
    monkeypatch.setitem(bench.PROFILES, "c5", str(p))
    assert bench._profile_figure("c5", "traffic_bytes_per_step") == 4.110283e9
    # taken on other sources: not reported
    assert bench._profile_figure("c5", "valu_instr_per_step") is None
    assert bench._profile_figure("c5", "missing_key") is None
    monkeypatch.setitem(bench.PROFILES, "c5", str(tmp_path / "absent.md"))
    assert bench._profile_figure("c5", "traffic_bytes_per_step") is None


def test_regime_follows_the_larger_measured_fraction():
    assert bench.regime_of(0.58, 0.16) == "VALU issue and per-cell latency"
    assert bench.regime_of(0.10, 0.70) == "HBM traffic"
    assert bench.regime_of(None, 0.2) == "HBM traffic"
    assert bench.regime_of(0.3, None) == "VALU issue and per-cell latency"
    assert bench.regime_of(None, None) == "unmeasured"
