"""Host logic of bench.py (no GPU): the HBM traffic it reports comes from a committed
counter summary only while the kernel sources still hash to the value the summary
names, and --gpus above 1 is refused."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _tree(tmp_path, source_text, summary_hash):
    (tmp_path / "paper_1811_10573_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1811_10573_amd" / "csrc" / "k_batch.hip").write_text(source_text)
    (tmp_path / "profiles" / "k_b_gemm_f32_batch512_counters.md").write_text(
        f"hbm_bytes_per_launch: 5.0e+09\n\nsource_sha256: {summary_hash}\n")


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    import hashlib
    src = "// kernel source\n"
    _tree(tmp_path, src, hashlib.sha256(src.encode()).hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_b_gemm", None, None, None, workload="f32_batch512") == 5.0e9
    # another workload has no summary
    assert bench.measured_traffic("k_b_gemm", None, None, None, workload="f32_batch64") is None
    # the source changed after the counters were taken
    (tmp_path / "paper_1811_10573_amd" / "csrc" / "k_batch.hip").write_text(src + "// edit\n")
    assert bench.measured_traffic("k_b_gemm", None, None, None, workload="f32_batch512") is None


def test_committed_summaries_name_their_sources():
    """Every committed counter summary that bench reads names a hash and a per-launch
    byte count it can parse."""
    import re
    names = {"level1_gemm": "level1_gemm_f32_800x800x800_r50", "pp_correct_ttv": "pp_correct_ttv_f32_800x800x800_r50",
             "k_b_gemm": "k_b_gemm_f32_batch512"}
    stems = list(names.items()) + [("level1_gemm", "level1_gemm_f64_800x800x800_r50"),
                                   ("pp_correct_ttv", "pp_correct_ttv_f64_800x800x800_r50")]
    for kernel, stem in stems:
        assert kernel in bench.TRAFFIC_SOURCE
        txt = open(os.path.join(ROOT, "profiles", f"{stem}_counters.md")).read()
        assert re.search(r"hbm_bytes_per_launch:\s*[0-9.eE+]+", txt), stem
        assert re.search(r"source_sha256:\s*[0-9a-f]{64}", txt), stem


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr), r.stderr[-400:]
