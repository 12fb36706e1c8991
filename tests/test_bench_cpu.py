"""bench.py pieces that run without a GPU: the one-GPU guard and the rule that a stored
counter figure counts only while its kernel source is unchanged."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


def test_stored_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    summary = tmp_path / "traffic_w.md"
    summary.write_text("- upd_source: `k.hip`\n"
                       f"- upd_source_sha256: `{bench.source_hash(str(src))}`\n"
                       "- upd_hbm_bytes_per_launch: `12345`\n")
    monkeypatch.setattr(bench, "CSRC", str(tmp_path))
    monkeypatch.setitem(bench.TRAFFIC_FILE, "w", str(summary))
    assert bench.stored_traffic("w", "upd") == 12345.0
    src.write_text("kernel v2\n")                  # the kernel changed: the figure is stale
    assert bench.stored_traffic("w", "upd") is None
    assert bench.stored_traffic("w", "other") is None
    assert bench.stored_traffic("missing", "upd") is None


def test_committed_summaries_match_the_current_kernels():
    """Every counter figure bench.py reads for the 2D line, the 3D patch, the
    single-virtual-source patch and the differentiation form belongs to the kernel source
    as it is now."""
    import bench
    for workload, keys in (("line2d", ("update", "gemm_fp32")),
                           ("patch3d", ("update", "gemm_fp32", "gemm_bf16x3", "gemm_fp16x3")),
                           ("patch3d_vs1", ("update", "gemv")),
                           ("diff301", ("products", "reciprocity", "spec_reciprocity"))):
        for k in keys:
            assert bench.stored_traffic(workload, k) is not None, (workload, k)
