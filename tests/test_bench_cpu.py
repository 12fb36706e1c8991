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


def _tiny_problem(nvs=12):
    import numpy as np
    import torch

    import synth
    wl = synth.WORKLOADS["tiny2d"].replace(ns=10, nr=9, nvs=nvs, nt=64, nf=20, nb=4)
    rng = np.random.default_rng(3)
    d = torch.from_numpy(rng.standard_normal((wl.ns, wl.nr, wl.nt)))
    u = torch.from_numpy(rng.standard_normal((wl.ns, wl.nvs, wl.nt)))
    onset = rng.integers(0, 8, size=(wl.nr, wl.nvs)).astype(np.int32)
    return wl, d, u, onset


def test_oracle_on_columns_equals_the_full_gradient_columns():
    """The bench checks the GPU gradient on a few virtual-source columns: without
    reciprocity those columns of the oracle's gradient do not depend on the others,
    also when several models' columns share one oracle call."""
    import numpy as np
    import torch

    import bench
    from oracle import freq, optim
    wl, d, u, onset = _tiny_problem()
    R = torch.from_numpy(np.random.default_rng(4).standard_normal((wl.nr, wl.nvs, wl.nt)))
    idx = np.array([1, 4, 7, 8])
    _, g = freq.batch_loss_grad(d.numpy(), R.numpy(), u.numpy(), idx, wl.nf)
    g = optim.apply_mask(g, onset)
    cols = np.array([0, 5, 11])
    gc = bench.oracle_gradient_columns(wl, d, u, onset, R[:, cols].numpy(), idx, cols)
    np.testing.assert_allclose(gc, g[:, cols], rtol=0, atol=1e-12 * np.abs(g).max())
    two = np.concatenate([R[:, cols].numpy(), 2 * R[:, cols].numpy()], axis=1)
    gg = bench.oracle_gradient_columns(wl, d, u, onset, two, idx, cols, reps=2)
    np.testing.assert_allclose(gg[:, :3], g[:, cols], rtol=0, atol=1e-12 * np.abs(g).max())
    errs = bench.gradient_errors(wl, d, u, onset, R, {"same": torch.from_numpy(g)}, idx, cols)
    assert errs["same"] < 1e-14


def test_cpu_baseline_on_columns_extrapolates_linearly():
    import bench
    wl, d, u, onset = _tiny_problem(nvs=40)
    cb = bench.cpu_baseline_columns(wl, d, u, onset, budget_s=30.0, ks=(4, 16), steps_per_k=1)
    t = {int(k): v for k, v in cb["seconds_per_step_measured"].items()}
    assert set(t) == {4, 16} and cb["value"] > 0 and cb["kind"] == "oracle"
    slope = (t[16] - t[4]) / 12
    assert abs(cb["seconds_per_full_step"] - (max(t[4] - 4 * slope, 0) + 40 * slope)) < 1e-12
    assert "columns" in cb["sample"] and cb["cores"] >= 1


def test_host_cpu_names_the_model():
    import bench
    model, n = bench.host_cpu()
    assert isinstance(model, str) and n >= 1
