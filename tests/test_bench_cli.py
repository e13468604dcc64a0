"""Host logic of the benchmark harness (no GPU): the one-GPU guard, the
missing-device exit, and the lookup of the committed HBM-traffic figure,
which is only used while the kernel sources hash as when it was taken."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, cwd=ROOT, env=env, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    env = dict(os.environ, WORLD_SIZE="4")
    assert _run(env=env).returncode == 2


def test_no_device_exits_with_a_message():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = _run("--only", "ppe:mixed", "--steps", "1", "--warmup", "0")
    assert r.returncode == 1
    assert "HIP device" in r.stderr


def test_traffic_lookup_follows_the_kernel_sources(tmp_path, monkeypatch):
    src = bench.kernel_source_hash()
    assert len(src) == 12 and src == bench.kernel_source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.txt").write_text(
        "# kernel workload hash bytes\n"
        f"cg_spmv wl_a {src} 123.0\n"
        f"cg_spmv wl_b 000000000000 456.0\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the kernel-source hash is read from the real tree, the table from tmp
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: src)
    assert bench.read_traffic("cg_spmv", "wl_a") == 123.0
    assert bench.read_traffic("cg_spmv", "wl_b") is None   # stale sources
    assert bench.read_traffic("sort", "wl_a") is None
    (prof / "traffic.txt").unlink()
    assert bench.read_traffic("cg_spmv", "wl_a") is None

