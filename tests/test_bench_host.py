"""Host-side parts of bench.py that need no GPU: it refuses more than one GPU
before touching the device, and it reports the solve GEMM's measured HBM
traffic only while the profile it reads was taken on the same kernel
sources."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_traffic_needs_a_matching_kernel_hash(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 16
    prof = tmp_path / "profiles"
    prof.mkdir()
    body = "- kernel_source_hash: {}\n- hbm_bytes_per_launch: 4.5e+10\n"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    (prof / "pmc_dgemm_apply_minv_w.md").write_text(body.format(h))
    assert bench.read_traffic("w") == 4.5e10
    (prof / "pmc_dgemm_apply_minv_w.md").write_text(body.format("0" * 16))
    assert bench.read_traffic("w") is None
    assert bench.read_traffic("missing") is None

