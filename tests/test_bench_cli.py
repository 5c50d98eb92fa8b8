"""bench.py's command-line contract on the host: more than one GPU is
refused with a message, and the traffic figures are reported only for the
kernel sources they were measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_traffic_is_gated_by_the_source_digest(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "profiles", "band_kernel_traffic_paper_grid.txt")
    text = open(src).read()
    fake = tmp_path / "profiles"
    fake.mkdir()
    dig = bench.kernel_source_digest()
    lines = [l for l in text.splitlines() if not l.startswith("kernel_source_sha256:")]
    (fake / "band_kernel_traffic_paper_grid.txt").write_text(
        "\n".join(lines + ["kernel_source_sha256: " + dig]) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: dig)
    assert bench.measured_traffic("bt_band_kernel<1, double>") is not None
    (fake / "band_kernel_traffic_paper_grid.txt").write_text(
        "\n".join(lines + ["kernel_source_sha256: " + "0" * 64]) + "\n")
    assert bench.measured_traffic("bt_band_kernel<1, double>") is None
