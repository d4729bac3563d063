"""The bench line's host-side arithmetic, on the CPU: the algorithmic byte
models the roofline and the field rate use (the survey's per-unit figures:
48 B per particle-step plus 40 B per face for the particle kernel; 28 B per
face, 8 B per SPAI non-zero and 20 B per free edge for the field update),
the diagnostics overhead and its 10 % cadence, the traffic summary's source
check, and the refusal of more than one GPU."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_byte_models_follow_the_per_unit_figures():
    assert bench.particle_bytes(1, 0) == 48.0
    assert bench.particle_bytes(0, 1) == 40.0
    # the tube: 7,896,000 live particles and 207,935 faces -> 387.3 MB per launch
    assert bench.particle_bytes(7_896_000, 207_935) == pytest.approx(387_325_400.0)
    assert bench.field_bytes(0, 1, 0) == 28.0
    assert bench.field_bytes(0, 0, 1) == 8.0
    assert bench.field_bytes(1, 0, 0) == 20.0


def test_diagnostics_cost_and_cadence():
    c = bench.diagnostics_cost(0.1723, 0.1445, 1)
    assert c["overhead"] == pytest.approx(0.1723 / 0.1445 - 1)
    assert c["overhead_per_diagnostic_step"] == pytest.approx(c["overhead"])
    assert c["diag_every_for_10pct"] == 2          # +19 % per diagnostic step -> every second step
    # at cadence 4 the same per-step cost is a quarter per step
    c4 = bench.diagnostics_cost(0.1445 * (1 + 0.19 / 4), 0.1445, 4)
    assert c4["overhead_per_diagnostic_step"] == pytest.approx(0.19)
    assert c4["diag_every_for_10pct"] == 2
    assert bench.diagnostics_cost(0.15, 0.15, 1)["diag_every_for_10pct"] == 1
    assert bench.diagnostics_cost(0.1445 * 1.10, 0.1445, 1)["diag_every_for_10pct"] == 1
    assert bench.diagnostics_cost(0.1445 * 1.35, 0.1445, 1)["diag_every_for_10pct"] == 4


def test_traffic_summary_is_used_only_for_its_kernel_source(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text(f"hbm_bytes_per_launch = 415722108\nkernel_source_sha256_16 = {bench.kernel_source_hash()}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() == 415722108.0
    f.write_text("hbm_bytes_per_launch = 415722108\nkernel_source_sha256_16 = 0000000000000000\n")
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
