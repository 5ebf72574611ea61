"""Host-side checks of bench.py (no GPU): the traffic models against the
per-configuration byte counts worked out for the workloads (compulsory:
density write, one read and one write per transform, G octant, potential
read; reference: five read+write sweeps of the half spectrum instead), the
counter-traffic summary's guards, and the one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n_p, meshes, compulsory_gb, reference_gb", [
    (256, [512, 128], 3.88, 7.17),      # clu256: 256^3 particles, fine 512^3, coarse 128^3
    (512, [1024, 256], 31.0, 57.3),     # clu512: 512^3 particles, fine 1024^3, coarse 256^3
])
def test_traffic_models(n_p, meshes, compulsory_gb, reference_gb):
    n = n_p ** 3
    assert abs(bench.step_compulsory_bytes(n, meshes) / 1e9 - compulsory_gb) < 0.01 * compulsory_gb
    assert abs(bench.step_reference_bytes(n, meshes) / 1e9 - reference_gb) < 0.01 * reference_gb
    # per level and cell: ~24.5 B (compulsory) and ~48.6 B (reference) at large n
    m = [4096]
    per_c = (bench.step_compulsory_bytes(0, m)) / 4096 ** 3
    per_r = (bench.step_reference_bytes(0, m)) / 4096 ** 3
    assert abs(per_c - 24.5) < 0.1 and abs(per_r - 48.5) < 0.2


def test_measured_traffic_guards(tmp_path, monkeypatch):
    """The counter-traffic summary counts only for its own workload and for
    the kernel source it was taken on."""
    digest = bench.source_digest(bench.PP_SOURCES)
    f = tmp_path / "t.txt"
    body = ("workload: {w}\nsource_digest: {d}\npp_fetch_kib: 1000\npp_write_kib: 500\n"
            "copy_bytes: 1048576\ncopy_fetch_kib: 512\ncopy_write_kib: 1024\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    f.write_text(body.format(w="clu512", d=digest))
    # fetch counts 0.5 per byte and write 1.0: 1000 KiB / 0.5 + 500 KiB / 1.0
    assert bench.measured_traffic("clu512") == pytest.approx(2000 * 1024 + 500 * 1024)
    assert bench.measured_traffic("clu256") is None
    f.write_text(body.format(w="clu512", d="0" * 16))
    assert bench.measured_traffic("clu512") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
