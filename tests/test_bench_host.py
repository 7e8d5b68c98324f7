"""Host-side parts of bench.py: the one-GPU contract and how the roofline's
measured traffic is read from a rocprofv3 summary (and refused once the
kernel source no longer matches the counters)."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_measured_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "kernel.hip"
    src.write_bytes(b"// a kernel\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    prof = tmp_path / "traffic.txt"
    row = "k_step_tile<float, 128, 8, false>              2691475      5246336     5.512     5.372    10.884   10.737    {n}\n"
    prof.write_text(f"kernel source ah_step_tile.hip sha256[:16] = {digest}\n\n" + row.format(n=2) + row.replace(
        "10.884", "11.000").format(n=6))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    # the row with the most dispatches is the benchmark's own configuration
    assert bench.measured_traffic("fp32", 512, (128, 8)) == 11.0e9
    assert bench.measured_traffic("fp32", 512, (64, 8)) is None       # no row for that tile
    assert bench.measured_traffic("fp32", 256, (128, 8)) is None      # counters were taken at 512^3
    src.write_bytes(b"// a changed kernel\n")
    assert bench.measured_traffic("fp32", 512, (128, 8)) is None      # stale counters are not reported
