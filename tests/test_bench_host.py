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
    digest = {"h": "0123456789abcdef"}
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel: digest["h"] if kernel == "tile2" else "x")
    prof = tmp_path / "traffic.txt"
    row = "k_step2_tile<float, 64, 8>              2691475      5246336     5.512     5.372    10.884   10.737    {n}\n"
    prof.write_text("tile2 sources sha256[:16] = 0123456789abcdef\n\n" + row.format(n=2) + row.replace(
        "10.884", "11.000").format(n=6))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    cfg = {"kernel": "tile2", "tile": (64, 8), "zchunk": 256}
    # the row with the most dispatches is the benchmark's own configuration
    assert bench.measured_traffic("fp32", 512, cfg) == 11.0e9
    assert bench.measured_traffic("fp32", 512, dict(cfg, tile=(32, 8))) is None    # no row for that tile
    assert bench.measured_traffic("fp32", 256, cfg) is None                        # counters were taken at 512^3
    assert bench.measured_traffic("fp32", 512, dict(cfg, kernel="tile")) is None   # nor for the one-step kernel
    digest["h"] = "fedcba9876543210"
    assert bench.measured_traffic("fp32", 512, cfg) is None                        # stale counters are not reported


def test_kernel_source_hash_covers_the_shared_stencil():
    import bench
    h = hashlib.sha256()
    for name in ("ah_step2.hip", "ah_stencil.h"):
        h.update(open(os.path.join(ROOT, "paper_2005_14454_amd", "csrc", name), "rb").read())
    assert bench.kernel_source_hash("tile2") == h.hexdigest()[:16]
    assert bench.step_kernel_name("fp64", {"kernel": "tile", "tile": (32, 8)}) == "k_step_tile<double, 32, 8, false>"
