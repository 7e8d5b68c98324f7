"""The workload entry points and the bandwidth probe on the GPU: workload 1
(64^3 FP64, 160 steps) runs through `workloads.py` with its diagnostics
every 10 steps and Gauss's law exact; the probe's streaming kernels report
plausible rates."""
import pytest

pytestmark = pytest.mark.gpu


def test_workload_1():
    from paper_2005_14454_amd.workloads import config1
    out = config1()
    steps = [m["step"] for m in out["series"]]
    assert steps == list(range(0, 161, 10))
    assert all(m["gauss_rel"] < 1e-13 and m["nonfinite"] == 0 and m["flags"] == 0 for m in out["series"])
    # the random-phase start winds a third of the plaquettes; the network then coarsens
    w = [m["winding_sum_abs"] for m in out["series"]]
    assert abs(w[0] / (64 ** 3) - 1.0) < 0.01 and w[-1] < w[0] / 10


def test_hbm_probe_small():
    import paper_2005_14454_amd as ah
    out = ah.hbm_probe(64 << 20, reps=2)
    for k in ("copy_GB/s", "read_GB/s", "write_GB/s"):
        assert 100.0 < out[k] < 20000.0, out
