"""The FP64 sincos the step kernels use for the link variables, compiled for
the host and checked against long-double sin and cos (the C library's
extended-precision routines, accurate well past double)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_link_sincos_accuracy(tmp_path):
    exe = tmp_path / "sincos_check"
    subprocess.run(["g++", "-O2", "-ffp-contract=off", "-I", os.path.join(ROOT, "paper_2005_14454_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sincos_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=300).stdout
    rows = {}
    for line in out.splitlines():
        f = line.split()
        if f[0] == "range":
            rows[float(f[1])] = (float(f[3]), float(f[5]))
        elif f[0] == "nearcut":
            near = float(f[2])
    print(out)
    for R, (ulp, abs_err) in rows.items():
        assert ulp <= (1.6 if R <= 1e3 else 2.5), (R, ulp)
        assert abs_err <= 1.6e-16, (R, abs_err)
    assert near <= 2.5
