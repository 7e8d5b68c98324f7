"""The C-ABI library loads and exports every entry point include/ah.h declares,
and the ctypes mirrors of its structs have the header's layout.  No GPU needed:
nothing here launches device work."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ah.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ah_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2005_14454_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2005_14454_amd import build
        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layout_matches_header(tmp_path):
    from paper_2005_14454_amd import _lib
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "ah.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(ah_params), sizeof(ah_measurement),'
        ' offsetof(ah_params, eta_ref), offsetof(ah_measurement, flags), offsetof(ah_measurement, nonfinite));'
        'return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(_lib.ah_params), ctypes.sizeof(_lib.ah_measurement),
            _lib.ah_params.eta_ref.offset, _lib.ah_measurement.flags.offset, _lib.ah_measurement.nonfinite.offset]
    assert got == want


def test_host_only_entry_points(lib):
    from paper_2005_14454_amd import Params, _lib
    p = _lib.ah_params()
    assert lib.ah_params_default(ctypes.byref(p)) == 0
    assert p.N == 64 and p.dx == 0.5 and p.deta == 0.1 and p.lambda0 == 2.0 and p.e0 == 1.0
    n = ctypes.c_size_t()
    assert lib.ah_required_bytes(ctypes.byref(Params(N=64).to_c()), ctypes.byref(n)) == 0
    assert n.value >= 20 * 8 * 64 ** 3
    n32 = ctypes.c_size_t()
    assert lib.ah_required_bytes(ctypes.byref(Params(N=64, precision="fp32").to_c()), ctypes.byref(n32)) == 0
    assert 20 * 4 * 64 ** 3 <= n32.value < n.value
    assert lib.ah_required_bytes(ctypes.byref(Params(N=3).to_c()), ctypes.byref(n)) == _lib.AH_E_INVAL
    bad = Params(N=16).to_c()
    bad.dx = -1.0
    assert lib.ah_required_bytes(ctypes.byref(bad), ctypes.byref(n)) == _lib.AH_E_INVAL
    assert lib.ah_strerror(_lib.AH_E_AGAIN).decode()
    assert lib.ah_last_error(None).decode() == ""
    # argument checks that come before any device work
    c, r, w = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    assert lib.ah_hbm_probe(1000, 1, ctypes.byref(c), ctypes.byref(r), ctypes.byref(w)) == _lib.AH_E_INVAL
    assert lib.ah_hbm_probe(1 << 26, 0, ctypes.byref(c), ctypes.byref(r), ctypes.byref(w)) == _lib.AH_E_INVAL
    assert lib.ah_hbm_probe(1 << 26, 1, None, ctypes.byref(r), ctypes.byref(w)) == _lib.AH_E_INVAL
    cfg = _lib.ah_step_config()
    assert lib.ah_pool_step_config(None, 1, ctypes.byref(cfg)) == _lib.AH_E_INVAL
