"""GPU parity at the benchmark's full size (512^3) in the launch configuration
the benchmark times (automatic kernel choice: the tiled step).

The oracle cannot evolve 512^3 in seconds, so one GPU step from a GPU-made
snapshot is checked against the oracle evaluated one site at a time on
sampled sites (corners, tile and z-chunk boundaries, random interior), the
windings on sampled plaquettes are checked bit for bit, and properties that
hold at any size are checked on the whole lattice (Gauss law, windings sum).
"""
import numpy as np
import pytest

from helpers import both_params, field_scaled_error
from inputs import sample_sites

pytestmark = pytest.mark.gpu

N = 512


def _boundary_sites(N):
    """Sites on tile edges (x0 = 63, 64, y = 7, 8) and z-chunk edges (z = 255, 256)."""
    out = []
    for x in (0, 63, 64, 511):
        for y in (0, 7, 8, 511):
            for z in (0, 255, 256, 511):
                out.append(x + N * (y + N * z))
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-6), ("fp64", 1e-13)])
def test_fullsize_one_step_sampled(oracle_mod, precision, tol):
    import paper_2005_14454_amd as ah
    op, gp = both_params(oracle_mod, N, precision, m=1.0)
    with ah.Lattice(gp) as lat:
        lat.init(1)
        lat.step(5)
        before = lat.get_state()
        lat.step(1)
        after = lat.get_state()
        meas = lat.measure()
        cfg = lat.get_step_config()
        w_sites = sample_sites(N, 3000, seed=17)
        w_gpu = lat.winding()[:, w_sites].T
    assert cfg["kernel"] == "tile"
    sites = np.unique(np.concatenate([sample_sites(N, 4000, seed=5), _boundary_sites(N)]))
    ref = oracle_mod.step_sites(op, before, 5, sites)
    got = after[:, sites]
    err = field_scaled_error(got, ref.T)
    print(precision, "512^3 sampled one-step error", err)
    assert max(err.values()) <= tol, err
    # windings of the GPU snapshot on sampled plaquettes, bit for bit
    w_ref = oracle_mod.winding_sites(op, after, w_sites)
    assert np.array_equal(w_gpu, w_ref.astype(np.int8))
    # whole-lattice properties
    assert meas["nonfinite"] == 0
    assert meas["gauss_rel"] < (1e-12 if precision == "fp64" else 1e-5)
    assert meas["winding_sum_abs"] > 0
