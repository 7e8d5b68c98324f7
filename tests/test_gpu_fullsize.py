"""GPU parity at the benchmark's full size (512^3) in the launch configuration
the benchmark times (the tiled step on the recorded tuning table's tiling).

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


@pytest.fixture(autouse=True)
def _release_cached_device_memory():
    """The lattices here take 8-132 GB each; hand torch's cached blocks back
    to the device between tests so that they never add up."""
    import torch
    torch.cuda.empty_cache()
    yield
    torch.cuda.empty_cache()

N = 512


def _boundary_sites(N):
    """Sites on tile edges (x0 = 63, 64, y = 7, 8) and z-chunk edges (z = 255, 256)."""
    out = []
    for x in (0, 63, 64, 511):
        for y in (0, 7, 8, 511):
            for z in (0, 255, 256, 511):
                out.append(x + N * (y + N * z))
    return np.array(out, dtype=np.int64)


@pytest.fixture
def bench_tiling():
    """The launch configuration the benchmark times: the recorded tuning table
    (cleared again afterwards, so that other tests see the defaults)."""
    import paper_2005_14454_amd as ah
    from paper_2005_14454_amd.tune import TABLE
    ah.tune_clear()
    ah.tune_load(TABLE)
    yield ah
    ah.tune_clear()


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-6), ("fp64", 1e-13)])
def test_fullsize_one_step_sampled(oracle_mod, bench_tiling, precision, tol):
    ah = bench_tiling
    op, gp = both_params(oracle_mod, N, precision, m=1.0)
    want = ah.tune_lookup(gp)
    with ah.Lattice(gp) as lat:
        cfg = lat.get_step_config()
        assert (cfg["kernel"], cfg["tile"], cfg["zchunk"]) == (want["kernel"], want["tile"], want["zchunk"]), (cfg, want)
        lat.init(1)
        lat.step(5)
        before = lat.get_state()
        lat.step(1)
        after = lat.get_state()
        meas = lat.measure()
        cfg = lat.get_step_config()
        w_sites = sample_sites(N, 3000, seed=17)
        w_gpu = lat.winding()[:, w_sites].T
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


def cube(N, site):
    """The 27 site indices of the 3x3x3 cube centred on `site`, in the index
    order of a 3^3 lattice (a + 3 (b + 3 c) for offsets a, b, c in 0..2)."""
    x0, x1, x2 = site % N, (site // N) % N, site // (N * N)
    out = []
    for c in range(3):
        for b in range(3):
            for a in range(3):
                out.append((x0 + a - 1) % N + N * (((x1 + b - 1) % N) + N * ((x2 + c - 1) % N)))
    return out


def test_fullsize_1024_matter_era_switch_sampled(oracle_mod):
    """1024^3 FP32, matter era (m = 2), s switching from 0 to 1 (moved to eta = 1.25
    so that the switch is inside the checked steps), a(eta_end = 256) = 1, seed 2:
    one GPU step after the switch against the oracle on sampled sites.  Each
    site's update reads only its 3x3x3 neighbourhood, which is gathered from the
    device and evaluated by the oracle as a 3^3 lattice (no wrap at its centre)."""
    import paper_2005_14454_amd as ah
    N = 1024
    gp = ah.Params(N=N, precision="fp32", m=2.0, s_early=0.0, s_late=1.0, eta_switch=1.25)
    op = oracle_mod.params(N=3, m=2.0, s_early=0.0, s_late=1.0, eta_switch=1.25, eta_ref=0.5 * 0.5 * N)
    rng = np.random.default_rng(31)
    centres = np.unique(np.concatenate([rng.integers(0, N ** 3, 300),
                                        [0, N - 1, N * N - 1, N ** 3 - 1, 127 + N * 7, 128 + N * 8]]))
    with ah.Lattice(gp) as lat:
        lat.init(2)
        lat.step(5)                          # eta = 1.5: s = 1, f = (1.5/256)^4
        cubes = np.array([cube(N, int(s)) for s in centres])
        before = lat.gather(cubes.reshape(-1)).reshape(len(centres), 27, 10)
        lat.step(1)
        after = lat.gather(centres)
        meas = lat.measure()
    ref = np.empty_like(after)
    for k in range(len(centres)):
        mini = np.ascontiguousarray(before[k].T)  # (10, 27)
        ref[k] = oracle_mod.step_sites(op, mini, 5, [13])[0]
    err = field_scaled_error(after.T, ref.T)
    print("1024^3 FP32 sampled one-step error", err)
    assert max(err.values()) <= 2e-6, err
    assert meas["nonfinite"] == 0 and meas["step"] == 6
    assert meas["winding_sum_abs"] > 0


def test_512_fp32_against_fp64_over_the_run():
    """512^3, radiation era, seed 1: the FP32 step against the FP64 step (whose
    parity with the oracle the tests above establish) after 100 steps, field
    by field over the whole lattice, within 1e-4 of each field's scale; then
    both to 1280 steps (eta = 129, half a light crossing) with the diagnostics
    at the end: Gauss's law holds to FP64 round-off on the FP64 lattice and to
    FP32 round-off on the FP32 one, and the two string lengths agree."""
    import paper_2005_14454_amd as ah
    lats = {prec: ah.Lattice(ah.Params(N=N, precision=prec, m=1.0)) for prec in ("fp32", "fp64")}
    try:
        for lat in lats.values():
            lat.init(1)
            lat.step(100)
        s64 = lats["fp64"].get_state()
        s32 = lats["fp32"].get_state()
        err = field_scaled_error(s32, s64)
        del s32, s64
        print("512^3 FP32 vs FP64 after 100 steps", err)
        assert max(err.values()) <= 1e-4, err
        end = {}
        for prec, lat in lats.items():
            lat.step(1180)
            end[prec] = lat.measure()
    finally:
        for lat in lats.values():
            lat.close()
    m32, m64 = end["fp32"], end["fp64"]
    ratio = m32["L_W"] / m64["L_W"]
    print("512^3 at step 1280: gauss_rel fp64 %.3e fp32 %.3e, L_W fp32/fp64 = %.5f (L_W fp64 %.1f)"
          % (m64["gauss_rel"], m32["gauss_rel"], ratio, m64["L_W"]))
    assert m64["step"] == m32["step"] == 1280
    assert m64["nonfinite"] == 0 and m32["nonfinite"] == 0
    assert m64["gauss_rel"] < 1e-12 and m32["gauss_rel"] < 1e-4
    assert m64["L_W"] > 0 and abs(ratio - 1.0) < 0.05


def test_1024_matter_era_core_growth_switch_full_run():
    """1024^3 FP32 (64 GB resident), matter era (m = 2), s = 0 until eta = 50
    and s = 1 after, a(eta_end = 257) = 1, seed 2: the whole 2560-step run with
    winding and velocity diagnostics every 20 steps.  The run stays finite and
    inside the leapfrog stability margin (the library never raises
    AH_FLAG_UNSTABLE), the network persists, Gauss's law holds to FP32
    round-off while s = 0 (s = 1 with m = 2 does not conserve the discrete
    constraint).  (After the switch the cores fatten, f drops to 1.4e-3, and
    the Lagrangian-weighted estimators, which assume thin cores, lose their
    meaning: sum_L can turn positive, xi_L is then NaN by definition.)"""
    import paper_2005_14454_amd as ah
    p = ah.Params(N=1024, precision="fp32", m=2.0, s_early=0.0, s_late=1.0, eta_switch=50.0)
    with ah.Lattice(p) as lat:
        lat.init(2)
        series = lat.step_measured(2560, 20) + [lat.measure()]
    for m in series[::8] + [series[-1]]:
        print("step %5d eta %6.1f f %.3e L_W %10.1f xi_W %7.3f xi_L %7.3f v2_phi %7.4f gauss_rel %.2e"
              % (m["step"], m["eta"], m["f"], m["L_W"], m["xi_W"], m["xi_L"], m["v2_phi"], m["gauss_rel"]))
    steps = [m["step"] for m in series]
    assert steps == list(range(0, 2561, 20))
    for m in series:
        assert m["nonfinite"] == 0 and m["flags"] == 0, m
    before = [m for m in series if m["eta"] < 50.0]
    assert max(m["gauss_rel"] for m in before) < 1e-4
    assert all(m["winding_sum_abs"] > 0 for m in series)


def test_beyond_2_31_sites_fp32_sampled(oracle_mod):
    """1300^3 FP32 (2.2e9 sites, past 2^31; 132 GB resident): every index of the
    path is 64-bit.  One step from a GPU-made snapshot against the oracle on
    sampled sites (each from its gathered 3x3x3 neighbourhood, as for 1024^3),
    including the sites whose flat index is just below and above 2^31 and the
    far corner."""
    import paper_2005_14454_amd as ah
    N = 1300
    gp = ah.Params(N=N, precision="fp32", m=1.0)
    op = oracle_mod.params(N=3, m=1.0, eta_ref=0.5 * 0.5 * N)
    rng = np.random.default_rng(41)
    special = [0, N ** 3 - 1, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + N * N - 1, N * N * (N - 1)]
    centres = np.unique(np.concatenate([rng.integers(0, N ** 3, 120), special]))
    with ah.Lattice(gp) as lat:
        lat.init(3)
        lat.step(2)
        cubes = np.array([cube(N, int(s)) for s in centres])
        before = lat.gather(cubes.reshape(-1)).reshape(len(centres), 27, 10)
        lat.step(1)
        after = lat.gather(centres)
        meas = lat.measure()
    ref = np.empty_like(after)
    for k in range(len(centres)):
        ref[k] = oracle_mod.step_sites(op, np.ascontiguousarray(before[k].T), 2, [13])[0]
    err = field_scaled_error(after.T, ref.T)
    print("1300^3 FP32 sampled one-step error", err)
    assert max(err.values()) <= 2e-6, err
    assert meas["nonfinite"] == 0 and meas["step"] == 3
    assert meas["gauss_rel"] < 1e-5 and meas["winding_sum_abs"] > 0
