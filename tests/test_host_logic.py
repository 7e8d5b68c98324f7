"""Host-side logic of the library that needs no GPU: parameter validation,
footprints, the stability margin behind AH_FLAG_UNSTABLE (checked against a
blow-up forced in the oracle), and the serving stream's request recipe."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def ah():
    import os
    import paper_2005_14454_amd as ah
    from paper_2005_14454_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2005_14454_amd import build
        build.build()
    return ah


def test_stability_margin_formula(ah):
    p = ah.Params(N=32)
    mu = ah.stability_margin(p, 0)
    assert abs(mu - 0.1 * math.sqrt(2.0 + 12.0 / 0.25)) < 1e-15
    # the paper's choices are stable; a large time step is not
    assert mu < 2.0
    assert ah.stability_margin(ah.Params(N=32, deta=0.29), 0) >= 2.0
    with pytest.raises(ah.AHError):
        ah.stability_margin(p, -1)


def test_stability_margin_predicts_blow_up(ah, oracle_mod):
    """Coupling f = a^(2s) grown past the margin makes the homogeneous mode of
    the oracle blow up; just below it, it stays bounded."""
    N = 4
    for f_scale, should_blow in ((150.0, False), (200.0, True)):
        # s = 1, slow expansion m = 0.01: f = (eta/eta_ref)^(2 m) equals f_scale at eta0
        # and grows by 8% over the 400 steps (eta from 1 to 41); damping is negligible
        m = 0.01
        eta_ref = f_scale ** (-1.0 / (2 * m))
        p = ah.Params(N=N, m=m, s_early=1.0, s_late=1.0, eta_ref=eta_ref)
        mu = ah.stability_margin(p, 0)
        assert (mu >= 2.0) == should_blow, (f_scale, mu)
        op = oracle_mod.params(N=N, m=m, s_early=1.0, s_late=1.0, eta_ref=eta_ref)
        st = np.zeros((10, N ** 3))
        st[0] = 1.0 + 1e-3 * np.cos(2 * np.pi * np.arange(N ** 3) / N)
        out = oracle_mod.step(op, st, 0, 400)
        blew = not np.all(np.isfinite(out)) or np.max(np.abs(out)) > 1e3
        assert blew == should_blow, (f_scale, mu, np.max(np.abs(out)))


def test_parameter_validation(ah):
    import ctypes
    from paper_2005_14454_amd import _lib
    lib = _lib.load()
    n = ctypes.c_size_t()
    good = ah.Params(N=16).to_c()
    assert lib.ah_required_bytes(ctypes.byref(good), ctypes.byref(n)) == 0
    for field, value in (("N", 3), ("precision", 7), ("gauge_action", 5), ("reserved", 1), ("dx", 0.0),
                         ("deta", -0.1), ("eta0", 0.0), ("e0", 0.0), ("lambda0", float("nan")),
                         ("damp_gamma", -1.0), ("damp_gamma", float("inf")), ("eta_damp", float("nan"))):
        bad = ah.Params(N=16).to_c()
        setattr(bad, field, value)
        assert lib.ah_required_bytes(ctypes.byref(bad), ctypes.byref(n)) == _lib.AH_E_INVAL, field


def test_pool_footprint_accounts_for_everything(ah):
    p32 = ah.Params(N=64, precision="fp32")
    p64 = ah.Params(N=64, precision="fp64")
    f32 = ah.pool_footprint(p32, 100, 10)
    f64 = ah.pool_footprint(p64, 100, 10)
    # 20 arrays: phi and A ping-pong, and Pi and E are double-buffered for the
    # two-step pass and the measured step
    assert 20 * 4 * 64 ** 3 < f32 < 20 * 4 * 64 ** 3 * 1.2
    assert 20 * 8 * 64 ** 3 < f64 < 20 * 8 * 64 ** 3 * 1.2
    assert ah.pool_footprint(p32, 1000, 10) > f32  # coefficient table and series grow with steps
    # rows are stored a whole number of 128-byte lines apart: 65 values take 96 (FP32) or 80 (FP64)
    assert ah.pool_footprint(ah.Params(N=65, precision="fp32"), 100, 10) > 20 * 4 * 65 * 65 * 96
    assert ah.pool_footprint(ah.Params(N=65, precision="fp64"), 100, 10) > 20 * 8 * 65 * 65 * 80
    with pytest.raises(ah.AHError):
        ah.pool_footprint(ah.Params(N=64, gauge_action="noncompact"), 10, 1)
    # a step count whose coefficient table could not be addressed is refused, not wrapped round
    for nsteps in (2 ** 62, 2 ** 63 - 1):
        with pytest.raises(ah.AHError):
            ah.pool_footprint(p32, nsteps, 10)


def test_request_stream_recipe(ah):
    from paper_2005_14454_amd.serve import make_stream, steps_to_half_light_crossing
    reqs = make_stream(200, rate=2.0, seed=5)
    fp32 = [r for r in reqs if r.params.precision == "fp32"]
    fp64 = [r for r in reqs if r.params.precision == "fp64"]
    assert len(fp32) == 200 and len(fp64) == 20
    Ns = np.array([r.params.N for r in fp32])
    assert Ns.min() >= 64 and Ns.max() <= 512
    # log-uniform: the median of N is near sqrt(64 * 512) = 181
    assert 140 < np.median(Ns) < 230
    assert {r.params.m for r in fp32} == {1.0, 2.0} and {r.params.s_early for r in fp32} == {0.0, 1.0}
    arr = np.array([r.arrival for r in fp32])
    assert np.all(np.diff(arr) > 0) and abs(np.mean(np.diff(arr)) - 0.5) < 0.1
    for r in fp64:
        twin = reqs[r.pair_of]
        assert twin.params.precision == "fp32" and twin.seed == r.seed and twin.params.N == r.params.N
    assert steps_to_half_light_crossing(256) == 630 and steps_to_half_light_crossing(512) == 1270


def test_tuning_table_roundtrip_and_validation(ah, tmp_path):
    """The autotuner's table (set, look up, save as JSON, load), host side; only
    supported tile shapes and z-chunks enter it, and a file with a bad entry
    changes nothing."""
    import json
    p32 = ah.Params(N=96, precision="fp32")
    p64 = ah.Params(N=40, precision="fp64")
    ah.tune_clear()
    try:
        assert ah.tune_lookup(p32) is None
        ah.tune_set(p32, (128, 8), 48)
        ah.tune_set(p64, (32, 8), 0)
        assert ah.tune_lookup(p32) == {"kernel": "tile", "tile": (128, 8), "zchunk": 48}
        assert ah.tune_lookup(p64) == {"kernel": "tile", "tile": (32, 8), "zchunk": 0}
        path = tmp_path / "tune.json"
        ah.tune_save(str(path))
        doc = json.loads(path.read_text())
        assert sorted((e["precision"], e["N"]) for e in doc["entries"]) == [("fp32", 96), ("fp64", 40)]
        ah.tune_clear()
        assert ah.tune_lookup(p32) is None and ah.tune_lookup(p64) is None
        ah.tune_load(str(path))
        assert ah.tune_lookup(p32)["tile"] == (128, 8) and ah.tune_lookup(p64)["tile"] == (32, 8)
        ah.tune_set(p32, (64, 8), 2)                     # short chunks are for lattices up to 128
        assert ah.tune_lookup(p32)["zchunk"] == 2
        p256 = ah.Params(N=256, precision="fp32")
        for bad in [(p64, (128, 8), 0), (p64, (64, 16), 0), (p32, (48, 8), 0), (p32, (64, 8), 1),
                    (p32, (64, 8), -1), (p256, (64, 8), 4)]:
            with pytest.raises(ah.AHError):
                ah.tune_set(*bad)
        assert ah.tune_lookup(p64)["tile"] == (32, 8)
        # two steps per pass: its own shapes (FP64 without 64 x 8), kept through save and load
        ah.tune_set(p32, (64, 8), 0, kernel="tile2")
        assert ah.tune_lookup(p32) == {"kernel": "tile2", "tile": (64, 8), "zchunk": 0}
        with pytest.raises(ah.AHError):
            ah.tune_set(p64, (64, 8), 0, kernel="tile2")
        with pytest.raises(ah.AHError):
            ah.tune_set(p32, (128, 8), 0, kernel="tile2")
        ah.tune_save(str(path))
        ah.tune_clear()
        ah.tune_load(str(path))
        assert ah.tune_lookup(p32)["kernel"] == "tile2" and ah.tune_lookup(p64)["kernel"] == "tile"
        badfile = tmp_path / "bad.json"
        badfile.write_text('{"version": 1, "entries": [\n'
                           '{"precision": "fp32", "N": 64, "tile_x": 64, "tile_y": 8, "zchunk": 0, "ms": 1},\n'
                           '{"precision": "fp32", "N": 80, "tile_x": 48, "tile_y": 8, "zchunk": 0, "ms": 1}\n]}\n')
        with pytest.raises(ah.AHError):
            ah.tune_load(str(badfile))
        assert ah.tune_lookup(ah.Params(N=64, precision="fp32")) is None
    finally:
        ah.tune_clear()


def test_scaling_fit_recovers_known_rates():
    """The scaling analysis fits a straight line over the eta window only and
    averages the velocity there; the isotropic winding rate is sqrt(3/2) times
    the printed one."""
    from paper_2005_14454_amd.scaling import analyse, mean_err
    series = []
    for k in range(0, 300):
        eta = 1.0 + 0.5 * k
        inside = 80.0 <= eta <= 128.0
        series.append({"eta": eta, "xi_L": 0.27 * eta + 3.0 if inside else 1e3,
                       "xi_W": 0.21 * eta - 1.0 if inside else -1e3,
                       "v2_phi": 0.268 if inside else 5.0, "v2_omega": 0.3 if inside else -5.0})
    f = analyse(series, (80.0, 128.0))
    assert f["points"] == 97
    assert abs(f["dxi_L"] - 0.27) < 1e-12 and abs(f["dxi_W"] - 0.21) < 1e-12
    assert abs(f["dxi_W_iso"] - 0.21 * math.sqrt(1.5)) < 1e-12
    assert abs(f["v2_phi"] - 0.268) < 1e-12 and abs(f["v2_omega"] - 0.3) < 1e-12
    mu, err = mean_err([1.0, 2.0, 3.0, 4.0])
    assert mu == 2.5 and abs(err - math.sqrt(5.0 / 3.0) / 2.0) < 1e-15
