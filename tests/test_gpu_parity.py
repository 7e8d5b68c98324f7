"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
identical seeded inputs.

Tolerances (field-scaled max norm per field, max over phi, Pi, A, E):
  one step from an identical FP64 snapshot      <= 1e-13
  64^3 radiation era, 100 steps, FP64            <= 1e-10, and <= the run's rounding
                                                 floor (what one ulp of phi in the start
                                                 grows to in the oracle by step 100)
  64^3 radiation era, 100 steps, FP32 vs FP64    <= 1e-4
  windings on identical snapshots                bit-exact
  FP64 diagnostics on identical snapshots        <= 1e-11 relative
"""
import math

import numpy as np
import pytest

from helpers import both_params, field_scaled_error, max_field_error, ulp_distance
from inputs import near_cut_state, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ah():
    import paper_2005_14454_amd as ah
    return ah


KERNELS = [("site", (0, 0), 0), ("tile", (64, 8), 0), ("tile", (64, 4), 8), ("tile", (32, 8), 9),
           ("tile", (128, 4), 16), ("tile", (64, 8), 2), ("tile", (32, 8), 3)]
KERNEL_IDS = ["site", "tile64x8", "tile64x4z8", "tile32x8z9", "tile128x4z16", "tile64x8z2", "tile32x8z3"]


def _run_gpu(ah, gp, state, step0, nsteps, kernel=None):
    with ah.Lattice(gp) as lat:
        if kernel is not None:
            lat.set_step_config(kernel[0], kernel[1], kernel[2])
        lat.set_state(state, step0)
        lat.step(nsteps)
        return lat.get_state()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_initial_condition_matches_oracle(oracle_mod, ah, precision):
    op, gp = both_params(oracle_mod, 20, precision, sigma=1.3)
    with ah.Lattice(gp) as lat:
        lat.init(1234)
        st = lat.get_state()
        assert lat.step_index == 0
    ref = oracle_mod.init(op, 1234)
    assert np.all(st[2:] == 0.0)
    if precision == "fp64":
        assert ulp_distance(st[:2], ref[:2]).max() <= 2.0
    else:
        r32 = ref[:2].astype(np.float32).astype(np.float64)
        assert np.max(np.abs(st[:2] - r32) / np.spacing(np.abs(r32).astype(np.float32)).astype(np.float64)) <= 1.0


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
@pytest.mark.parametrize("N", [4, 5, 20, 67])
@pytest.mark.parametrize("m,s", [(1.0, 0.0), (2.0, 1.0)])
def test_one_step_fp64(oracle_mod, ah, N, m, s, kernel):
    op, gp = both_params(oracle_mod, N, "fp64", m=m, s_early=s, s_late=s)
    st = random_state(N, seed=100 + N)
    got = _run_gpu(ah, gp, st, 3, 1, kernel)
    ref = oracle_mod.step(op, st, 3, 1)
    err = field_scaled_error(got, ref)
    print("one-step fp64", N, m, s, err)
    assert max(err.values()) <= 1e-13, err


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_artificial_damping_phase(oracle_mod, ah, precision, tol):
    """Random-phase start damped with friction 3 until eta = 3.05 (21 steps),
    then the radiation-era Hubble damping: 60 steps against the oracle, and the
    diagnostics of the last snapshot (Gauss's law stays exact for s = 0)."""
    op, gp = both_params(oracle_mod, 24, precision, m=1.0, damp_gamma=3.0, eta_damp=3.05)
    ic = oracle_mod.init(op, 4)
    ref = oracle_mod.step(op, ic, 0, 60)
    with ah.Lattice(gp) as lat:
        lat.set_state(ic, 0)
        lat.step(60)
        got = lat.get_state()
        gm = lat.measure()
    err = field_scaled_error(got, ref)
    print(f"damping phase {precision}: {err}")
    assert max(err.values()) <= tol, err
    om = oracle_mod.measure(op, got, 60)
    assert gm["winding_sum_abs"] == om["winding_sum_abs"]
    assert abs(gm["energy"] - om["energy"]) <= (1e-11 if precision == "fp64" else 1e-6) * om["energy"]
    assert gm["gauss_rel"] < (1e-12 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_core_growth_negative_s(oracle_mod, ah, precision, tol):
    """s = -1 (the cores grow with a, the paper's option for resolving them
    early) switching to s = 1 at eta = 3, radiation era, 40 steps from the
    random-phase IC, against the oracle."""
    N = 24
    op, gp = both_params(oracle_mod, N, precision, m=1.0, s_early=-1.0, s_late=1.0, eta_switch=3.0, eta_ref=2.0)
    ic = oracle_mod.init(op, 9)
    with ah.Lattice(gp) as lat:
        lat.set_state(ic, 0)
        lat.step(40)
        got = lat.get_state()
    ref = oracle_mod.step(op, ic, 0, 40)
    err = field_scaled_error(got, ref)
    print("core growth", precision, err)
    assert max(err.values()) <= tol, err


@pytest.mark.parametrize("gauge", ["compact", "noncompact"])
def test_one_step_gauge_actions(oracle_mod, ah, gauge):
    N = 12
    op, gp = both_params(oracle_mod, N, "fp64", gauge_action=gauge)
    st = random_state(N, seed=7, a_amp=2.0)
    got = _run_gpu(ah, gp, st, 0, 1)
    ref = oracle_mod.step(op, st, 0, 1)
    assert max_field_error(got, ref) <= 1e-13


@pytest.mark.parametrize("kernel", KERNELS + [("tile", (64, 16), 0), ("tile", (128, 8), 0)],
                         ids=KERNEL_IDS + ["tile64x16", "tile128x8"])
@pytest.mark.parametrize("N", [24, 70])
def test_one_step_fp32(oracle_mod, ah, N, kernel):
    op, gp = both_params(oracle_mod, N, "fp32")
    st = random_state(N, seed=3).astype(np.float32).astype(np.float64)
    got = _run_gpu(ah, gp, st, 2, 1, kernel)
    ref = oracle_mod.step(op, st, 2, 1)
    err = field_scaled_error(got, ref)
    print("one-step fp32", err)
    assert max(err.values()) <= 2e-6, err


@pytest.fixture(scope="module")
def config1_reference(oracle_mod):
    """64^3 radiation era, s = 0, random-phase IC from seed 0, 100 oracle steps."""
    op = oracle_mod.params(N=64, m=1.0)
    ic = oracle_mod.init(op, 0)
    return op, ic, oracle_mod.step(op, ic, 0, 100)


@pytest.fixture(scope="module")
def config1_rounding_floor(oracle_mod):
    """What one ulp of phi in the start grows to by step 100 of the same run."""
    from helpers import rounding_floor
    return max(rounding_floor(oracle_mod).values())


@pytest.mark.parametrize("kernel", ["site", "tile"])
def test_config1_fp64_100_steps(oracle_mod, ah, config1_reference, config1_rounding_floor, kernel):
    op, ic, ref = config1_reference
    _, gp = both_params(oracle_mod, 64, "fp64", m=1.0)
    with ah.Lattice(gp) as lat:
        lat.set_step_config(kernel)
        lat.set_state(ic, 0)
        for _ in range(10):
            lat.step(10)
        got = lat.get_state()
        err = field_scaled_error(got, ref)
        print(f"config1 fp64 100 steps {err}; rounding floor of the run {config1_rounding_floor:.2e}, "
              f"ratio {max(err.values()) / config1_rounding_floor:.1f}")
        assert max(err.values()) <= 1e-10, err
        # and no further from the oracle than the oracle is from itself after a one-ulp change of the start
        assert max(err.values()) <= config1_rounding_floor, (err, config1_rounding_floor)
        # diagnostics of the GPU snapshot against the oracle on the same snapshot
        gm = lat.measure()
        om = oracle_mod.measure(op, got, 100)
        assert gm["winding_sum_abs"] == om["winding_sum_abs"]
        for k in ("energy", "e_kin", "e_grad", "e_pot", "e_el", "e_mag", "sum_L", "xi_L", "R", "v2_phi", "v2_omega",
                  "xi_W"):
            assert abs(gm[k] - om[k]) <= 1e-11 * abs(om[k]), (k, gm[k], om[k])
        assert gm["gauss_rel"] < 1e-12 and om["gauss_rel"] < 1e-12
        assert gm["nonfinite"] == 0 and gm["flags"] == 0
        assert gm["step"] == 100 and abs(gm["eta"] - 11.0) < 1e-12
        assert np.array_equal(lat.winding(), oracle_mod.winding(op, got).astype(np.int8))


def test_config0_series_fp64_fused(oracle_mod, ah):
    """64^3 FP64 radiation era, seed 0, 160 steps with the diagnostics every 10
    steps formed in the same pass as the step (ah_step_measured): every record
    against the oracle's diagnostics of its own snapshot at that step."""
    op, gp = both_params(oracle_mod, 64, "fp64", m=1.0)
    with ah.Lattice(gp) as lat:
        lat.init(0)
        series = lat.step_measured(160, 10) + [lat.measure()]
    assert [m["step"] for m in series] == list(range(0, 161, 10))
    st = oracle_mod.init(op, 0)
    for k, gm in enumerate(series):
        n = 10 * k
        if n > 0:
            st = oracle_mod.step(op, st, n - 10, 10)
        om = oracle_mod.measure(op, st, n)
        assert gm["winding_sum_abs"] == om["winding_sum_abs"], n
        for key in ("energy", "e_kin", "e_grad", "e_pot", "e_el", "e_mag", "sum_L", "R", "v2_omega"):
            assert abs(gm[key] - om[key]) <= 1e-9 * abs(om[key]) + 1e-12, (n, key, gm[key], om[key])
        assert gm["gauss_rel"] < 1e-12 and om["gauss_rel"] < 1e-12, n
        assert gm["nonfinite"] == 0 and gm["flags"] == 0


@pytest.mark.parametrize("kernel", ["site", "tile"])
def test_config1_fp32_100_steps(oracle_mod, ah, config1_reference, kernel):
    op, ic, ref = config1_reference
    _, gp = both_params(oracle_mod, 64, "fp32", m=1.0)
    with ah.Lattice(gp) as lat:
        lat.set_step_config(kernel)
        lat.set_state(ic, 0)
        lat.step(100)
        got = lat.get_state()
        err = field_scaled_error(got, ref)
        print("config1 fp32 vs fp64 oracle, 100 steps", err)
        assert max(err.values()) <= 1e-4, err
        # windings bit-exact on the identical (FP32) snapshot, computed in FP64 on both sides
        assert np.array_equal(lat.winding(), oracle_mod.winding(op, got).astype(np.int8))
        # site densities in FP32, sums in FP64: relative to the energy scale
        gm = lat.measure()
        om = oracle_mod.measure(op, got, 100)
        assert gm["winding_sum_abs"] == om["winding_sum_abs"]
        scale = sum(om[k] for k in ("e_kin", "e_grad", "e_pot", "e_el", "e_mag"))
        for k in ("energy", "e_kin", "e_grad", "e_pot", "e_el", "e_mag", "sum_L"):
            assert abs(gm[k] - om[k]) <= 1e-6 * scale, (k, gm[k], om[k])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_measure_on_random_snapshot(oracle_mod, ah, precision):
    N = 20
    op, gp = both_params(oracle_mod, N, precision, m=2.0)
    st = random_state(N, seed=77)
    if precision == "fp32":
        st = st.astype(np.float32).astype(np.float64)
    with ah.Lattice(gp) as lat:
        lat.set_state(st, 5)
        gm = lat.measure()
        w = lat.winding()
    om = oracle_mod.measure(op, st, 5)
    assert gm["winding_sum_abs"] == om["winding_sum_abs"]
    assert np.array_equal(w, oracle_mod.winding(op, st).astype(np.int8))
    # FP64 lattices: everything FP64.  FP32 lattices: site densities in FP32
    # (relative to the energy scale), Gauss residual from exactly widened
    # values in FP64.
    scale = sum(om[k] for k in ("e_kin", "e_grad", "e_pot", "e_el", "e_mag"))
    tol_e = 1e-11 if precision == "fp64" else 1e-6
    for k in ("energy", "e_kin", "e_grad", "e_pot", "e_el", "e_mag", "sum_L"):
        assert abs(gm[k] - om[k]) <= tol_e * scale, (k, gm[k], om[k])
    assert abs(gm["R"] - om["R"]) <= (1e-11 if precision == "fp64" else 1e-4) * abs(om["R"])
    # the equation-of-state velocity: ratio of L-weighted sums, w = (2 v^2 - 1)/3
    assert abs(gm["v2_omega"] - om["v2_omega"]) <= (1e-11 if precision == "fp64" else 1e-4) * max(1.0, abs(om["v2_omega"]))
    for k in ("gauss_rms", "gauss_max", "gauss_rel"):
        assert abs(gm[k] - om[k]) <= 1e-11 * abs(om[k]), (k, gm[k], om[k])


@pytest.mark.parametrize("tile", [(64, 8), (32, 8), (64, 4)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_windings_on_decision_boundaries(oracle_mod, ah, precision, tile):
    """Link phases within ~1e-4 of the cut at +-pi, |dx A| up to ~6e3 and
    plaquette angles on half turns: every winding still equals the oracle's,
    in the fused diagnostics pass (several tiles, halo columns) and in the
    winding field."""
    N = 40
    op, gp = both_params(oracle_mod, N, precision)
    st = near_cut_state(N, seed=8, dx=op["dx"])
    if precision == "fp32":
        st = st.astype(np.float32).astype(np.float64)
    with ah.Lattice(gp) as lat:
        lat.set_step_config("tile", tile, 0)
        lat.set_state(st, 3)
        gm = lat.measure()
        w = lat.winding()
    om = oracle_mod.measure(op, st, 3)
    wo = oracle_mod.winding(op, st)
    assert np.count_nonzero(wo) > 0
    assert gm["winding_sum_abs"] == om["winding_sum_abs"]
    assert np.array_equal(w, wo.astype(np.int8))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_windings_with_zero_phi_sites(oracle_mod, ah, precision):
    """Degenerate link phases: phi exactly zero (of either sign) at 10% of the
    sites, so z = conj(phi) U phi' is a signed zero and the phase follows the
    definition's convention for atan2(0, +-0); windings and their sum equal
    the oracle's."""
    N = 24
    op, gp = both_params(oracle_mod, N, precision)
    st = random_state(N, seed=19)
    rng = np.random.default_rng(20)
    zero = rng.random(N ** 3) < 0.1
    neg = rng.random(N ** 3) < 0.5
    st[0, zero] = np.where(neg[zero], -0.0, 0.0)
    st[1, zero] = np.where(neg[zero], 0.0, -0.0)
    if precision == "fp32":
        st = st.astype(np.float32).astype(np.float64)
    with ah.Lattice(gp) as lat:
        lat.set_state(st, 2)
        gm = lat.measure()
        w = lat.winding()
    om = oracle_mod.measure(op, st, 2)
    assert gm["winding_sum_abs"] == om["winding_sum_abs"]
    assert np.array_equal(w, oracle_mod.winding(op, st).astype(np.int8))


def test_deterministic_and_resumable(ah):
    from paper_2005_14454_amd import Params
    gp = Params(N=32, m=1.0)
    with ah.Lattice(gp) as a:
        a.init(5)
        a.step(30)
        full = a.get_state()
        ma = a.measure()
    with ah.Lattice(gp) as b:
        b.init(5)
        b.step(15)
        mid = b.get_state()
    with ah.Lattice(gp, arena="library") as c:
        c.set_state(mid, 15)
        c.step(15)
        resumed = c.get_state()
        mc = c.measure()
    assert np.array_equal(full, resumed)
    assert ma == mc


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_dump_and_restore(oracle_mod, ah, tmp_path, precision):
    """A dump holds the snapshot exactly (storage precision) with its windings,
    and a lattice restored from it continues bitwise like the original."""
    from paper_2005_14454_amd import Params, read_dump
    gp = Params(N=20, precision=precision, m=2.0)
    path = str(tmp_path / "snap.npz")
    with ah.Lattice(gp) as a:
        a.init(9)
        a.step(12)
        a.dump(path)
        st = a.get_state()
        a.step(5)
        after = a.get_state()
    d = read_dump(path)
    assert d["step"] == 12 and d["params"] == gp
    assert d["fields"].dtype == (np.float32 if precision == "fp32" else np.float64)
    assert np.array_equal(d["fields"].astype(np.float64), st)
    op = oracle_mod.params(N=20, m=2.0)
    assert np.array_equal(d["windings"], oracle_mod.winding(op, st).astype(np.int8))
    with ah.Lattice(gp) as b:
        b.restore(path)
        assert b.step_index == 12
        b.step(5)
        assert np.array_equal(b.get_state(), after)


def test_errors_and_edge_cases(ah):
    from paper_2005_14454_amd import Params, _lib
    with pytest.raises(ah.AHError):
        ah.Lattice(Params(N=3))
    with ah.Lattice(Params(N=8)) as lat:
        with pytest.raises(ah.AHError) as ei:
            lat.step(1)
        assert ei.value.code == _lib.AH_E_STATE
        lat.init(1)
        before = lat.get_state()
        lat.step(0)
        assert np.array_equal(before, lat.get_state())
        with pytest.raises(ah.AHError):
            lat.step(-1)
        with pytest.raises(ValueError):
            lat.set_state(np.zeros(5))


def test_vacuum_bitwise_static_on_gpu(ah):
    from paper_2005_14454_amd import Params
    for prec in ("fp64", "fp32"):
        gp = Params(N=9, precision=prec, m=2.0)
        st = np.zeros((10, 9 ** 3))
        st[0] = 1.0
        with ah.Lattice(gp) as lat:
            lat.set_state(st, 0)
            lat.step(20)
            assert np.array_equal(lat.get_state(), st)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tile_shapes_bitwise_identical(ah, precision):
    """Every tile shape and z-chunk computes each site with the same expression
    tree from the same inputs, so the fields agree bit for bit."""
    from paper_2005_14454_amd import Params
    N = 40
    gp = Params(N=N, precision=precision, m=2.0)
    st = random_state(N, seed=9)
    shapes = [((64, 8), 0), ((64, 4), 8), ((32, 8), 9), ((64, 8), 40), ((32, 8), 13), ((128, 4), 8),
              ((64, 8), 2), ((32, 8), 3), ((64, 4), 5)]
    if precision == "fp32":
        shapes += [((64, 16), 11), ((128, 8), 10)]
    outs = [_run_gpu(ah, gp, st, 0, 12, ("tile", t, z)) for t, z in shapes]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    again = _run_gpu(ah, gp, st, 0, 12, ("tile", (64, 8), 0))
    assert np.array_equal(again, outs[0])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("zchunk", [2, 3])
def test_short_chunks_diagnostics_vs_oracle(oracle_mod, ah, precision, zchunk):
    """Two- and three-plane z-chunks (N = 20: a ragged last chunk for 3) in the
    measured march, which completes each chunk's windings at its last plane:
    the diagnostics of a generic snapshot and of a fused series against the
    oracle."""
    N = 20
    op, gp = both_params(oracle_mod, N, precision, m=1.0)
    tile = (32, 8) if precision == "fp64" else (64, 8)
    st = random_state(N, seed=31)
    if precision == "fp32":
        st = st.astype(np.float32).astype(np.float64)
    with ah.Lattice(gp) as lat:
        lat.set_step_config("tile", tile, zchunk)
        assert lat.get_step_config()["zchunk"] == zchunk
        lat.set_state(st, 4)
        gm = lat.measure()
        assert np.array_equal(lat.winding(), oracle_mod.winding(op, st).astype(np.int8))
        lat.init(6)
        series = lat.step_measured(10, 5) + [lat.measure()]
        got = lat.get_state()
    om = oracle_mod.measure(op, st, 4)
    scale = sum(om[k] for k in ("e_kin", "e_grad", "e_pot", "e_el", "e_mag"))
    tol = 1e-11 if precision == "fp64" else 1e-6
    assert gm["winding_sum_abs"] == om["winding_sum_abs"]
    for k in ("energy", "e_kin", "e_grad", "e_pot", "e_el", "e_mag", "sum_L"):
        assert abs(gm[k] - om[k]) <= tol * scale, (k, gm[k], om[k])
    ref = oracle_mod.init(op, 6)
    for k, m in enumerate(series):
        n = 5 * k
        if n > 0:
            ref = oracle_mod.step(op, ref, n - 5, 5)
        assert m["step"] == n
        if precision == "fp64":
            om = oracle_mod.measure(op, ref, n)
            assert m["winding_sum_abs"] == om["winding_sum_abs"], n
            assert abs(m["energy"] - om["energy"]) <= 1e-9 * om["energy"], n
    assert max(field_scaled_error(got, ref).values()) <= (1e-10 if precision == "fp64" else 1e-4)


def test_default_kernel_choice(ah):
    from paper_2005_14454_amd import Params
    with ah.Lattice(Params(N=16)) as lat:
        assert lat.get_step_config()["kernel"] == "tile"
    with ah.Lattice(Params(N=16, gauge_action="noncompact")) as lat:
        assert lat.get_step_config()["kernel"] == "site"
        with pytest.raises(ah.AHError):
            lat.set_step_config("tile")
    with ah.Lattice(Params(N=16, precision="fp64")) as lat:
        with pytest.raises(ah.AHError):
            lat.set_step_config("tile", (64, 16))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_diagnostics_equal_separate_pass(ah, precision):
    """ah_step_measured forms the diagnostics of each due snapshot in the pass
    that steps it: the fields are bitwise those of plain steps and the records
    bitwise those of ah_measure on the same snapshots."""
    from paper_2005_14454_amd import Params
    N = 48
    gp = Params(N=N, precision=precision, m=2.0, s_early=0.0, s_late=1.0, eta_switch=2.05)
    with ah.Lattice(gp) as a, ah.Lattice(gp) as b:
        a.init(21)
        b.init(21)
        fused = a.step_measured(25, 5)
        separate = []
        for k in range(25):
            if k % 5 == 0:
                separate.append(b.measure())
            b.step(1)
        assert np.array_equal(a.get_state(), b.get_state())
        assert [m["step"] for m in fused] == [0, 5, 10, 15, 20]
        for x, y in zip(fused, separate):
            for key in x:
                assert x[key] == y[key] or (x[key] != x[key] and y[key] != y[key]), key
        # the tail: 3 more steps from step 25 measure snapshot 25 only
        more = a.step_measured(3, 5)
        assert [m["step"] for m in more] == [25]


@pytest.mark.parametrize("precision,kernel,tile,zchunk", [
    ("fp32", "tile", (64, 8), 0), ("fp32", "tile", (64, 8), 3), ("fp32", "tile", (64, 8), 37),
    ("fp32", "tile2", (64, 8), 5), ("fp64", "tile", (64, 8), 0), ("fp64", "tile", (32, 8), 3),
    ("fp64", "tile2", (32, 8), 5)])
def test_gauss_in_measured_march(oracle_mod, ah, precision, kernel, tile, zchunk):
    """The measured march forms the Gauss residual: E_x, E_y of the -x / -y
    neighbours (FP32 through LDS with the -x column and -y row of the halo,
    FP64 loaded with the plane's Pi and E and summed per wave and plane), E_z
    of the plane below carried in a register and loaded afresh at each
    z-chunk's first plane; a measured step then writes Pi and E into the
    other buffer.  N = 37 gives ragged x and y tiles; the norms on a
    Gauss-violating random snapshot against the oracle, the series of
    measured steps (every step, then every third) against the oracle's norms
    of its own snapshots, and the fields after them (with a two-step pass
    between the measured steps 9 and 12 for kernel tile2)."""
    N = 37
    op, gp = both_params(oracle_mod, N, precision, m=2.0)
    st = random_state(N, seed=91)
    if precision == "fp32":
        st = st.astype(np.float32).astype(np.float64)
    with ah.Lattice(gp) as lat:
        lat.set_step_config(kernel, tile, zchunk)
        lat.set_state(st, 5)
        gm = lat.measure()
        series = lat.step_measured(3, 1) + lat.step_measured(6, 3)
        got = lat.get_state()
    om = oracle_mod.measure(op, st, 5)
    assert om["gauss_rel"] > 0.1  # a random snapshot violates the constraint
    for k in ("gauss_rms", "gauss_max", "gauss_rel"):
        assert abs(gm[k] - om[k]) <= 1e-11 * abs(om[k]), (k, gm[k], om[k])
    assert [m["step"] for m in series] == [5, 6, 7, 9, 12]
    assert all(series[0][k] == gm[k] for k in ("gauss_rms", "gauss_max", "gauss_rel", "energy"))
    # FP32: the snapshots differ from the oracle's by FP32 rounding (relative
    # ~1e-6 after these few steps) and the norms follow them
    tol = 1e-10 if precision == "fp64" else 1e-4
    ref = st
    for m in series:
        n = m["step"]
        if n > 5:
            ref = oracle_mod.step(op, ref, prev, n - prev)
        prev = n
        on = oracle_mod.measure(op, ref, n)
        for k in ("gauss_rms", "gauss_max", "gauss_rel"):
            assert abs(m[k] - on[k]) <= tol * abs(on[k]), (n, k, m[k], on[k])
    ref = oracle_mod.step(op, ref, prev, 14 - prev)
    assert max(field_scaled_error(got, ref).values()) <= (1e-10 if precision == "fp64" else 1e-4)
