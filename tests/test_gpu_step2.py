"""Two steps per pass (kernel "tile2"): the temporally blocked z-march forms
step n -> n+1 on the tile plus a one-site ring in LDS and step n+1 -> n+2
on the tile from it.  Every site goes through the same arithmetic as the
single-step march, so any sequence of steps is bitwise the one the
single-step kernel gives: even and odd step counts, ragged tiles, short
z-chunks, coefficients that change from step to step (expansion, an s
switch, a damping phase), fused diagnostics in between, and state I/O
after a pass has swapped the Pi/E buffers.
"""
import numpy as np
import pytest

from helpers import both_params, field_scaled_error
from inputs import random_state, sample_sites

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ah():
    import paper_2005_14454_amd as ah
    return ah


def _params(ah, N, precision):
    # m = 2 with an s switch and a damping phase inside the run: every step
    # has its own kick coefficients, so a pass that used one step's for both
    # would show
    return ah.Params(N=N, precision=precision, m=2.0, s_early=0.0, s_late=1.0, eta_switch=1.45,
                     damp_gamma=2.0, eta_damp=1.25, eta_ref=3.0)


def _run(ah, gp, st, step0, nsteps, kernel, tile=(0, 0), zchunk=0):
    with ah.Lattice(gp) as lat:
        lat.set_step_config(kernel, tile, zchunk)
        lat.set_state(st, step0)
        lat.step(nsteps)
        return lat.get_state()


CASES = [((32, 8), 0), ((64, 4), 0), ((32, 8), 2), ((64, 4), 3), ((32, 8), 7), ((64, 8), 0), ((64, 8), 5)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [4, 5, 20, 37, 70])
def test_two_step_bitwise_equals_single_steps(ah, precision, N):
    gp = _params(ah, N, precision)
    st = random_state(N, seed=100 + N)
    if precision == "fp32":
        st = st.astype(np.float32).astype(np.float64)
    want = _run(ah, gp, st, 1, 7, "tile", (32, 8), 0)
    for tile, zc in CASES:
        if precision == "fp64" and tile == (64, 8):
            continue
        if zc > N or (zc and zc < 8 and N > 128):
            continue
        got = _run(ah, gp, st, 1, 7, "tile2", tile, zc)
        assert np.array_equal(got, want), (precision, N, tile, zc)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
def test_two_step_against_oracle(oracle_mod, ah, precision, tol):
    N = 24
    op, gp = both_params(oracle_mod, N, precision, m=1.0)
    st = random_state(N, seed=5)
    if precision == "fp32":
        st = st.astype(np.float32).astype(np.float64)
    got = _run(ah, gp, st, 3, 6, "tile2")
    ref = oracle_mod.step(op, st, 3, 6)
    err = max(field_scaled_error(got, ref).values())
    assert err <= tol, err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_step_measured_series_and_state_io(ah, precision):
    """Fused diagnostics every 5 steps split the plain steps into two pairs;
    the series and fields equal the single-step kernel's.  After an odd
    number of steps (Pi/E in the second buffer) downloads, gathers, uploads
    and continued steps see the current snapshot."""
    N = 36
    gp = _params(ah, N, precision)
    tile = (32, 8)
    runs = {}
    for kernel in ("tile", "tile2"):
        with ah.Lattice(gp) as lat:
            lat.set_step_config(kernel, tile, 0)
            lat.init(7)
            series = lat.step_measured(23, 5)
            st = lat.get_state()
            sites = sample_sites(N, 200, seed=3)
            assert np.array_equal(lat.gather(sites), st[:, sites].T)
            assert np.array_equal(lat.gather_noalloc(sites), st[:, sites].T)
            lat.step(3)
            after = lat.get_state()
            lat.set_state(st, 23)
            lat.step(3)
            assert np.array_equal(lat.get_state(), after)
            w = lat.winding()
            m = lat.measure()
        runs[kernel] = (series, st, after, w, m)
    a, b = runs["tile"], runs["tile2"]
    assert [r["step"] for r in a[0]] == [0, 5, 10, 15, 20]
    for x, y in zip(a[0], b[0]):
        assert x == y or all((x[k] == y[k]) or (x[k] != x[k] and y[k] != y[k]) for k in x), (x, y)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_two_step_timing_counts_steps(ah):
    gp = ah.Params(N=32, precision="fp32", m=1.0)
    with ah.Lattice(gp) as lat:
        lat.set_step_config("tile2", (32, 8), 0)
        lat.init(1)
        lat.set_timing(True)
        lat.step(5)
        ms, n = lat.get_timing()
        assert n == 5 and ms > 0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_two_step_full_size_512_sampled(ah, precision):
    """The 512^3 benchmark lattice: four steps as two passes against four
    single steps, bitwise at 65536 sampled sites (the lattice is too large to
    download twice)."""
    N = 512
    gp = ah.Params(N=N, precision=precision, m=1.0)
    sites = sample_sites(N, 65536 - 8, seed=11)
    got = {}
    for kernel, tile in (("tile", (32, 8)), ("tile2", (32, 8))):
        with ah.Lattice(gp) as lat:
            lat.set_step_config(kernel, tile, 0)
            lat.init(1)
            lat.step(4)
            got[kernel] = lat.gather(sites)
    assert np.array_equal(got["tile"], got["tile2"])
    assert np.all(np.isfinite(got["tile2"]))
