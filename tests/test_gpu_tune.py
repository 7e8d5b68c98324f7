"""The autotuner: it times the tiled step's tile shapes and z-chunks, with one
and with two steps per pass, for a (precision, N), records the fastest per
step, and lattices created afterwards with automatic configuration use it.
Every tile shape and kernel computes the same fields bit for bit, so a
tuned lattice evolves exactly as an untuned one."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPES = {(64, 8), (64, 4), (32, 8), (128, 4), (64, 16), (128, 8)}
SHAPES2 = {(32, 8), (64, 4), (64, 8)}  # two steps per pass


@pytest.fixture
def ah():
    import paper_2005_14454_amd as ah
    ah.tune_clear()
    yield ah
    ah.tune_clear()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_autotune_records_and_is_used(ah, precision):
    p = ah.Params(N=48, precision=precision)
    best = ah.autotune(p, steps=2)
    assert best["kernel"] in ("tile", "tile2") and best["ms"] > 0
    assert tuple(best["tile"]) in (SHAPES if best["kernel"] == "tile" else SHAPES2)
    if precision == "fp64":
        assert tuple(best["tile"]) not in {(64, 16), (128, 8)}
        assert best["kernel"] == "tile" or tuple(best["tile"]) != (64, 8)
    assert 2 <= best["zchunk"] <= 48
    assert ah.tune_lookup(p)["tile"] == best["tile"]
    with ah.Lattice(p) as lat:
        cfg = lat.get_step_config()
        assert (cfg["kernel"], cfg["tile"], cfg["zchunk"]) == (best["kernel"], best["tile"], best["zchunk"])
        lat.init(3)
        lat.step(4)
        tuned = lat.get_state()
    ah.tune_clear()
    with ah.Lattice(p) as lat:
        lat.init(3)
        lat.step(4)
        assert np.array_equal(lat.get_state(), tuned)


def test_tuned_automatic_zchunk_is_resolved(ah):
    p = ah.Params(N=40, precision="fp32")
    ah.tune_set(p, (64, 4), 0)
    with ah.Lattice(p) as lat:
        cfg = lat.get_step_config()
        assert cfg["tile"] == (64, 4) and 2 <= cfg["zchunk"] <= 40
        lat.init(5)
        lat.step(3)
        m = lat.measure()
    assert m["nonfinite"] == 0 and m["step"] == 3


def test_hbm_probe_is_plausible(ah):
    """The bandwidth probe reports rates that a device can reach: above 1 TB/s
    and not above the nominal 8 TB/s HBM peak (with a margin for timing)."""
    out = ah.hbm_probe(1 << 30, 3)
    for k in ("copy_GB/s", "read_GB/s", "write_GB/s"):
        assert 1000.0 < out[k] < 8400.0, out
    with pytest.raises(ah.AHError):
        ah.hbm_probe(1000, 1)
