"""The serving loop: a Poisson stream of requests shares one GPU through the
lattice pool.  With fewer slots than requests, later requests wait and are
admitted while earlier ones are still running (they join the same per-step
graph replay); every result is bitwise the one the same lattice gives when
run alone with the same tiling."""
import numpy as np
import pytest

from helpers import run_alone, same_record

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    from paper_2005_14454_amd.serve import make_stream, run_stream
    reqs = make_stream(8, rate=200.0, seed=11, nmin=16, nmax=40, fp64_every=4, measure_every=5)
    out = run_stream(reqs, hbm_budget=1 << 30, max_slots=3, chunk=2)
    assert out["requests"] == len(reqs) == 10
    for r in reqs:
        assert r.arrival <= r.admitted <= r.done
        assert len(r.series) == r.nsteps // r.measure_every + 1 + (r.nsteps % r.measure_every != 0)
    # continuous batching: some request was admitted while another was running
    assert any(a.admitted > b.admitted and a.admitted < b.done for a in reqs for b in reqs if a is not b)
    assert out["ttc_p99_s"] >= out["ttc_p50_s"] > 0
    assert out["fp64_spot_checks"] == 2 and out["fp32_vs_fp64_snapshots_compared"] > 0
    for r in reqs:
        _, ser = run_alone(r.params, r.seed, r.nsteps, r.measure_every, r.step_config["tile"],
                           r.step_config["zchunk"])
        assert len(ser) == len(r.series)
        for a, b in zip(r.series, ser):
            assert same_record(a, b), (r.rid, r.params.N, a["step"])
