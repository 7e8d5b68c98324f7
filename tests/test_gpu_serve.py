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


def test_served_request_and_its_fp64_rerun_match_the_oracle(oracle_mod):
    """A served FP32 request and its FP64 rerun, taken from a stream that
    shares the pool with other requests, against the oracle's evolution of
    the same lattice from the same seed: every diagnostics snapshot of the
    FP64 rerun has the oracle's windings and its energies to 1e-10; the FP32
    request's energies are within 1e-4 of the oracle's and its string length
    within 1e-3."""
    from paper_2005_14454_amd.serve import make_stream, run_stream
    from helpers import both_params
    reqs = make_stream(3, rate=200.0, seed=12, nmin=16, nmax=28, fp64_every=3, measure_every=10)
    out = run_stream(reqs, hbm_budget=1 << 30, max_slots=2, chunk=2)
    assert out["requests"] == len(reqs) == 4 and out["fp64_spot_checks"] == 1
    r64 = next(r for r in reqs if r.params.precision == "fp64")
    r32 = reqs[r64.pair_of]
    assert (r32.params.N, r32.seed, r32.nsteps) == (r64.params.N, r64.seed, r64.nsteps)
    p = r64.params
    op, _ = both_params(oracle_mod, p.N, "fp64", m=p.m, s_early=p.s_early, s_late=p.s_late)
    st = oracle_mod.init(op, r64.seed)
    k = 0
    ref = []
    for rec in r64.series:
        st = oracle_mod.step(op, st, k, rec["step"] - k)
        k = rec["step"]
        ref.append(oracle_mod.measure(op, st, k))
    assert [m["step"] for m in ref] == [m["step"] for m in r32.series]
    for a, b, o in zip(r64.series, r32.series, ref):
        assert a["winding_sum_abs"] == o["winding_sum_abs"], a["step"]
        assert abs(a["energy"] - o["energy"]) <= 1e-10 * abs(o["energy"]), a["step"]
        assert abs(b["energy"] - o["energy"]) <= 1e-4 * abs(o["energy"]), b["step"]
        if o["winding_sum_abs"] > 0:
            assert abs(b["L_W"] - o["L_W"]) <= 1e-3 * o["L_W"], b["step"]
