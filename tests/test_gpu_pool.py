"""The lattice pool (batched persistent step, continuous batching).

- every lattice advanced in the pool is bitwise identical, fields and
  diagnostics series, to the same lattice run alone through ah_step/ah_measure
  with the same tile shape;
- a pool lattice matches the oracle;
- admission by footprint: requests that do not fit now are refused with
  AH_E_AGAIN (submit returns None), requests larger than the budget raise;
- lattices of different lengths finish at different steps and are reported
  once each; memory returns to the pool.
"""
import numpy as np
import pytest

from helpers import both_params, field_scaled_error, run_alone, same_record

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ah():
    import paper_2005_14454_amd as ah
    return ah


def test_pool_alone_vs_mix_bitwise(ah):
    from paper_2005_14454_amd import Params
    reqs = [
        (Params(N=16, precision="fp32", m=1.0), 11, 25, 5),
        (Params(N=40, precision="fp64", m=2.0), 12, 18, 6),
        (Params(N=24, precision="fp32", m=2.0, s_early=1.0, s_late=1.0), 13, 30, 10),
        (Params(N=64, precision="fp32", m=1.0), 14, 12, 4),
        (Params(N=20, precision="fp64", m=1.0), 15, 22, 0),
        (Params(N=24, precision="fp32", m=1.0, damp_gamma=3.0, eta_damp=2.05), 16, 28, 7),
        # measured steps write Pi and E into the other buffer: every step
        # measured (the buffer flips each replay), and FP32 measured steps
        # between two-step passes
        (Params(N=16, precision="fp32", m=2.0), 17, 9, 1),
        (Params(N=20, precision="fp32", m=1.0), 18, 14, 3),
        (Params(N=24, precision="fp64", m=2.0), 19, 7, 1),
    ]
    with ah.Pool(hbm_budget=1 << 30, max_slots=16) as pool:
        ids = [pool.submit(p, seed, n, every) for p, seed, n, every in reqs]
        assert all(i is not None for i in ids)
        cfgs = {rid: pool.step_config(rid) for rid in ids}
        states, series = {}, {}
        finished = []
        for step in range(40):
            pool.advance(1)
            for rid in pool.poll():
                finished.append(rid)
                k = ids.index(rid)
                states[rid] = pool.get_state(rid, reqs[k][0].N)
                series[rid] = pool.results(rid)
        assert sorted(finished) == sorted(ids)
        assert pool.stats()["active"] == 0 and pool.stats()["bytes_in_use"] == 0
    # the pool runs the default tile shape with z-chunks of at least 16
    # planes; alone with the same tiling the diagnostics records are summed in
    # the same order
    for (p, seed, n, every), rid in zip(reqs, ids):
        cfg = cfgs[rid]
        with ah.Lattice(p) as lat:
            default = lat.get_step_config()
        assert cfg["kernel"] == "tile" and cfg["tile"] == default["tile"]
        assert min(p.N, 16) <= cfg["zchunk"] <= p.N
        st, ser = run_alone(p, seed, n, every, cfg["tile"], cfg["zchunk"])
        assert np.array_equal(states[rid], st), (p, seed)
        assert len(series[rid]) == len(ser)
        for a, b in zip(series[rid], ser):
            assert same_record(a, b), (p.N, a["step"], b["step"])


def test_pool_matches_oracle(oracle_mod, ah):
    op, gp = both_params(oracle_mod, 20, "fp64", m=2.0)
    with ah.Pool(hbm_budget=256 << 20, max_slots=4) as pool:
        rid = pool.submit(gp, 3, 30, 10)
        pool.advance(31)
        assert pool.poll() == [rid]
        st = pool.get_state(rid, 20)
        ser = pool.results(rid)
    ref = oracle_mod.step(op, oracle_mod.init(op, 3), 0, 30)
    assert max(field_scaled_error(st, ref).values()) <= 1e-10
    assert [m["step"] for m in ser] == [0, 10, 20, 30]
    om = oracle_mod.measure(op, st, 30)
    assert ser[-1]["winding_sum_abs"] == om["winding_sum_abs"]
    assert abs(ser[-1]["energy"] - om["energy"]) <= 1e-10 * abs(om["energy"])


def test_pool_admission_by_footprint(ah):
    from paper_2005_14454_amd import Params, pool_footprint, AHError
    p = Params(N=32, precision="fp32")
    fp = pool_footprint(p, 10, 5)
    assert fp >= 15 * 4 * 32 ** 3
    with ah.Pool(hbm_budget=int(2.5 * fp), max_slots=8) as pool:
        a = pool.submit(p, 1, 10, 5)
        b = pool.submit(p, 2, 10, 5)
        assert a is not None and b is not None
        assert pool.submit(p, 3, 10, 5) is None          # does not fit now
        with pytest.raises(AHError):
            pool.submit(Params(N=64, precision="fp64"), 4, 10, 5)  # larger than the budget
        assert pool.stats()["bytes_in_use"] <= pool.stats()["budget"]
        pool.advance(11)
        assert sorted(pool.poll()) == sorted([a, b])
        pool.results(a)
        c = pool.submit(p, 3, 10, 5)                       # fits once memory is back
        assert c is not None
        pool.advance(11)
        assert pool.poll() == [c]
        assert len(pool.results(c)) == 3
    with ah.Pool(hbm_budget=1 << 28, max_slots=1) as pool:
        assert pool.submit(p, 1, 5, 0) is not None
        assert pool.submit(p, 2, 5, 0) is None             # no free slot


def test_pool_error_paths(ah):
    """Unknown ids and unfinished requests are refused without touching the
    pool; a refused submission takes nothing."""
    from paper_2005_14454_amd import AHError, Params
    with ah.Pool(hbm_budget=256 << 20, max_slots=2) as pool:
        rid = pool.submit(Params(N=16, precision="fp32"), 1, 4, 2)
        before = pool.stats()
        with pytest.raises(AHError):
            pool.step_config(rid + 1000)
        with pytest.raises(AHError):
            pool.progress(rid + 1000)
        with pytest.raises(KeyError):
            pool.get_state(rid + 1000)
        with pytest.raises(ValueError):
            pool.get_state(rid, 17)                       # not the lattice's N
        with pytest.raises(AHError):
            pool.results(rid)                              # not finished yet
        with pytest.raises(AHError):
            pool.submit(Params(N=16, gauge_action="noncompact"), 1, 4, 2)
        with pytest.raises(AHError):
            pool.submit(Params(N=400, precision="fp64"), 1, 4, 2)   # larger than the whole budget
        after = pool.stats()
        assert (after["active"], after["bytes_in_use"]) == (before["active"], before["bytes_in_use"])
        pool.advance(5)
        assert pool.poll() == [rid]
        assert [m["step"] for m in pool.results(rid)] == [0, 2, 4]


def test_pool_staggered_completion_and_progress(ah):
    from paper_2005_14454_amd import Params
    with ah.Pool(hbm_budget=512 << 20, max_slots=8) as pool:
        ids = [pool.submit(Params(N=16, precision="fp32"), s, n, 0) for s, n in ((1, 3), (2, 7), (3, 12))]
        done_at = {}
        for step in range(1, 16):
            pool.advance(1)
            for rid in pool.poll():
                done_at[rid] = step
        # FP32 lattices advance two steps in a replay where neither snapshot
        # is due (here only the last one is): 3 steps take a two-step pass, a
        # step and the final measurement; 7 and 12 steps three and five
        # passes, a step and the measurement
        assert done_at == {ids[0]: 3, ids[1]: 5, ids[2]: 7}
        # a lattice admitted while others run joins the same graph
        late = pool.submit(Params(N=24, precision="fp64"), 9, 5, 2)
        assert pool.progress(late) == (0, 5)
        pool.advance(2)
        assert pool.progress(late) == (2, 5)
        pool.advance(4)
        assert pool.poll() == [late]
        ser = pool.results(late)
        assert [m["step"] for m in ser] == [0, 2, 4, 5]
        for rid in ids:
            assert len(pool.results(rid)) == 1


def test_pool_admissions_within_capacity_reuse_the_graph(ah):
    """The per-step graph is captured once per node layout: admissions and
    releases that fit its work-list capacities only rewrite the lists, and a
    lattice admitted that way still evolves exactly as alone."""
    from paper_2005_14454_amd import Params
    p = Params(N=16, precision="fp32", m=1.0)
    with ah.Pool(hbm_budget=512 << 20, max_slots=8) as pool:
        first = [pool.submit(p, s, 4, 2) for s in (1, 2)]
        pool.advance(2)
        assert pool.stats()["graph_captures"] == 1
        late = pool.submit(p, 5, 7, 2)
        cfg = pool.step_config(late)
        pool.advance(3)
        done = pool.poll()
        assert sorted(done) == sorted(first)  # both have run their 4 steps and the final snapshot
        for rid in done:
            pool.results(rid)
        pool.advance(5)
        assert pool.poll() == [late]
        state = pool.get_state(late, p.N)
        series = pool.results(late)
        assert pool.stats()["graph_captures"] == 1
        # a new precision is a new node: captured anew
        pool.submit(Params(N=16, precision="fp64"), 3, 2, 0)
        pool.advance(1)
        assert pool.stats()["graph_captures"] == 2
    st, ser = run_alone(p, 5, 7, 2, cfg["tile"], cfg["zchunk"])
    assert np.array_equal(state, st)
    assert len(series) == len(ser) and all(same_record(a, b) for a, b in zip(series, ser))


def test_pool_after_host_only_calls_in_a_fresh_process():
    """Host-only calls made before anything touches the GPU (a footprint)
    still leave the process able to create and run a pool: the library loads
    the HIP runtime that torch uses, whatever is called first."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import paper_2005_14454_amd as ah\n"
            "p = ah.Params(N=16)\n"
            "fp = ah.pool_footprint(p, 4, 2)\n"
            "with ah.Pool(4 * fp, 2) as pool:\n"
            "    rid = pool.submit(p, 1, 4, 2)\n"
            "    pool.advance(5)\n"
            "    assert pool.poll() == [rid]\n"
            "    assert [m['step'] for m in pool.results(rid)] == [0, 2, 4]\n"
            "print('ok', flush=True)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr[-3000:]


def test_pool_recorded_tiles_match_alone_and_oracle(oracle_mod, ah):
    """The tile shapes the pool runs for the ensemble workloads (FP32 64 x 4,
    32 x 8, 128 x 8 and 128 x 4, FP64 32 x 8 and 64 x 8), forced through the
    tuning table on small and ragged N, plain and measured steps mixed in one
    pool.  Each lattice's fields and diagnostics equal the same lattice's run
    alone with the same tiling bitwise (the measured step runs the measured
    march's tiling in both); after 40 steps its fields are within the
    scope's tolerance of the oracle
    (FP32 1e-4, FP64 1e-10, field-scaled), its windings equal the oracle's on
    the same snapshot, and its other diagnostics agree with the oracle's
    measurement of that snapshot."""
    from helpers import both_params
    cases = [  # (N, precision, tile recorded, tile the pool runs, m, seed)
        (48, "fp32", (64, 4), (64, 4), 1.0, 21),
        (36, "fp32", (64, 4), (64, 4), 2.0, 22),
        (32, "fp32", (32, 8), (32, 8), 1.0, 23),
        (20, "fp32", (32, 8), (32, 8), 2.0, 24),
        (40, "fp32", (128, 8), (128, 8), 1.0, 25),
        (44, "fp32", (128, 4), (128, 4), 2.0, 27),
        (24, "fp64", (32, 8), (32, 8), 2.0, 26),
        (28, "fp64", (64, 8), (64, 8), 1.0, 28),
    ]
    nsteps, every = 40, 8
    ah.tune_clear()
    try:
        reqs = []
        for N, prec, rec, _, m, seed in cases:
            op, gp = both_params(oracle_mod, N, prec, m=m)
            ah.tune_set(gp, rec, 0)
            reqs.append((op, gp, seed))
        with ah.Pool(hbm_budget=1 << 30, max_slots=len(cases)) as pool:
            ids = [pool.submit(gp, seed, nsteps, every) for _, gp, seed in reqs]
            assert all(i is not None for i in ids)
            cfgs = [pool.step_config(rid) for rid in ids]
            pool.advance(nsteps + 1)
            assert sorted(pool.poll()) == sorted(ids)
            states = [pool.get_state(rid, gp.N) for rid, (_, gp, _) in zip(ids, reqs)]
            series = [pool.results(rid) for rid in ids]
    finally:
        ah.tune_clear()
    for (N, prec, rec, runs, m, seed), (op, gp, _), cfg, st, ser in zip(cases, reqs, cfgs, states, series):
        assert cfg["tile"] == runs, (N, prec, cfg)
        alone_st, alone_ser = run_alone(gp, seed, nsteps, every, cfg["tile"], cfg["zchunk"])
        assert np.array_equal(st, alone_st), (N, prec, runs)
        assert len(ser) == len(alone_ser) == nsteps // every + 1
        for a, b in zip(ser, alone_ser):
            assert same_record(a, b), (N, prec, a["step"])
        ref = oracle_mod.step(op, oracle_mod.init(op, seed), 0, nsteps)
        err = max(field_scaled_error(st, ref).values())
        assert err <= (1e-10 if prec == "fp64" else 1e-4), (N, prec, err)
        om = oracle_mod.measure(op, st, nsteps)
        last = ser[-1]
        assert last["step"] == nsteps
        assert last["winding_sum_abs"] == om["winding_sum_abs"], (N, prec)
        rtol = 1e-11 if prec == "fp64" else 1e-5
        for k in ("energy", "e_kin", "e_grad", "e_pot", "e_el", "e_mag"):
            assert abs(last[k] - om[k]) <= rtol * abs(om["energy"]), (N, prec, k, last[k], om[k])
        assert abs(last["gauss_rms"] - om["gauss_rms"]) <= (1e-12 if prec == "fp64" else 1e-5), (N, prec)
