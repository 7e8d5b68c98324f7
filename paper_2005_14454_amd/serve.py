"""Serving loop: simulation requests arrive over time and share one GPU.

Requests (lattice size, expansion rate, coupling-scaling exponent, seed,
precision) arrive as a Poisson stream.  Each is admitted into a lattice pool
as soon as a slot and enough contiguous HBM for its footprint are free;
admitted lattices stay resident and are advanced together, one graph replay
per step (continuous batching: requests that arrive while others run join
the next replay).  A request completes when its last diagnostics record is
on the host; time-to-completion (TTC) runs from arrival to that moment.

The loop never waits for the GPU to drain: each advance queues one replay
(the pool keeps up to eight queued, waiting only for older ones), finished
requests are found from counter copies that land behind the replays, and
admissions and series downloads are queued or run beside them.

`python -m paper_2005_14454_amd.serve --requests 500` runs the full stream;
the function `run_stream` is what bench.py calls.
"""
import argparse
import json
import math
import sys
import time
from collections import deque
from dataclasses import dataclass, field, replace

import numpy as np

from . import Params, Pool, pool_footprint


@dataclass
class Request:
    rid: int
    params: Params
    seed: int
    nsteps: int
    measure_every: int
    arrival: float
    pair_of: int = -1          # index of the FP32 request this FP64 rerun checks
    admitted: float = math.nan
    done: float = math.nan
    pool_id: int = -1
    step_config: dict = None   # tile shape and z-chunk the pool stepped it with
    series: list = field(default_factory=list)


def steps_to_half_light_crossing(N: int, dx: float = 0.5, deta: float = 0.1, eta0: float = 1.0) -> int:
    """Steps from eta0 until the horizon reaches half the box, eta = dx N / 2."""
    return int(round((0.5 * dx * N - eta0) / deta))


def make_stream(n: int, rate: float, seed: int = 5, nmin: int = 64, nmax: int = 512, fp64_every: int = 10,
                measure_every: int = 10):
    """n FP32 requests with N log-uniform on [nmin, nmax], m in {1, 2}, s in
    {0, 1}, random seeds, Poisson arrivals at `rate` per second; every
    fp64_every-th request is followed by an FP64 rerun of the same lattice
    arriving at the same time."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        N = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        m = float(rng.choice([1.0, 2.0]))
        s = float(rng.choice([0.0, 1.0]))
        lat_seed = int(rng.integers(0, 2 ** 63 - 1))
        p = Params(N=N, precision="fp32", m=m, s_early=s, s_late=s)
        nsteps = steps_to_half_light_crossing(N)
        reqs.append(Request(len(reqs), p, lat_seed, nsteps, measure_every, t))
        if fp64_every > 0 and i % fp64_every == 0:
            p64 = Params(N=N, precision="fp64", m=m, s_early=s, s_late=s)
            reqs.append(Request(len(reqs), p64, lat_seed, nsteps, measure_every, t, pair_of=len(reqs) - 1))
    return reqs


def saturated_throughput(reqs, hbm_budget: int, max_slots: int = 256, chunk: int = 1) -> float:
    """Site-updates/s the pool sustains on this request mix when every
    request is there from the start (the serving capacity the arrival rate
    is set against).  The requests are copied; their records stay empty."""
    burst = [replace(r, arrival=0.0, admitted=math.nan, done=math.nan, pool_id=-1, step_config=None, series=[])
             for r in reqs]
    return run_stream(burst, hbm_budget, max_slots, chunk)["throughput_su_per_s"]


def run_stream(reqs, hbm_budget: int, max_slots: int = 256, chunk: int = 1, log=None):
    """Serve the requests; returns a summary dict and fills the Request records."""
    pool = Pool(hbm_budget, max_slots)
    future = deque(sorted(reqs, key=lambda r: r.arrival))
    waiting = []
    by_pool = {}
    done = 0
    site_updates = 0
    empty = 0.0  # seconds with no request resident or waiting (the next one has not arrived)
    t0 = time.perf_counter()
    try:
        while done < len(reqs):
            now = time.perf_counter() - t0
            while future and future[0].arrival <= now:
                waiting.append(future.popleft())
            # first-fit admission in arrival order
            still = []
            for r in waiting:
                pid = pool.submit(r.params, r.seed, r.nsteps, r.measure_every)
                if pid is None:
                    still.append(r)
                    continue
                r.admitted = time.perf_counter() - t0
                r.pool_id = pid
                r.step_config = pool.step_config(pid)
                by_pool[pid] = r
            waiting = still
            if by_pool:
                pool.advance(chunk)
                for pid in pool.poll_async():
                    r = by_pool.pop(pid)
                    r.series = pool.results(pid)
                    r.done = time.perf_counter() - t0
                    site_updates += r.params.N ** 3 * r.nsteps
                    done += 1
                    if log:
                        log(f"done {r.rid} N={r.params.N} {r.params.precision} ttc={r.done - r.arrival:.3f}s")
            elif future:
                ts = time.perf_counter()
                time.sleep(max(0.0, min(0.05, future[0].arrival - (ts - t0))))
                empty += time.perf_counter() - ts
            elif waiting:
                raise RuntimeError("a waiting request can never be admitted (budget too small)")
        wall = time.perf_counter() - t0
    finally:
        pool.close()
    ttc = np.array([r.done - r.arrival for r in reqs])
    # FP32 against its FP64 rerun: relative string-length deviation on every
    # common diagnostics snapshot where the FP64 network still has strings
    # (the final one alone can be empty on small lattices), and at the last
    # such snapshot
    dev, dev_last, compared = [], [], 0
    for r in reqs:
        if r.pair_of < 0:
            continue
        a = {m["step"]: m["L_W"] for m in reqs[r.pair_of].series}
        pts = [(abs(a[m["step"]] - m["L_W"]) / m["L_W"]) for m in r.series if m["step"] in a and m["L_W"] > 0]
        compared += len(pts)
        if pts:
            dev.append(max(pts))
            dev_last.append(pts[-1])
    return {
        "requests": len(reqs),
        "wall_s": wall,
        "empty_s": empty,
        "site_updates": site_updates,
        "throughput_su_per_s": site_updates / wall,
        "ttc_p50_s": float(np.percentile(ttc, 50)),
        "ttc_p99_s": float(np.percentile(ttc, 99)),
        "ttc_mean_s": float(ttc.mean()),
        "fp32_vs_fp64_LW_rel_dev_max": max(dev) if dev else None,
        "fp32_vs_fp64_LW_rel_dev_last_mean": float(np.mean(dev_last)) if dev_last else None,
        "fp32_vs_fp64_snapshots_compared": compared,
        "fp64_spot_checks": sum(1 for r in reqs if r.pair_of >= 0),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=500)
    ap.add_argument("--rate", type=float, default=0.0, help="arrivals per second; 0 = 0.7 x measured capacity")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--nmin", type=int, default=64)
    ap.add_argument("--nmax", type=int, default=512)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--capacity-su", type=float, default=0.0,
                    help="site-updates/s the rate is set against; 0 = measure it (all of the first "
                         "--capacity-sample requests at once)")
    ap.add_argument("--capacity-sample", type=int, default=60)
    args = ap.parse_args(argv)
    budget = int(args.budget_gb * 1e9)
    probe = make_stream(args.requests, 1.0, args.seed, args.nmin, args.nmax)
    work = np.mean([r.params.N ** 3 * r.nsteps for r in probe])
    capacity = args.capacity_su
    if args.rate <= 0 and capacity <= 0:
        capacity = saturated_throughput(probe[:args.capacity_sample], budget)
        print(f"capacity on the request mix: {capacity:.4e} site-updates/s", file=sys.stderr, flush=True)
    rate = args.rate if args.rate > 0 else 0.7 * capacity / work
    reqs = make_stream(args.requests, rate, args.seed, args.nmin, args.nmax)
    out = run_stream(reqs, budget, log=lambda s: print(s, file=sys.stderr, flush=True))
    out["arrival_rate_per_s"] = rate
    out["capacity_su_per_s"] = capacity if args.rate <= 0 else None
    out["mean_site_updates_per_request"] = float(work)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
