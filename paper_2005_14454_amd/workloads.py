"""The workloads the path is exercised on, as runnable entry points.

1. 64^3 FP64, radiation era, random-phase start from seed 0, 160 steps with
   the diagnostics every 10 steps.
2. 512^3 from seed 1, radiation era: FP32 against FP64 from the same start
   (the FP32 start is the rounding of the FP64 one), 1280 steps with the
   diagnostics every 10 steps; the field-scaled FP32-FP64 difference after
   100 steps, and Gauss's law and the string-length ratio at the end.
3. 1024^3 FP32, matter era, s = 0 until eta = 50 then s = 1 (core growth,
   then the true equations), seed 2, 2560 steps, diagnostics every 20.
4. An ensemble of 64 FP32 lattices, N uniform on {64, 96, 128, 192, 256},
   m on {1, 2}, seeds 100..163, each to eta = dx N / 2, in one lattice pool.
5. The request stream of the serving loop (`serve.py`).

`python -m paper_2005_14454_amd.workloads 2` runs one of them and prints one
JSON line.  Section 2 of the paper fixes the parameters (dx = 0.5,
deta = 0.1, lambda0 = 2, e0 = 1, sigma = 1, eta0 = 1).
"""
import argparse
import json
import sys
import time

import numpy as np

from . import Lattice, Params, Pool, pool_footprint
from .serve import steps_to_half_light_crossing

KEYS = ("step", "eta", "f", "winding_sum_abs", "L_W", "xi_W", "xi_L", "v2_phi", "v2_omega", "energy",
        "gauss_rel", "nonfinite", "flags")


def _brief(m: dict) -> dict:
    return {k: m[k] for k in KEYS}


def _field_scaled(a: np.ndarray, b: np.ndarray) -> float:
    """max over phi, Pi, A, E of max|a - b| / max|b| (components in the order
    phi_re, phi_im, pi_re, pi_im, A0..A2, E0..E2)."""
    out = 0.0
    for comps in ((0, 1), (2, 3), (4, 5, 6), (7, 8, 9)):
        scale = float(np.max(np.abs(b[list(comps)])))
        diff = float(np.max(np.abs(a[list(comps)] - b[list(comps)])))
        out = max(out, diff / scale if scale > 0 else diff)
    return out


def config1():
    p = Params(N=64, precision="fp64", m=1.0)
    t0 = time.perf_counter()
    with Lattice(p) as lat:
        lat.init(0)
        series = lat.step_measured(160, 10) + [lat.measure()]
    return {"workload": "64^3 FP64 radiation era, seed 0, 160 steps", "wall_s": time.perf_counter() - t0,
            "series": [_brief(m) for m in series]}


def config2():
    lats = {prec: Lattice(Params(N=512, precision=prec, m=1.0)) for prec in ("fp32", "fp64")}
    out = {"workload": "512^3 radiation era, seed 1, FP32 against FP64, 1280 steps"}
    try:
        series = {}
        for prec, lat in lats.items():
            lat.init(1)
            series[prec] = lat.step_measured(100, 10)
        s64 = lats["fp64"].get_state()
        s32 = lats["fp32"].get_state()
        out["fp32_vs_fp64_field_scaled_diff_step100"] = _field_scaled(s32, s64)
        del s32, s64
        for prec, lat in lats.items():
            series[prec] += lat.step_measured(1180, 10) + [lat.measure()]
    finally:
        for lat in lats.values():
            lat.close()
    end32, end64 = series["fp32"][-1], series["fp64"][-1]
    out["final"] = {"fp32": _brief(end32), "fp64": _brief(end64)}
    out["L_W_ratio_fp32_over_fp64"] = end32["L_W"] / end64["L_W"]
    out["gauss_rel_max"] = {prec: max(m["gauss_rel"] for m in s) for prec, s in series.items()}
    return out


def config3():
    p = Params(N=1024, precision="fp32", m=2.0, s_early=0.0, s_late=1.0, eta_switch=50.0)
    t0 = time.perf_counter()
    with Lattice(p) as lat:
        lat.init(2)
        series = lat.step_measured(2560, 20) + [lat.measure()]
    return {"workload": "1024^3 FP32 matter era, s = 0 -> 1 at eta = 50, seed 2, 2560 steps",
            "wall_s": time.perf_counter() - t0, "flags_raised": sum(1 for m in series if m["flags"]),
            "series": [_brief(m) for m in series]}


def config4(measure_every: int = 20):
    rng = np.random.default_rng(4)
    Ns = [int(v) for v in rng.choice([64, 96, 128, 192, 256], 64)]
    ms = [float(v) for v in rng.choice([1.0, 2.0], 64)]
    reqs = [(Params(N=N, precision="fp32", m=m), 100 + i, steps_to_half_light_crossing(N))
            for i, (N, m) in enumerate(zip(Ns, ms))]
    budget = sum(pool_footprint(p, n, measure_every) for p, _, n in reqs) + (64 << 20)
    su = sum(p.N ** 3 * n for p, _, n in reqs)
    finals = {}
    with Pool(budget, max_slots=len(reqs)) as pool:
        ids = [pool.submit(p, seed, n, measure_every) for p, seed, n in reqs]
        if None in ids:
            raise RuntimeError("the ensemble does not fit the pool")
        t0 = time.perf_counter()
        left = set(ids)
        while left:
            pool.advance(16)
            for rid in pool.poll():
                left.discard(rid)
                finals[rid] = pool.results(rid)[-1]
        wall = time.perf_counter() - t0
    return {"workload": "64 FP32 lattices, N on {64..256}, m on {1, 2}, seeds 100..163, to eta = dx N / 2",
            "wall_s": wall, "site_updates": su, "site_updates_per_s": su / wall,
            "lattices": [{"N": p.N, "m": p.m, "seed": seed, "steps": n, **_brief(finals[rid])}
                         for (p, seed, n), rid in zip(reqs, ids)]}


def config5(requests: int = 500):
    from .serve import main as serve_main
    serve_main(["--requests", str(requests)])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("config", type=int, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--requests", type=int, default=500, help="stream length of workload 5")
    args = ap.parse_args(argv)
    if args.config == 5:
        config5(args.requests)
        return
    out = {1: config1, 2: config2, 3: config3, 4: config4}[args.config]()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
