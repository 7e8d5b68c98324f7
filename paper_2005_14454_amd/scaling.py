"""Scaling analysis of string networks: an ensemble of random-phase lattices
is evolved through a constant expansion era, and the late-time rates
d xi_L / d eta, d xi_W / d eta and the means of <v^2>_phi and <v^2>_omega are
fitted over a conformal-time window, one value per realisation, then
averaged.  This is
the validation the paper runs with its code (section 4, Table 1: for 512^3
boxes in the radiation era the window is eta in [80, 128]).

All realisations are resident at once in a lattice pool and advance
together (one graph replay per step); the diagnostics are taken every
`every` steps (the paper's production runs use 5).

`python -m paper_2005_14454_amd.scaling --N 512 --seeds 12` runs the 512^3
radiation-era ensemble and prints one JSON line.
"""
import argparse
import json
import math
import sys

import numpy as np

from . import Params, Pool, pool_footprint


def fit_slope(eta: np.ndarray, y: np.ndarray) -> float:
    """Least-squares slope of y against eta."""
    A = np.stack([eta, np.ones_like(eta)], axis=1)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(coef[0])


# A straight string of direction n pierces |n_x| + |n_y| + |n_z| plaquettes
# per lattice spacing of its length, 3/2 on average over directions, so the
# winding count dx sum|W| is 3/2 of the length of an isotropic network and
# xi_W is sqrt(3/2) short of the separation it would give with the length.
MANHATTAN = 1.5


def analyse(series, window):
    """Rates and mean velocities of one realisation over the eta window
    (dxi_W_iso: the rate of xi_W with the winding count divided by the
    isotropic-orientation factor 3/2)."""
    lo, hi = window
    rows = [m for m in series if lo <= m["eta"] <= hi]
    eta = np.array([m["eta"] for m in rows])
    out = {"points": len(rows)}
    out["dxi_L"] = fit_slope(eta, np.array([m["xi_L"] for m in rows]))
    out["dxi_W"] = fit_slope(eta, np.array([m["xi_W"] for m in rows]))
    out["dxi_W_iso"] = out["dxi_W"] * math.sqrt(MANHATTAN)
    out["v2_phi"] = float(np.mean([m["v2_phi"] for m in rows]))
    out["v2_omega"] = float(np.mean([m["v2_omega"] for m in rows]))
    return out


def mean_err(values):
    """Mean and standard error of the mean."""
    v = np.asarray(values, dtype=np.float64)
    return float(v.mean()), (float(v.std(ddof=1) / math.sqrt(len(v))) if len(v) > 1 else float("nan"))


def run_ensemble(N=512, seeds=range(12), m=1.0, precision="fp32", every=5, window=(80.0, 128.0), nsteps=None,
                 log=None, batch=None):
    """Evolve one lattice per seed to eta0 + nsteps deta (default: half a
    light crossing, eta = dx N / 2) and fit each over the window.  batch: at
    most that many lattices resident at once (one pool per batch, in turn;
    at 1024^3 FP32 a lattice takes 64 GB), default all."""
    seeds = list(seeds)
    p = Params(N=N, precision=precision, m=m)
    if nsteps is None:
        nsteps = int(round(0.5 * p.dx * N / p.deta))
    batch = len(seeds) if not batch else batch
    per_seed = {}
    for b0 in range(0, len(seeds), batch):
        group = seeds[b0:b0 + batch]
        budget = len(group) * pool_footprint(p, nsteps, every) + (256 << 20)
        with Pool(budget, max_slots=len(group)) as pool:
            ids = {pool.submit(p, s, nsteps, every): s for s in group}
            if None in ids:
                raise RuntimeError("the ensemble does not fit the pool")
            left = set(ids)
            done = 0
            while left:
                pool.advance(10)
                done += 10
                for rid in pool.poll():
                    left.discard(rid)
                    per_seed[ids[rid]] = pool.results(rid)
                if log and done % 200 == 0:
                    log(f"seeds {group}: step {done} of {nsteps}")
    fits = {s: analyse(per_seed[s], window) for s in seeds}
    out = {"N": N, "m": m, "precision": precision, "seeds": seeds, "steps": nsteps, "every": every,
           "window": list(window), "per_seed": {str(s): f for s, f in fits.items()}}
    for k in ("dxi_L", "dxi_W", "dxi_W_iso", "v2_phi", "v2_omega"):
        mu, err = mean_err([f[k] for f in fits.values()])
        out[k] = {"mean": mu, "stderr": err}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--seeds", type=int, default=12)
    ap.add_argument("--m", type=float, default=1.0)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--every", type=int, default=5)
    ap.add_argument("--window", type=float, nargs=2, default=(80.0, 128.0))
    ap.add_argument("--first-seed", type=int, default=1)
    ap.add_argument("--batch", type=int, default=0, help="lattices resident at once (0: all)")
    args = ap.parse_args(argv)
    seeds = range(args.first_seed, args.first_seed + args.seeds)
    out = run_ensemble(args.N, seeds, args.m, args.precision, args.every, tuple(args.window),
                       log=lambda s: print(s, file=sys.stderr, flush=True), batch=args.batch or None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
