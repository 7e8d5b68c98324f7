"""Tuning table for a device: autotune the tiled step for a set of
(precision, N) and save the choices as JSON (the format ah_tune_save writes
and ah_tune_load reads).

`python -m paper_2005_14454_amd.tune --N 32 48 64 96 128 192 256 512 --out TABLE`
times every supported tile shape and z-chunk of each (precision, N) and
writes the fastest.  `tune_mi355x.json` next to this file is that table for
MI355X; bench.py loads it so that its runs use fixed, recorded tilings.
"""
import argparse
import json
import os
import sys

from . import Params, autotune, tune_clear, tune_load, tune_save

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_mi355x.json")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--N", type=int, nargs="+", default=[32, 48, 64, 96, 128, 192, 256, 512])
    ap.add_argument("--precision", nargs="+", default=["fp32", "fp64"])
    ap.add_argument("--steps", type=int, default=20, help="timed steps per candidate")
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--merge", action="store_true", help="keep the entries already in --out for other sizes")
    args = ap.parse_args(argv)
    tune_clear()
    if args.merge and os.path.exists(args.out):
        tune_load(args.out)
    for prec in args.precision:
        for N in args.N:
            best = autotune(Params(N=N, precision=prec), steps=args.steps)
            print(json.dumps({"precision": prec, "N": N, **best}), file=sys.stderr, flush=True)
    tune_save(args.out)
    print(open(args.out).read(), end="", flush=True)


if __name__ == "__main__":
    main()
