#!/usr/bin/env python3
"""Benchmark: leapfrog site-updates/s of the Abelian-Higgs step on one MI355X.

Workload: one periodic 512^3 lattice, dx = 0.5, deta = 0.1, lambda0 = 2,
e0 = 1, sigma = 1, s = 0, radiation era (m = 1), random-phase initial
condition from seed 1 (section 2 of Correia & Martins), diagnostics every 10
steps.  The FP32 step is the headline number; the FP64 step of the same
workload is reported beside it.  A "step" is one full leapfrog step
(kick + drift) of the lattice; every 10th step is followed by the full
diagnostics pass (windings, energy split, Lagrangian estimators, Gauss
residual), which is inside the timed region.

Prints one JSON line.  Flags: --gpus N (only 1 is supported), --steps K,
--warmup W, --no-cpu-baseline, --no-fp64.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
BYTES_PER_SITE = {"fp32": 80, "fp64": 160}  # read 10 reals + write 10 reals per site-update


def run_gpu(precision, N, steps, warmup, measure_every, seed):
    import torch
    import paper_2005_14454_amd as ah

    p = ah.Params(N=N, precision=precision, m=1.0)
    lat = ah.Lattice(p)
    lat.init(seed)
    lat.step(warmup)
    lat.measure()
    torch.cuda.synchronize()
    lat.set_timing(True)
    meas = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        lat.step(1)
        if (k + 1) % measure_every == 0:
            meas.append(lat.measure())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = lat.get_timing()
    lat.set_timing(False)
    last = meas[-1] if meas else lat.measure()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    sec = t1 - t0
    V = N ** 3
    avg_kernel_s = kern_ms / 1e3 / max(launches, 1)
    achieved = BYTES_PER_SITE[precision] * V / avg_kernel_s / 1e9
    return {
        "value": V * steps / sec,
        "ms_per_step": 1e3 * sec / steps,
        "kernel_ms": 1e3 * avg_kernel_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "last_measurement": {k: last[k] for k in ("step", "winding_sum_abs", "xi_W", "xi_L", "v2_phi",
                                                  "energy", "gauss_rel", "nonfinite")},
    }


def copy_probe(nbytes=8 << 30, reps=10):
    """Achievable HBM bandwidth of a plain device-to-device copy (torch's copy
    kernel) of nbytes: (read + write bytes) / time."""
    import torch
    n = nbytes // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * n * 4, "ms": ms, "GB/s": 2 * n * 4 / ms / 1e6}


def cpu_baseline(N, seed, steps=4):
    """The FP64 CPU oracle timed on this host: `steps` steps of the same 512^3
    workload after one untimed step (so that the links are non-trivial)."""
    import oracle

    p = oracle.params(N=N, m=1.0)
    st = oracle.init(p, seed)
    st = oracle.step(p, st, 0, 1)
    t0 = time.perf_counter()
    oracle.step(p, st, 1, steps)
    dt = time.perf_counter() - t0
    return {"value": steps * N ** 3 / dt, "unit": "site-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} FP64 steps of the {N}^3 lattice after one untimed step, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--measure-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the lattice is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    seed = 1
    fp32 = run_gpu("fp32", args.N, args.steps, args.warmup, args.measure_every, seed)
    print(f"# fp32: {fp32['value']:.4e} su/s, {fp32['ms_per_step']:.3f} ms/step, kernel {fp32['kernel_ms']:.3f} ms",
          file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_gpu("fp64", args.N, args.steps, args.warmup, args.measure_every, seed)
        print(f"# fp64: {fp64['value']:.4e} su/s, {fp64['ms_per_step']:.3f} ms/step, kernel "
              f"{fp64['kernel_ms']:.3f} ms", file=sys.stderr, flush=True)
    probe = None if args.no_copy_probe else copy_probe()
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.N, seed)

    out = {
        "metric": "lattice site-updates/s (FP64 vs FP32, % HBM peak); batched p50/p99 run latency",
        "value": fp32["value"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (random-phase initial condition, seed 1)",
        "config": {"workload": f"single {args.N}^3 periodic lattice, radiation era m=1, s=0, dx=0.5, deta=0.1, "
                               f"lambda0=2, e0=1, sigma=1, diagnostics every {args.measure_every} steps",
                   "N": args.N, "measure_every": args.measure_every, "parallelism": "single GPU"},
        "roofline": fp32["roofline"],
        "cpu_baseline": cpu,
        "hbm_copy_probe": probe,
        "fp64": None if fp64 is None else {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"],
                                           "roofline": fp64["roofline"], "dtype": "f64"},
        "kernel_ms": {"fp32": fp32["kernel_ms"], "fp64": None if fp64 is None else fp64["kernel_ms"]},
        "last_measurement": {"fp32": fp32["last_measurement"],
                             "fp64": None if fp64 is None else fp64["last_measurement"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
