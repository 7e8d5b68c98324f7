#!/usr/bin/env python3
"""Benchmark: leapfrog site-updates/s of the Abelian-Higgs step on one MI355X.

Workload: one periodic 512^3 lattice, dx = 0.5, deta = 0.1, lambda0 = 2,
e0 = 1, sigma = 1, s = 0, radiation era (m = 1), random-phase initial
condition from seed 1 (section 2 of Correia & Martins), diagnostics every 10
steps.  The FP32 step is the headline number; the FP64 step of the same
workload is reported beside it.  A "step" is one full leapfrog step
(kick + drift) of the lattice; every 10th snapshot also gets the full
diagnostics (windings, energy split, Lagrangian estimators, Gauss residual),
formed in the same pass as its step, inside the timed region.

Prints one JSON line.  Flags: --gpus N (only 1 is supported), --steps K,
--warmup W, --no-cpu-baseline, --cpu-sweep, --pcie, --no-fp64, --no-batched,
--no-served, --no-copy-probe.
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
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "step_kernel_512cubed_hbm_traffic.txt")


STEP_SOURCES = {"tile": ("ah_step_tile.hip", "ah_stencil.h"), "tile2": ("ah_step2.hip", "ah_stencil.h")}


def kernel_source_hash(kernel):
    """sha256[:16] of the sources of the plain step kernel `kernel` ("tile": one
    step per pass, "tile2": two), as the committed profiles record it."""
    import hashlib
    h = hashlib.sha256()
    for name in STEP_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2005_14454_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def step_kernel_name(precision, cfg):
    real = "float" if precision == "fp32" else "double"
    tx, ty = cfg["tile"]
    if cfg["kernel"] == "tile2":
        return f"k_step2_tile<{real}, {tx}, {ty}>"
    return f"k_step_tile<{real}, {tx}, {ty}, false>"


def measured_traffic(precision, N, cfg):
    """HBM bytes per plain-step launch at 512^3 from the committed rocprofv3
    PMC summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None
    when the kernel's sources have changed since the counters were taken."""
    if N != 512 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
    if f"{cfg['kernel']} sources sha256[:16] = {kernel_source_hash(cfg['kernel'])}" not in text:
        return None
    name = step_kernel_name(precision, cfg)
    # one row per launch geometry; the autotuner's candidates have few
    # dispatches, the benchmark's own configuration the most
    best = None
    for line in text.splitlines():
        if line.startswith(name + " "):
            cols = line[len(name):].split()
            n, total_gb = int(cols[6]), float(cols[4])
            if best is None or n > best[0]:
                best = (n, total_gb)
    return best[1] * 1e9 if best else None


BYTES_PER_SITE = {"fp32": 80, "fp64": 160}  # read 10 reals + write 10 reals per site-update


def tiling(ah, p):
    """Tile shape and z-chunk for (precision, N): the recorded MI355X tuning
    table's entry when it has one (so that runs use the same, recorded
    tiling), else a fresh autotuning run; either way it is in the process's
    tuning table afterwards, where lattices and pools pick it up."""
    from paper_2005_14454_amd.tune import TABLE
    if os.path.exists(TABLE) and ah.tune_lookup(p) is None:
        ah.tune_load(TABLE)
    got = ah.tune_lookup(p)
    if got is not None:
        got["source"] = "table"
        return got
    got = ah.autotune(p, steps=5)
    got["source"] = "autotuned"
    return got


def run_gpu(precision, N, steps, warmup, measure_every, seed, m=1.0):
    import torch
    import paper_2005_14454_amd as ah

    p = ah.Params(N=N, precision=precision, m=m)
    tuned = tiling(ah, p)  # tile shape and z-chunk for this (precision, N)
    lat = ah.Lattice(p)
    cfg = lat.get_step_config()
    lat.init(seed)
    lat.step(warmup)
    lat.measure()
    torch.cuda.synchronize()
    # The timed job with an event pair around every launch (the kernel times
    # come from them).  On a lattice of N <= 128, whose launches take tens of
    # microseconds, the two event records per launch would add to the job's
    # time: there the job is timed without them and the same number of steps
    # is then run again with them, for the kernel times.
    split = N <= 128
    lat.set_timing(not split)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    meas = lat.step_measured(steps, measure_every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    last = meas[-1] if meas else lat.measure()
    if split:
        lat.set_timing(True)
        lat.step_measured(steps, measure_every)
    kern_ms, launches = lat.get_timing()
    meas_ms, meas_launches = lat.get_timing_split()
    lat.set_timing(False)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    sec = t1 - t0
    V = N ** 3
    # the plain step kernel (launches that did not also form diagnostics):
    # the timing counts steps, so this is its time per step; a two-step
    # launch covers two steps and moves the algorithmic bytes of two
    per_launch = 2 if cfg["kernel"] == "tile2" else 1
    avg_kernel_s = (kern_ms - meas_ms) / 1e3 / max(launches - meas_launches, 1)
    avg_measured_s = meas_ms / 1e3 / max(meas_launches, 1)
    algo = BYTES_PER_SITE[precision] * V * per_launch
    launch_s = avg_kernel_s * per_launch
    achieved = algo / launch_s / 1e9
    return {
        "value": V * steps / sec,
        "tuned": tuned,
        "step_kernel": {"kernel": cfg["kernel"], "tile": list(cfg["tile"]), "zchunk": cfg["zchunk"],
                        "steps_per_launch": per_launch, "launch_ms": 1e3 * launch_s},
        "ms_per_step": 1e3 * sec / steps,
        "kernel_ms": 1e3 * avg_kernel_s,
        "measured_step_ms": 1e3 * avg_measured_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(precision, N, cfg),
                     "traffic_unit": "bytes per launch", "algorithmic_bytes": algo},
        "last_measurement": {k: last[k] for k in ("step", "winding_sum_abs", "xi_W", "xi_L", "v2_phi", "v2_omega",
                                                  "energy", "gauss_rel", "nonfinite")},
    }


def pcie_job(N, seed, steps, precision="fp32"):
    """The same stepping with the state handed over in host memory: upload a
    FP64 host snapshot (ah_set_state), `steps` plain steps, download it
    again (ah_get_state); each part timed on the host clock."""
    import torch
    import paper_2005_14454_amd as ah

    p = ah.Params(N=N, precision=precision, m=1.0)
    tiling(ah, p)
    with ah.Lattice(p) as lat:
        lat.init(seed)
        host = lat.get_state()
        lat.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.set_state(host, 0)
        t1 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out = lat.get_state()
        t3 = time.perf_counter()
    del host, out
    V = N ** 3
    return {"steps": steps, "upload_s": t1 - t0, "step_s": t2 - t1, "download_s": t3 - t2,
            "value": V * steps / (t3 - t0), "unit": "site-updates/s",
            "host_bytes_each_way": 10 * 8 * V}


def single_rate(N, precision="fp32", steps=10):
    """su/s of the plain single-lattice step (kernel time) at N."""
    import paper_2005_14454_amd as ah
    with ah.Lattice(ah.Params(N=N, precision=precision, m=1.0)) as lat:
        lat.init(0)
        lat.step(2)
        lat.set_timing(True)
        lat.step(steps)
        ms, n = lat.get_timing()
    return N ** 3 * n / (ms / 1e3)


def batched_ensemble(sizes=(64, 96, 128, 192, 256), nlat=64, rng_seed=4, measure_every=20, chunk=16):
    """nlat independent FP32 lattices, N uniform on `sizes`, m on {1, 2}
    (PCG64 rng_seed), seeds 100.., s = 0, each to eta = dx N / 2, in one pool:
    one graph replay per step advances every unfinished lattice; tile shape
    and z-chunk per size class from the tuning table (or autotuned).  Reported
    beside the same lattices run one after another through the single-lattice
    path (each with its own launches, same diagnostics cadence); both sides
    time the stepping only (allocation and initial conditions outside)."""
    import numpy as np
    import torch
    import paper_2005_14454_amd as ah
    from paper_2005_14454_amd.serve import steps_to_half_light_crossing

    rng = np.random.default_rng(rng_seed)
    Ns = [int(v) for v in rng.choice(list(sizes), nlat)]
    ms = [float(v) for v in rng.choice([1.0, 2.0], nlat)]
    tuned = {}
    for N in sorted(set(Ns)):
        tuned[N] = tiling(ah, ah.Params(N=N, precision="fp32"))
    reqs = [(ah.Params(N=N, precision="fp32", m=m), 100 + i, steps_to_half_light_crossing(N))
            for i, (N, m) in enumerate(zip(Ns, ms))]
    budget = sum(ah.pool_footprint(p, n, measure_every) for p, _, n in reqs) + (64 << 20)
    su = sum(p.N ** 3 * n for p, _, n in reqs)
    with ah.Pool(budget, max_slots=nlat) as pool:
        ids = [pool.submit(p, seed, n, measure_every) for p, seed, n in reqs]
        assert all(i is not None for i in ids)
        pool.advance(1)  # builds and instantiates the graph
        pool.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        left = set(ids)
        steps = 1
        need = max(n for _, _, n in reqs) + 1  # replays until the longest lattice has finished
        while steps < need:
            k = min(chunk, need - steps)
            pool.advance(k)
            steps += k
            for rid in pool.poll_async():
                left.discard(rid)
        for rid in pool.poll():  # waits for the last replays
            left.discard(rid)
        assert not left
        t1 = time.perf_counter()
        finals = [pool.results(rid)[-1] for rid in ids]
    # the same lattices one after another through the single-lattice path,
    # with the same diagnostics cadence (fused into the step) and final record
    rate = {N: single_rate(N) for N in sorted(set(Ns))}
    sequential_s = 0.0
    for p, seed, n in reqs:
        with ah.Lattice(p) as lat:
            lat.init(seed)
            lat.synchronize()
            s0 = time.perf_counter()
            lat.step_measured(n, measure_every)
            lat.measure()
            lat.synchronize()
            sequential_s += time.perf_counter() - s0
    sec = t1 - t0
    return {"lattices": nlat, "sizes": list(sizes), "site_updates": su, "wall_s": sec, "value": su / sec,
            "unit": "site-updates/s", "graph_replays": steps, "sequential_wall_s": sequential_s,
            "sequential_value": su / sequential_s, "speedup_vs_sequential": sequential_s / sec,
            "tuned": {str(k): v for k, v in tuned.items()},
            "single_lattice_su_per_s": {str(k): v for k, v in rate.items()},
            "nonfinite": sum(m["nonfinite"] for m in finals)}


def served(nreq=40):
    """A shortened request stream (the full 500-request stream is
    `python -m paper_2005_14454_amd.serve`): N log-uniform on [64, 512],
    m in {1, 2}, s in {0, 1}, FP32 with an FP64 rerun of every 10th request,
    Poisson arrivals at 0.7 x the capacity, which is the throughput the pool
    sustains on the same requests when they all arrive at once."""
    import numpy as np
    from paper_2005_14454_amd.serve import make_stream, run_stream, saturated_throughput
    budget = int(200e9)
    probe = make_stream(nreq, 1.0)
    work = float(np.mean([r.params.N ** 3 * r.nsteps for r in probe]))
    capacity = saturated_throughput(probe, budget)
    rate = 0.7 * capacity / work
    out = run_stream(make_stream(nreq, rate), hbm_budget=budget)
    out["arrival_rate_per_s"] = rate
    out["capacity_su_per_s"] = capacity
    return out


def copy_probe(nbytes=8 << 30, reps=10):
    """Achievable HBM bandwidth: torch's device-to-device copy of nbytes
    ((read + write bytes) / time; also the known-size copy the PMC traffic
    figures are calibrated with) and the library's streaming copy, read-only
    and write-only kernels (best launch shape)."""
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
    import paper_2005_14454_amd as ah
    return {"bytes_per_copy": 2 * n * 4, "ms": ms, "GB/s": 2 * n * 4 / ms / 1e6,
            "streaming_kernels": ah.hbm_probe(nbytes // 2, 5)}


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


def cpu_sweep(seed, repeats=3):
    """The oracle timed at the sizes of its own timing protocol: 64^3 and
    128^3 for 20 steps and 256^3 for 5, each after one untimed step, on all
    host threads and on one; median of `repeats` runs."""
    import platform
    import statistics

    import oracle

    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    full = oracle.num_threads()
    rows = []
    for threads in (full, 1):
        oracle.set_threads(threads)
        for N, steps in ((64, 20), (128, 20), (256, 5)):
            p = oracle.params(N=N, m=1.0)
            st = oracle.step(p, oracle.init(p, seed), 0, 1)
            times = []
            for _ in range(repeats):
                t0 = time.perf_counter()
                oracle.step(p, st, 1, steps)
                times.append(time.perf_counter() - t0)
            dt = statistics.median(times)
            rows.append({"N": N, "steps": steps, "threads": threads, "median_s": dt,
                         "su_per_s": steps * N ** 3 / dt})
            print(f"# oracle {N}^3 x {steps} steps, {threads} threads: {rows[-1]['su_per_s']:.3e} su/s",
                  file=sys.stderr, flush=True)
    oracle.set_threads(full)
    return {"cpu": model, "nproc": os.cpu_count(), "threads": full, "repeats": repeats, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--measure-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pcie", action="store_true",
                    help="also time a job whose state is uploaded from and downloaded to host memory")
    ap.add_argument("--cpu-sweep", action="store_true",
                    help="also time the oracle at 64^3, 128^3 and 256^3 on all host threads and on one")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=40)
    ap.add_argument("--no-config1", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the lattice path runs on one GPU (asked for --gpus {args.gpus}); "
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
    # the small single-lattice workload: 64^3 FP64 from the random-phase start
    # of seed 0, 160 steps, diagnostics every 10 steps (snapshots 0 .. 150)
    config1 = None if args.no_config1 else run_gpu("fp64", 64, 160, 0, 10, 0)
    if config1:
        print(f"# 64^3 fp64: {config1['value']:.4e} su/s, {config1['ms_per_step'] * 1e3:.1f} us/step, "
              f"kernel {config1['kernel_ms'] * 1e3:.1f} us", file=sys.stderr, flush=True)
    batched = None if args.no_batched else batched_ensemble()
    if batched:
        print(f"# batched: {batched['value']:.4e} su/s over {batched['lattices']} lattices, "
              f"{batched['speedup_vs_sequential']:.2f}x vs sequential", file=sys.stderr, flush=True)
    # many small lattices, where the single-lattice path is launch-bound
    batched_small = None if args.no_batched else batched_ensemble((32, 48, 64), nlat=128, rng_seed=6)
    if batched_small:
        print(f"# batched small: {batched_small['value']:.4e} su/s over {batched_small['lattices']} lattices, "
              f"{batched_small['speedup_vs_sequential']:.2f}x vs sequential", file=sys.stderr, flush=True)
    serv = None if args.no_served else served(args.served_requests)
    if serv:
        print(f"# served: {serv['throughput_su_per_s']:.4e} su/s, p50 {serv['ttc_p50_s']:.2f} s, "
              f"p99 {serv['ttc_p99_s']:.2f} s", file=sys.stderr, flush=True)
    probe = None if args.no_copy_probe else copy_probe()
    pcie = pcie_job(args.N, seed, args.steps) if args.pcie else None
    if pcie:
        print(f"# pcie-inclusive: {pcie['value']:.4e} su/s (upload {pcie['upload_s']:.2f} s, "
              f"{pcie['steps']} steps {pcie['step_s']:.2f} s, download {pcie['download_s']:.2f} s)",
              file=sys.stderr, flush=True)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.N, seed)
    if cpu is not None and args.cpu_sweep:
        cpu["sweep"] = cpu_sweep(seed)

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
        **({"pcie_inclusive": pcie} if pcie else {}),
        "batched": batched,
        "batched_small": batched_small,
        "served": serv,
        "fp64": None if fp64 is None else {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"],
                                           "roofline": fp64["roofline"], "dtype": "f64", "tuned": fp64["tuned"],
                                           "step_kernel": fp64["step_kernel"]},
        "config1_64cubed_fp64": None if config1 is None else {
            "workload": "single 64^3 periodic lattice, FP64, radiation era m=1, s=0, seed 0, 160 steps from the "
                        "initial condition, diagnostics every 10 steps",
            "value": config1["value"], "unit": "site-updates/s", "ms_per_step": config1["ms_per_step"],
            "roofline": config1["roofline"], "measured_step_ms": config1["measured_step_ms"],
            "step_kernel": config1["step_kernel"], "tuned": config1["tuned"],
            "last_measurement": config1["last_measurement"]},
        "step_kernel": fp32["step_kernel"],
        "tuned": fp32["tuned"],
        "kernel_ms": {"fp32": fp32["kernel_ms"], "fp64": None if fp64 is None else fp64["kernel_ms"]},
        "measured_step_ms": {"fp32": fp32["measured_step_ms"],
                             "fp64": None if fp64 is None else fp64["measured_step_ms"]},
        "last_measurement": {"fp32": fp32["last_measurement"],
                             "fp64": None if fp64 is None else fp64["last_measurement"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
