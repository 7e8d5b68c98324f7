"""Summaries of rocprofv3 output for the profiles the repository keeps.

    python -m paper_2005_14454_amd.profile_summary trace DIR [--note TEXT]
        per kernel and launch geometry (workgroup and grid size): calls, mean,
        min and max duration from the kernel trace (rocprofv3 --kernel-trace
        --output-format csv -d DIR)

    python -m paper_2005_14454_amd.profile_summary traffic FETCH_DIR WRITE_DIR [--N 512]
        HBM bytes per dispatch from two counter passes (--pmc FETCH_SIZE, then
        --pmc WRITE_SIZE), scaled by what the counters read for the largest
        device copy in the same run (a copy of known size: it reads and writes
        its byte count), next to the algorithmic bytes of the step kernels

    python -m paper_2005_14454_amd.profile_summary counters DIR [--N 512]
        mean of every counter per kernel from one --pmc pass, and for the
        step kernels the wave64 VALU instructions per site-update

Every figure printed is computed from the named raw output, so a kept
summary can be recomputed from the run it names.
"""
import argparse
import csv
import glob
import hashlib
import os
import re
import statistics
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows(directory, suffix):
    paths = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not paths:
        raise SystemExit(f"no *{suffix} under {directory}")
    for path in paths:
        with open(path, newline="") as f:
            yield from csv.DictReader(f)


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(f"none of {names} in {sorted(row)}")


def short_name(name):
    """Kernel name without namespaces, argument list and template noise."""
    name = name.replace("(anonymous namespace)::", "").replace("ah::", "").replace("void ", "")
    name = re.sub(r"\(.*$", "", name)
    return name.strip()


def source_hashes():
    """sha256[:16] of the sources of each plain step kernel (as bench.py checks them)."""
    out = {}
    for kernel, names in (("tile", ("ah_step_tile.hip", "ah_stencil.h")), ("tile2", ("ah_step2.hip", "ah_stencil.h"))):
        h = hashlib.sha256()
        for n in names:
            h.update(open(os.path.join(HERE, "csrc", n), "rb").read())
        out[kernel] = h.hexdigest()[:16]
    return out


def busy_fraction(intervals):
    """Share of the span from the first kernel start to the last kernel end
    during which at least one kernel ran (the union of the intervals)."""
    if not intervals:
        return 0.0, 0.0
    iv = sorted(intervals)
    busy, cur_s, cur_e = 0, iv[0][0], iv[0][1]
    for s, e in iv[1:]:
        if s > cur_e:
            busy += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    busy += cur_e - cur_s
    span = max(e for _, e in iv) - iv[0][0]
    return busy / span if span else 0.0, span / 1e9


def idle_gaps(intervals, min_s):
    """(start offset in s, length in s) of every stretch of at least min_s
    seconds between kernels (no kernel running), in time order."""
    iv = sorted(intervals)
    out, end = [], iv[0][1] if iv else 0
    for s, e in iv[1:]:
        if s - end >= min_s * 1e9:
            out.append(((end - iv[0][0]) / 1e9, (s - end) / 1e9))
        end = max(end, e)
    return out


def trace(directory, note="", window=None):
    """Per-kernel statistics; window = a kernel name: the busy fraction is
    also given from its first to its last launch."""
    per = defaultdict(list)
    spans = []
    for r in _rows(directory, "kernel_trace.csv"):
        name = short_name(_col(r, "Kernel_Name", "Kernel-Name"))
        wg = _col(r, "Workgroup_Size", "Workgroup_Size_X", "Workgroup-Size")
        grid = _col(r, "Grid_Size", "Grid_Size_X", "Grid-Size")
        t0, t1 = int(_col(r, "Start_Timestamp")), int(_col(r, "End_Timestamp"))
        per[(name, int(wg), int(grid))].append((t1 - t0) / 1e6)
        spans.append((t0, t1, name))
    lines = [f"rocprofv3 kernel trace summary of {directory}"]
    if note:
        lines.append(note)
    frac, span_s = busy_fraction([(a, b) for a, b, _ in spans])
    lines.append(f"GPU busy (union of kernel intervals) {frac:.3f} of {span_s:.2f} s from the first kernel to the last")
    long_gaps = idle_gaps([(a, b) for a, b, _ in spans], 0.1)
    if long_gaps:
        gap_s = sum(g for _, g in long_gaps)
        lines.append(f"idle gaps of 0.1 s or more: {len(long_gaps)}, {gap_s:.2f} s in all (at "
                     + ", ".join(f"{t:.2f} s: {g:.2f} s" for t, g in long_gaps[:8])
                     + (", ..." if len(long_gaps) > 8 else "") + ")")
        lines.append(f"GPU busy outside those gaps {frac * span_s / (span_s - gap_s):.3f} of {span_s - gap_s:.2f} s")
    if window:
        w = [(a, b) for a, b, n in spans if window in n]
        if w:
            lo, hi = min(a for a, _ in w), max(b for _, b in w)
            f2, s2 = busy_fraction([(a, b) for a, b, _ in spans if a >= lo and b <= hi])
            lines.append(f"GPU busy between the first and last {window}: {f2:.3f} of {s2:.2f} s")
    for k, h in source_hashes().items():
        lines.append(f"{k} sources sha256[:16] = {h}")
    lines.append("")
    lines.append(f"{'kernel':<48} {'wg':>5} {'threads':>10} {'calls':>6} {'avg_ms':>9} {'min_ms':>9} {'max_ms':>9}")
    for (name, wg, grid), d in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{name[:48]:<48} {wg:>5} {grid:>10} {len(d):>6} {statistics.mean(d):>9.4f} {min(d):>9.4f} "
                     f"{max(d):>9.4f}")
    return "\n".join(lines)


def _counters(directory, counter):
    """{dispatch id: (kernel name, value in KiB)} for one counter pass."""
    vals = defaultdict(float)
    names = {}
    for r in _rows(directory, "counter_collection.csv"):
        if _col(r, "Counter_Name", "Counter-Name") != counter:
            continue
        d = int(_col(r, "Dispatch_Id", "Dispatch-Id", "Correlation_Id"))
        vals[d] += float(_col(r, "Counter_Value", "Counter-Value"))
        names[d] = short_name(_col(r, "Kernel_Name", "Kernel-Name"))
    return {d: (names[d], v) for d, v in vals.items()}


ALGO_PER_SITE = {  # algorithmic bytes per site of one launch
    ("k_step_tile", "false"): 20, ("k_step2_tile", None): 40, ("k_step_tile", "true"): 10,
}


def algorithmic_gb(name, N):
    m = re.match(r"(\w+)<(float|double)(?:, (\d+), (\d+))?(?:, (true|false))?>", name)
    if not m:
        return None
    base, real, meas = m.group(1), m.group(2), m.group(5)
    reals = ALGO_PER_SITE.get((base, meas))
    if reals is None:
        return None
    return reals * (4 if real == "float" else 8) * N ** 3 / 1e9


def traffic(fetch_dir, write_dir, N=512, note="", copy_bytes=8 << 30):
    """Bytes per dispatch from the two counter passes.  Each counter is scaled
    by what it reads for the largest device copy in the run, which reads and
    writes copy_bytes (bench.py's copy probe: 8 GiB each way)."""
    fetch = _counters(fetch_dir, "FETCH_SIZE")
    write = _counters(write_dir, "WRITE_SIZE")

    def copy_max(tab):
        c = [v for n, v in tab.values() if "copyBuffer" in n]
        return max(c) if c else None

    cf, cw = copy_max(fetch), copy_max(write)
    lines = [f"HBM traffic per dispatch from rocprofv3 PMC counters: {fetch_dir} (FETCH_SIZE), "
             f"{write_dir} (WRITE_SIZE)"]
    if note:
        lines.append(note)
    for k, h in source_hashes().items():
        lines.append(f"{k} sources sha256[:16] = {h}")
    if not cf or not cw:
        lines.append("no device copy in the run: counters not calibrated")
        return "\n".join(lines)
    kib = copy_bytes / 1024
    ff, wf = kib / cf, kib / cw
    lines.append(f"calibration: the largest device copy ({copy_bytes / 2**30:.0f} GiB read and written) reads "
                 f"FETCH_SIZE {cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB -> fetch factor {ff:.4f}, write factor {wf:.4f}")
    lines.append("")
    agg = defaultdict(lambda: [[], []])
    for name, v in fetch.values():
        agg[name][0].append(v)
    for name, v in write.values():
        agg[name][1].append(v)
    lines.append(f"{'kernel':<40} {'FETCH_KiB':>12} {'WRITE_KiB':>12} {'read_GB':>8} {'write_GB':>8} {'total_GB':>8} "
                 f"{'algo_GB':>8} {'n':>4}")
    for name, (fv, wv) in sorted(agg.items()):
        fk = statistics.mean(fv) if fv else 0.0
        wk = statistics.mean(wv) if wv else 0.0
        rd = fk * ff * 1024 / 1e9
        wr = wk * wf * 1024 / 1e9
        algo = algorithmic_gb(name, N)
        lines.append(f"{name[:40]:<40} {fk:>12.0f} {wk:>12.0f} {rd:>8.3f} {wr:>8.3f} {rd + wr:>8.3f} "
                     f"{(f'{algo:.3f}' if algo else '-'):>8} {len(fv):>4}")
    return "\n".join(lines)


SITE_UPDATES_PER_SITE = {"k_step_tile": 1, "k_step2_tile": 2}


def counters(directory, N=512, note=""):
    """Mean of every counter per kernel (one --pmc pass); SQ_INSTS_VALU per
    site-update for the step kernels at N^3 (a rough figure where a kernel
    name covers several lattice sizes)."""
    vals = defaultdict(lambda: defaultdict(float))
    names = {}
    for r in _rows(directory, "counter_collection.csv"):
        d = int(_col(r, "Dispatch_Id", "Dispatch-Id", "Correlation_Id"))
        vals[d][_col(r, "Counter_Name", "Counter-Name")] += float(_col(r, "Counter_Value", "Counter-Value"))
        names[d] = short_name(_col(r, "Kernel_Name", "Kernel-Name"))
    per = defaultdict(list)
    for d, v in vals.items():
        per[names[d]].append(v)
    cols = sorted({c for v in vals.values() for c in v})
    lines = [f"rocprofv3 counters per dispatch (mean over dispatches) of {directory}"]
    if note:
        lines.append(note)
    for k, h in source_hashes().items():
        lines.append(f"{k} sources sha256[:16] = {h}")
    lines.append("")
    lines.append(f"{'kernel':<44} {'n':>4} " + " ".join(f"{c[:22]:>22}" for c in cols) + f" {'VALU/site-update':>16}")
    for name, vs in sorted(per.items()):
        means = [statistics.mean(v.get(c, 0.0) for v in vs) for c in cols]
        base = re.match(r"(\w+)<", name)
        upd = SITE_UPDATES_PER_SITE.get(base.group(1) if base else "", 0)
        vpu = "-"
        if upd and "SQ_INSTS_VALU" in cols:
            vpu = f"{means[cols.index('SQ_INSTS_VALU')] * 64 / (upd * N ** 3):.1f}"
        lines.append(f"{name[:44]:<44} {len(vs):>4} " + " ".join(f"{m:>22.4g}" for m in means) + f" {vpu:>16}")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--note", default="")
    t.add_argument("--window", default=None, help="kernel name whose first and last launch bound a busy figure")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--N", type=int, default=512)
    c.add_argument("--note", default="")
    c.add_argument("--copy-bytes", type=int, default=8 << 30)
    q = sub.add_parser("counters")
    q.add_argument("dir")
    q.add_argument("--N", type=int, default=512)
    q.add_argument("--note", default="")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace(a.dir, a.note, a.window))
    elif a.cmd == "counters":
        print(counters(a.dir, a.N, a.note))
    else:
        print(traffic(a.fetch_dir, a.write_dir, a.N, a.note, a.copy_bytes))


if __name__ == "__main__":
    sys.exit(main())
