#!/usr/bin/env python3
"""Benchmark: block-multicolored ICCG time-to-solve on one MI355X.

A step is one full ICCG solve (IC(0)-preconditioned CG, relative residual
1e-8, x0 = 0) of the 3D 7-point variable-coefficient Poisson system on a 128^3
grid (n = 2,097,152, nnz = 14,581,760; face coefficients lognormal(0, 1);
diagonal = sum of off-diagonals + 1e-6; b uniform[-1, 1], seed 42), with the
matrix, ordering and factor already resident in HBM.  Like the paper's Table 2
it sweeps the ABMC block size (8/16/32/64) and reports the best; Leiden-CPM
blocks are measured beside it.  Ordering and factorization are setup and are
not timed (the paper's solve times also exclude blocking).

Reported on one JSON line: time-to-solve (the metric), the substitution and
SpMV bandwidth of the instrumented solve, a roofline entry for the dominant
kernel, the FP32 form against FP64, and the serial CPU oracle timed on a
bounded sample of the same solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the timed kernels, from two rocprofv3 --pmc passes (FETCH_SIZE,
# then WRITE_SIZE) over `bench.py --traffic-run`, scaled by what the same
# counters read for a plain streaming kernel of known size (torch.neg over
# 2^26 doubles: 512 MiB read, 512 MiB written).  The summary records a hash
# of the sources that shape those kernels; a stale summary gives null.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweep_spmv_poisson7_128_abmc16.md")
TRAFFIC_SOURCES = ["paper_2609_00561_amd/csrc/iccg.hip", "paper_2609_00561_amd/csrc/iccg_device.h",
                   "paper_2609_00561_amd/csrc/iccg_internal.h", "paper_2609_00561_amd/csrc/setup.cpp"]
CALIB_ELEMS = 1 << 26
KERNEL_CLASSES = {            # rocprofv3 kernel name pattern -> report name
    "k_sweep(forward)": r"k_sweep<double, true, \d+, 1,",
    "k_sweep(backward)": r"k_sweep<double, false, \d+, 2,",
    "k_sweep_wide(forward)": r"k_sweep_wide<double, true, \d+, 1,",
    "k_sweep_wide(backward)": r"k_sweep_wide<double, false, \d+, 2,",
    "k_spmv": r"k_spmv<0,",
    "calibration": r"neg",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _counter_rows(directory):
    """(kernel name, counter value) per dispatch from a rocprofv3 csv pass."""
    import csv
    import glob
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {directory}")
    rows = []
    for fn in files:
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                rows.append((r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    return rows


def traffic_file(workload, block_size, tag=None):
    if workload == "poisson7_128" and block_size == 16 and tag is None:
        return TRAFFIC_FILE
    return os.path.join(ROOT, "profiles", f"traffic_sweep_spmv_{workload}_{tag or f'abmc{block_size}'}.md")


# the orderings the profiling program can use besides ABMC (the paper's
# Leiden-CPM at its resolution 0.05 and Leiden-MD at resolution 1)
PROFILE_LEIDEN = {"leiden-cpm": ("cpm", 0.05, "Leiden-CPM gamma=0.05"),
                  "leiden-md": ("modularity", 1.0, "Leiden-MD gamma=1")}


def profile_ordering(args):
    """(file tag, label) of the ordering the profiling program runs."""
    if args.ordering == "abmc":
        s = int(args.block_sizes.split(",")[0])
        return f"abmc{s}", f"{args.workload} (ABMC s={s})"
    quality, gamma, label = PROFILE_LEIDEN[args.ordering]
    return args.ordering.replace("-", ""), f"{args.workload} ({label})"


def traffic_summary(fetch_dir, write_dir, command_fetch, command_write, out_file=TRAFFIC_FILE,
                    label="poisson7_128 (ABMC s=16)"):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE of the timed kernels, scaled by the
    calibration kernel, written to the committed summary."""
    import re
    calib_bytes = 8.0 * CALIB_ELEMS
    per = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        for name, cname, v in _counter_rows(d):
            if cname != counter:
                continue
            for cls, pat in KERNEL_CLASSES.items():
                if re.search(pat, name):
                    per.setdefault((cls, counter), []).append(v)
    lines = [f"# HBM traffic per dispatch: ICCG kernels on {label}", "",
             "Counters in KiB per dispatch, averaged over the dispatches of one class; the",
             "scale factor is the known bytes of the calibration kernel (torch.neg over",
             f"{CALIB_ELEMS} doubles: {calib_bytes:.0f} B read, {calib_bytes:.0f} B written) divided",
             "by what the counter reads for it.", "",
             f"FETCH pass: `{command_fetch}`", "",
             f"WRITE pass: `{command_write}`", "",
             f"source-hash: {source_hash()}", "",
             "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled read B | scaled write B |",
             "|---|---|---|---|---|---|"]
    cf = calib_bytes / (1024.0 * np.mean(per[("calibration", "FETCH_SIZE")]))
    cw = calib_bytes / (1024.0 * np.mean(per[("calibration", "WRITE_SIZE")]))
    result = {}
    for cls in KERNEL_CLASSES:
        f = per.get((cls, "FETCH_SIZE"), [])
        w = per.get((cls, "WRITE_SIZE"), [])
        if not f or not w:
            continue
        rb = 1024.0 * float(np.mean(f)) * cf
        wb = 1024.0 * float(np.mean(w)) * cw
        result[cls] = rb + wb
        lines.append(f"| {cls} | {len(f)} | {np.mean(f):.1f} | {np.mean(w):.1f} | {rb:.0f} | {wb:.0f} |")
    lines += ["", f"scale: FETCH x{cf:.4f}, WRITE x{cw:.4f}", ""]
    for cls, v in result.items():
        if cls != "calibration":
            lines.append(f"traffic-bytes-per-launch {cls} {v:.0f}")
    os.makedirs(os.path.dirname(out_file), exist_ok=True)
    with open(out_file, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _csv_rows(directory, suffix):
    import csv
    import glob
    files = glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise SystemExit(f"no *{suffix} under {directory}")
    rows = []
    for fn in files:
        with open(fn, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def tcc_summary(directory, command, out_file, label):
    """L2 (TCC) hits and misses per dispatch of the timed kernels, from one
    rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum pass: the GPU analogue of the
    paper's L2 hit-rate measurements (Tables 3 and 7)."""
    import re
    per = {}
    for r in _csv_rows(directory, "counter_collection.csv"):
        for cls, pat in KERNEL_CLASSES.items():
            if cls != "calibration" and re.search(pat, r["Kernel_Name"]):
                per.setdefault((cls, r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    lines = [f"# L2 (TCC) hit rate per dispatch: ICCG kernels on {label}", "",
             "TCC_HIT_sum and TCC_MISS_sum: L2 requests that hit or missed, summed over the L2",
             "channels, averaged over the dispatches of one kernel class.  Misses go to the",
             "Infinity Fabric (the 256 MB memory-side Infinity Cache or HBM).", "",
             f"Command: `{command}`", "", f"source-hash: {source_hash()}", "",
             "| kernel | dispatches | hits | misses | hit rate |", "|---|---|---|---|---|"]
    for cls in KERNEL_CLASSES:
        h = per.get((cls, "TCC_HIT_sum"), [])
        m = per.get((cls, "TCC_MISS_sum"), [])
        if not h or not m:
            continue
        hm, mm = float(np.mean(h)), float(np.mean(m))
        lines.append(f"| {cls} | {len(h)} | {hm:.0f} | {mm:.0f} | {hm / max(hm + mm, 1.0):.3f} |")
    with open(out_file, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_summary(directory, command, out_file, label):
    """Kernel-time summary of one rocprofv3 --kernel-trace --stats run: the
    statistics table and one CG iteration in trace order (the dispatches
    from one k_update_p to the next, the iteration of median span)."""
    stats = _csv_rows(directory, "kernel_stats.csv")
    trace = _csv_rows(directory, "kernel_trace.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# Kernel time: ICCG solve on {label}", "",
             "Command (rocprofv3 kernel trace with statistics, csv output):", "", f"`{command}`", "",
             f"source-hash: {source_hash()}", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in stats[:14]:
        name = r["Name"].split("(")[0] if "(" in r["Name"] and "<" not in r["Name"].split("(")[0] else r["Name"]
        name = name.replace("void ", "")
        if "(" in name:
            name = name[:name.rfind("(")] if name.endswith(")") else name
        if len(name) > 80:
            name = name[:56] + " ... " + ("neg" if "neg" in name else "fill" if "Fill" in name else "")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {100.0 * float(r['TotalDurationNs']) / tot:.2f} |")
    trace.sort(key=lambda r: int(r["Start_Timestamp"]))
    ups = [i for i, r in enumerate(trace) if "k_update_p" in r["Kernel_Name"] and "cols" not in r["Kernel_Name"]]
    if len(ups) >= 4:
        # the iteration of median span (a span that holds the host's check
        # between two replayed batches is not one iteration's work)
        spans = sorted((int(trace[ups[j + 1]]["Start_Timestamp"]) - int(trace[ups[j]]["Start_Timestamp"]), j)
                       for j in range(len(ups) - 1))
        j = spans[len(spans) // 2][1]
        a, b = ups[j], ups[j + 1]
        seg = trace[a:b]
        span = (int(trace[b]["Start_Timestamp"]) - int(seg[0]["Start_Timestamp"])) / 1e3
        lines += ["", f"One CG iteration in trace order ({len(seg)} kernels, {span:.1f} us from the start of",
                  "one k_update_p to the start of the next):", "",
                  "| kernel | workgroups | us |", "|---|---|---|"]
        for r in seg:
            nm = r["Kernel_Name"].replace("void ", "")
            nm = nm[:nm.find("(")] if "(" in nm else nm
            wg = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0) // max(int(r.get("Workgroup_Size", r.get("Workgroup_Size_X", 1)) or 1), 1)
            lines.append(f"| `{nm}` | {wg} | {(int(r['End_Timestamp']) - int(r['Start_Timestamp'])) / 1e3:.2f} |")
    with open(out_file, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def traffic_for(kernel, path=TRAFFIC_FILE):
    """Scaled HBM bytes per launch of `kernel` from the committed summary, or
    None when it is missing or was taken from other kernel sources."""
    try:
        with open(path) as fh:
            text = fh.read().splitlines()
    except OSError:
        return None
    if f"source-hash: {source_hash()}" not in text:
        return None
    for ln in text:
        parts = ln.split()
        if len(parts) == 3 and parts[0] == "traffic-bytes-per-launch" and parts[1] == kernel:
            return float(parts[2])
    return None


def traffic_run(args):
    """The program the --pmc passes profile: the calibration kernel, then 30
    iterations of the timed solve configuration."""
    import torch
    import synth
    from paper_2609_00561_amd import iccg
    x = torch.ones(CALIB_ELEMS, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y
    A, b = synth.workload(args.workload, args.seed)
    if args.ordering == "abmc":
        order = iccg.iccg_order_abmc(A, int(args.block_sizes.split(",")[0]))
    else:
        quality, gamma, _ = PROFILE_LEIDEN[args.ordering]
        order = iccg.iccg_order_leiden(A, quality, gamma)
    rp, cl, vl = iccg.iccg_permute(A, order.perm)
    # --unfused: the last color's sweeps as two launches, so the counted
    # forward-sweep dispatches are the n_c per-color launches the roofline's
    # instrumented solve times
    with iccg.Context(rp, cl, vl, order.block_ptr, order.color_ptr, fuse_turn=not args.unfused) as ctx:
        ctx.ic0_factor()
        bd = torch.tensor(b[order.perm], device="cuda")
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        r = ctx.solve(bd, xd, tol=args.tol, maxit=30, raise_on_noconv=False)
        torch.cuda.synchronize()
    log(f"[traffic-run] done: {r['iters']} iterations")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poisson7_128")
    ap.add_argument("--block-sizes", default="8,16,32,64",
                    help="ABMC block sizes swept on the timed matrix; the fastest is the headline")
    ap.add_argument("--extra-block-sizes", default="2,4",
                    help="smaller ABMC block sizes also solved and reported, outside the headline sweep")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--ordering", default="abmc", choices=["abmc"] + sorted(PROFILE_LEIDEN),
                    help="ordering of the profiling program (--traffic-run) and its summaries")
    ap.add_argument("--no-leiden", action="store_true")
    ap.add_argument("--no-hybrid", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=100)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the Leiden seed and resolution studies")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--no-other-matrices", action="store_true",
                    help="skip the FEM-like kNN and 27-point stencil entries")
    ap.add_argument("--leiden-seeds", default="9,31,42,58,74")
    ap.add_argument("--cpm-gammas", default="0.001,0.01,0.2")
    ap.add_argument("--other-block-sizes", default="2,4,8,16,32",
                    help="ABMC block sizes swept on the kNN graph and the 27-point stencil")
    ap.add_argument("--md-gammas", default="4,16",
                    help="Leiden-MD resolutions for the kNN graph beside gamma = 1")
    ap.add_argument("--multi-k", type=int, default=8)
    ap.add_argument("--learned-matrices", type=int, default=256)
    ap.add_argument("--learned-epochs", type=int, default=4)
    ap.add_argument("--learned-seeds", type=int, default=3,
                    help="unseen seeds per sigma in {0.5, 1, 2} and per grid (64^3, 128^3)")
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--unfused", action="store_true",
                    help="with --traffic-run: the last color's two sweeps as separate launches")
    ap.add_argument("--traffic-run", action="store_true",
                    help="run only the program profiled by the --pmc traffic passes")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "CMD_FETCH", "CMD_WRITE"),
                    help="write the traffic summary from two rocprofv3 csv passes (no GPU)")
    ap.add_argument("--tcc-summary", nargs=2, metavar=("DIR", "CMD"),
                    help="write the L2 hit-rate summary from a TCC_HIT_sum/TCC_MISS_sum pass (no GPU)")
    ap.add_argument("--trace-summary", nargs=2, metavar=("DIR", "CMD"),
                    help="write the kernel-time summary from a --kernel-trace --stats run (no GPU)")
    return ap.parse_args()


def cpu_info():
    """CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail, os.cpu_count()


class Bench:
    """Shared helpers: contexts, timed solves, instrumented solves."""

    def __init__(self, args, dev, iccg, log):
        import torch
        self.torch = torch
        self.args, self.dev, self.iccg, self.log = args, dev, iccg, log

    def ctx(self, A, order, **kw):
        rp, cl, vl = self.iccg.iccg_permute(A, order.perm)
        c = self.iccg.Context(rp, cl, vl, order.block_ptr, order.color_ptr, **kw)
        c.ic0_factor()
        return c

    def time_solves(self, ctx, bp, steps, warmup):
        torch = self.torch
        bd = torch.tensor(bp, device=self.dev)
        xd = torch.zeros(ctx.n, dtype=torch.float64, device=self.dev)
        for _ in range(warmup):
            xd.zero_()
            ctx.solve(bd, xd, tol=self.args.tol, maxit=100000)
        torch.cuda.synchronize()
        times, res = [], None
        t_start = time.perf_counter()
        for _ in range(steps):
            xd.zero_()
            ts = time.perf_counter()
            res = ctx.solve(bd, xd, tol=self.args.tol, maxit=100000)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        return time.perf_counter() - t_start, times, res, xd

    def phases(self, ctx, bp):
        """Instrumented solve: the paper's Table 8 split (forward, backward,
        SpMV, other) and the per-launch sweep and SpMV bandwidth."""
        torch = self.torch
        prof = ctx.profile_solve(torch.tensor(bp, device=self.dev),
                                 torch.zeros(ctx.n, dtype=torch.float64, device=self.dev),
                                 tol=self.args.tol, maxit=100000)
        info = ctx.info()
        fwd_bytes = info["sweep_bytes"] + 16.0 * ctx.n
        fwd_ms = prof["fwd_ms"] / max(prof["fwd_launches"], 1)
        spmv_ms = prof["spmv_ms"] / max(prof["spmv_launches"], 1)
        nc = info["ncolors"]
        return {"phases_ms": {k: round(prof[k], 3) for k in ("total_ms", "fwd_ms", "bwd_ms", "spmv_ms", "other_ms")},
                "forward_sweep_GBps": round((fwd_bytes / nc) / (fwd_ms * 1e-3) / 1e9, 1),
                "spmv_GBps": round(info["spmv_bytes"] / (spmv_ms * 1e-3) / 1e9, 1)}

    def entry(self, A, b, order, label, precision="fp64", timed=2, phases=True, blocking_s=None, extra=None,
              x_ref=None):
        """One ordering of one matrix: Table 6 statistics, timed solves,
        iterations, and (optionally) the Table 8 phase split."""
        iccg, np_ = self.iccg, np
        st = iccg.iccg_block_stats(order)
        bp = b[np_.asarray(order.perm)]
        ctx = self.ctx(A, order, precision=precision)
        try:
            _, times, res, xd = self.time_solves(ctx, bp, timed, 1 if timed > 1 else 0)
            info = ctx.info()
            e = {"matrix": label, "precision": precision, "n": A.n, "nnz": A.nnz,
                 "n_b": st["n_b"], "n_c": st["n_c"], "G": round(st["gini"], 4), "B_max": st["B_max"],
                 "B_max_over_avg": round(st["B_max_over_avg"], 3),
                 "C_max_over_avg": round(st["C_max_over_avg"], 3),
                 "iters": res["iters"], "ms": round(1e3 * float(np_.median(times)), 3),
                 "relres_true": res["relres_true"], "max_block": info["max_block"]}
            if blocking_s is not None:
                e["blocking_s"] = round(blocking_s, 2)
            if phases:
                e.update(self.phases(ctx, bp))
            if x_ref is not None:
                x = xd.cpu().numpy()
                e["x_rel_diff_vs_fp64"] = float(np_.linalg.norm(x - x_ref) / np_.linalg.norm(x_ref))
            if extra:
                e.update(extra)
            x_out = xd.cpu().numpy()
        finally:
            ctx.close()
        self.log(f"[bench] {label} {precision}: {e}")
        return e, x_out


def other_matrices(B, args, synth):
    """The FEM-like unstructured matrix (13-NN graph Laplacian on 10^6
    points) and the 27-point stencil on 96^3.  Like the paper's Table 2, each
    sweeps the ABMC block size and its best FP64 ordering is also solved with
    the FP32 form; the kNN graph is also blocked by Leiden-CPM and Leiden-MD
    (with the resolution study of Fig. 4)."""
    iccg = B.iccg
    entries = []

    def abmc_sweep(name, A, b):
        best = None
        for s in [int(v) for v in args.other_block_sizes.split(",") if v]:
            tb = time.time()
            o = iccg.iccg_order_abmc(A, s)
            tb = time.time() - tb
            e, x64 = B.entry(A, b, o, f"{name} ABMC s={s}", blocking_s=tb)
            entries.append(e)
            if best is None or e["ms"] < best[0]["ms"]:
                best = (e, x64, o, s)
        e, x64, o, s = best
        e["best_of_sweep"] = True
        entries.append(B.entry(A, b, o, f"{name} ABMC s={s}", precision="fp32", x_ref=x64)[0])

    A, b = synth.workload("knn13_1m", args.seed)
    abmc_sweep("knn13_1m", A, b)
    tb = time.time()
    o = iccg.iccg_order_leiden(A, "cpm", 0.05)
    tb = time.time() - tb
    entries.append(B.entry(A, b, o, "knn13_1m Leiden-CPM gamma=0.05", blocking_s=tb)[0])
    # Leiden-MD: a few dozen communities of 10^4 rows; one timed solve each,
    # over resolutions (the paper's gamma_MD study, Fig. 4)
    for g in [1.0] + ([] if args.no_studies else [float(v) for v in args.md_gammas.split(",") if v]):
        tb = time.time()
        o = iccg.iccg_order_leiden(A, "modularity", g)
        tb = time.time() - tb
        entries.append(B.entry(A, b, o, f"knn13_1m Leiden-MD gamma={g:g}", timed=1, phases=False,
                               blocking_s=tb)[0])
    A, b = synth.workload("stencil27_96", args.seed)
    abmc_sweep("stencil27_96", A, b)
    return entries


def main():
    args = parse()
    s0 = int(args.block_sizes.split(",")[0])
    tag, label = profile_ordering(args)
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary,
                        out_file=traffic_file(args.workload, s0, None if args.ordering == "abmc" else tag),
                        label=label)
        return
    if args.tcc_summary:
        tcc_summary(*args.tcc_summary, os.path.join(ROOT, "profiles", f"l2_hit_sweep_spmv_{args.workload}_{tag}.md"),
                    label)
        return
    if args.trace_summary:
        trace_summary(*args.trace_summary, os.path.join(ROOT, "profiles", f"kernels_iccg_solve_{args.workload}_{tag}.md"),
                      label)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this method is a design note, not a built path.", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_2609_00561_amd import iccg

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    iccg.load()
    dev = torch.device("cuda:0")
    if args.traffic_run:
        traffic_run(args)
        return
    B = Bench(args, dev, iccg, log)

    t0 = time.time()
    A, b = synth.workload(args.workload, args.seed)
    log(f"[bench] workload {args.workload}: n={A.n} nnz={A.nnz} ({time.time() - t0:.1f}s)")

    # --- the paper's Table 2 comparison: ABMC block sizes, node-level MC,
    # Leiden-CPM and Leiden-MD; Table 6 statistics and the Table 8 phase
    # split for every ordering
    sweep = []
    best = None
    for s in [int(v) for v in args.block_sizes.split(",") if v]:
        tb = time.time()
        order = iccg.iccg_order_abmc(A, s)
        tb = time.time() - tb
        e, _ = B.entry(A, b, order, f"ABMC s={s}", timed=max(1, min(args.steps, 3)), blocking_s=tb)
        e["ordering"] = e.pop("matrix")
        sweep.append(e)
        if best is None or e["ms"] < best[0]:
            best = (e["ms"], s, order)
    tb = time.time()
    order_mc = iccg.iccg_order_abmc(A, 1)
    tb = time.time() - tb
    e, _ = B.entry(A, b, order_mc, "MC (ABMC s=1)", timed=2, blocking_s=tb)
    e["ordering"] = e.pop("matrix")
    sweep.append(e)
    # smaller blocks than the configured sweep: reported beside it, not
    # candidates for the headline
    for s in [int(v) for v in args.extra_block_sizes.split(",") if v]:
        tb = time.time()
        order_x = iccg.iccg_order_abmc(A, s)
        tb = time.time() - tb
        e, _ = B.entry(A, b, order_x, f"ABMC s={s} (outside the configured sweep)", timed=2, blocking_s=tb)
        e["ordering"] = e.pop("matrix")
        sweep.append(e)
    if not args.no_leiden:
        for quality, gamma, label in (("cpm", 0.05, "Leiden-CPM gamma=0.05"), ("modularity", 1.0, "Leiden-MD gamma=1")):
            tb = time.time()
            order = iccg.iccg_order_leiden(A, quality, gamma)
            tb = time.time() - tb
            md = quality == "modularity"
            e, _ = B.entry(A, b, order, label, timed=1 if md else 2, phases=not md, blocking_s=tb)
            e["ordering"] = e.pop("matrix")
            sweep.append(e)

    _, s_best, order = best
    ctx = B.ctx(A, order)
    bp = b[order.perm]
    # the same ordering with the hybrid sweeps (one launch per large color,
    # the small colors as one dataflow launch), reported beside; the timed
    # run keeps one launch per color, which the profiles and counters cover
    if not args.no_hybrid:
        ctx_h = B.ctx(A, order, sweep_launch="hybrid")
        _, times_h, res_h, _ = B.time_solves(ctx_h, bp, max(1, min(args.steps, 3)), 1)
        ms_h = 1e3 * float(np.median(times_h))
        log(f"[bench] ABMC s={s_best}, hybrid sweeps: {ms_h:.2f} ms")
        sweep.append({"ordering": f"ABMC s={s_best}, hybrid sweeps", "n_b": order.nblocks,
                      "n_c": order.ncolors, "iters": res_h["iters"], "ms": round(ms_h, 3),
                      "relres_true": res_h["relres_true"]})
        ctx_h.close()
    info = ctx.info()
    log(f"[bench] timed: ABMC s={s_best}, {args.warmup} warmup + {args.steps} steps")
    total, times, res, xd = B.time_solves(ctx, bp, args.steps, args.warmup)
    ms_per_step = 1e3 * total / args.steps
    tms = 1e3 * np.asarray(times)
    x64 = xd.cpu().numpy()

    # instrumented solve: per-launch HIP events on the library's stream
    prof = ctx.profile_solve(torch.tensor(bp, device=dev),
                             torch.zeros(A.n, dtype=torch.float64, device=dev), tol=args.tol)
    # algorithmic bytes per sweep: the substitution's compulsory bytes (library
    # info) plus the fused CG work: the forward sweep also reads q and writes r
    # (16 B/row); the backward sweep also reads r for (r, z)
    sweep_bytes = info["sweep_bytes"]
    fwd_bytes = sweep_bytes + 16.0 * A.n
    bwd_bytes = sweep_bytes + 8.0 * A.n
    fwd_launch_ms = prof["fwd_ms"] / max(prof["fwd_launches"], 1)
    bwd_launch_ms = prof["bwd_ms"] / max(prof["bwd_launches"], 1)
    spmv_launch_ms = prof["spmv_ms"] / max(prof["spmv_launches"], 1)
    nc = info["ncolors"]
    fwd_gbs = (fwd_bytes / nc) / (fwd_launch_ms * 1e-3) / 1e9
    bwd_gbs = (bwd_bytes / nc) / (bwd_launch_ms * 1e-3) / 1e9
    spmv_gbs = info["spmv_bytes"] / (spmv_launch_ms * 1e-3) / 1e9
    kernels = {"k_sweep(forward)": (prof["fwd_ms"], fwd_gbs, fwd_launch_ms, fwd_bytes / nc),
               "k_sweep(backward)": (prof["bwd_ms"], bwd_gbs, bwd_launch_ms, bwd_bytes / nc),
               "k_spmv": (prof["spmv_ms"], spmv_gbs, spmv_launch_ms, info["spmv_bytes"])}
    dom = max(kernels, key=lambda k: kernels[k][0])
    traffic = traffic_for(dom) if s_best == 16 and args.workload == "poisson7_128" else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(kernels[dom][1], 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(kernels[dom][1] / HBM_PEAK_GBS, 4),
                "traffic": round(traffic) if traffic is not None else None,
                "bytes_per_launch": round(kernels[dom][3]),
                "avg_launch_us": round(kernels[dom][2] * 1e3, 3)}
    if traffic is not None:
        # the same launch duration against the counted HBM bytes
        roofline["traffic_GBps"] = round(traffic / (kernels[dom][2] * 1e-3) / 1e9, 1)
        roofline["traffic_frac"] = round(roofline["traffic_GBps"] / HBM_PEAK_GBS, 4)

    # the preconditioner on its own: 100 back-to-back applications on a fixed
    # r; algorithmic bytes = two sweeps of 12 nnz_L + 28 n + 4
    rfix = torch.tensor(np.random.default_rng(args.seed + 7).standard_normal(A.n), device=dev)
    zfix = torch.empty_like(rfix)
    ctx.ic_apply(rfix, zfix)
    torch.cuda.synchronize()
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ea.record()
    for _ in range(100):
        ctx.ic_apply(rfix, zfix)
    eb.record()
    torch.cuda.synchronize()
    apply_us = 1e3 * ea.elapsed_time(eb) / 100
    apply_gbs = 2.0 * sweep_bytes / (apply_us * 1e-6) / 1e9
    ic_apply_entry = {"applies": 100, "us": round(apply_us, 2), "GBps": round(apply_gbs, 1),
                      "frac": round(apply_gbs / HBM_PEAK_GBS, 4)}
    log(f"[bench] ic_apply: {ic_apply_entry}")

    # IC(0) factorization: on the device (the default) and serially on the host
    rp, cl, vl = iccg.iccg_permute(A, order.perm)
    fac = {}
    for host in (False, True):
        with iccg.Context(rp, cl, vl, order.block_ptr, order.color_ptr, host_factor=host) as cf:
            cf.ic0_factor()
            torch.cuda.synchronize()
            tf = []
            for _ in range(3):
                t1 = time.perf_counter()
                cf.ic0_factor()
                torch.cuda.synchronize()
                tf.append(time.perf_counter() - t1)
        fac["host_ms" if host else "device_ms"] = round(1e3 * float(np.median(tf)), 3)
    fac["factor_plus_solve_ms"] = round(fac["device_ms"] + float(np.median(tms)), 3)
    log(f"[bench] IC(0) factor: {fac}")

    out = {
        "metric": "ICCG time-to-solve @1e-8 resid; substitution HBM GB/s; FP32/learned vs FP64",
        "value": round(ms_per_step, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: 3D 7-point lognormal(sigma=1) Poisson 128^3, "
                               f"b uniform[-1,1], seed {args.seed}",
                   "n": A.n, "nnz": A.nnz, "ordering": f"ABMC s={s_best}", "sweep_launch": "per_color",
                   "n_b": info["nblocks"], "n_c": nc, "tol": args.tol},
        "solve_ms": {"mean": round(float(tms.mean()), 3), "sd": round(float(tms.std(ddof=1)) if tms.size > 1 else 0.0, 3),
                     "median": round(float(np.median(tms)), 3), "runs": int(tms.size)},
        "iters": res["iters"],
        "relres_true": res["relres_true"],
        "solves_per_s": round(1e3 / ms_per_step, 3),
        "sweep_GBps": {"forward": round(fwd_gbs, 1), "backward": round(bwd_gbs, 1)},
        "spmv_GBps": round(spmv_gbs, 1),
        "phases_ms": {k: round(prof[k], 3) for k in ("total_ms", "fwd_ms", "bwd_ms", "spmv_ms",
                                                      "other_ms")},
        "roofline": roofline,
        "ic_apply": ic_apply_entry,
        "ic0_factor": fac,
        "sweep": sweep,
    }

    # the 64x64 Laplacian: ten timed solves (latency-bound: 4,096 rows)
    A1, b1 = synth.workload("laplace2d_64", args.seed)
    o1 = iccg.iccg_order_abmc(A1, 64)
    c1 = B.ctx(A1, o1)
    _, t1s, r1, x1d = B.time_solves(c1, b1[o1.perm], 10, 2)
    c1.close()
    x1 = x1d.cpu().numpy()
    t1s = 1e3 * np.asarray(t1s)
    out["laplace2d_64"] = {"ordering": "ABMC s=64", "n_b": o1.nblocks, "n_c": o1.ncolors, "iters": r1["iters"],
                           "ms_mean": round(float(t1s.mean()), 3), "ms_sd": round(float(t1s.std(ddof=1)), 3),
                           "ms_median": round(float(np.median(t1s)), 3), "runs": 10}
    if not args.no_fp32:
        # the FP32 form on the same system: time and distance from the FP64 solution
        c1 = B.ctx(A1, o1, precision="fp32")
        _, t1f, r1f, x1f = B.time_solves(c1, b1[o1.perm], 10, 2)
        c1.close()
        x1f = x1f.cpu().numpy()
        out["laplace2d_64"]["fp32"] = {
            "ms_median": round(1e3 * float(np.median(t1f)), 3), "iters": r1f["iters"],
            "x_rel_diff_vs_fp64": float(np.linalg.norm(x1f - x1) / np.linalg.norm(x1))}
    log(f"[bench] laplace2d_64: {out['laplace2d_64']}")

    if not args.no_fp32:
        e, _ = B.entry(A, b, order, f"{args.workload} ABMC s={s_best}", precision="fp32", timed=3, x_ref=x64)
        e["speedup_vs_fp64"] = round(float(np.median(tms)) / e["ms"], 3)
        out["fp32"] = e

    if not args.no_multi:
        # k right-hand sides in one block solve (repeated solves reusing the
        # ordering and factor): time per solve against k single solves
        k = args.multi_k
        rng = np.random.default_rng(args.seed + 1)
        Bk = rng.uniform(-1, 1, (k, A.n))
        Bk[0] = bp
        Bd = torch.tensor(Bk, device=dev)
        Xd = torch.zeros_like(Bd)
        ctx.solve_multi(Bd, Xd, tol=args.tol)
        Xd.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rm = ctx.solve_multi(Bd, Xd, tol=args.tol)
        torch.cuda.synchronize()
        tmulti = 1e3 * (time.perf_counter() - t1)
        single_iters = []
        t_single = 0.0
        for j in range(k):
            xj = torch.zeros(A.n, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rj = ctx.solve(Bd[j].contiguous(), xj, tol=args.tol)
            torch.cuda.synchronize()
            t_single += time.perf_counter() - t1
            single_iters.append(rj["iters"])
        out["multi_rhs"] = {"k": k, "block_solve_ms": round(tmulti, 3), "per_rhs_ms": round(tmulti / k, 3),
                            "k_single_solves_ms": round(1e3 * t_single, 3),
                            "speedup_vs_single_solves": round(1e3 * t_single / tmulti, 3),
                            "iters": [int(v) for v in rm["iters"]], "single_iters": single_iters,
                            "max_relres_true": float(np.max(rm["relres_true"]))}
        # the preconditioner on its own: one block application (forward and
        # backward sweeps over k columns, the schedule read once) against one
        # single-column application; algorithmic bytes = the two schedules
        # (12 nnz_L + 12 n + 4 each) + 32 n per column (r in, y out, y in,
        # z out), so the intensity grows with k
        Rk = torch.tensor(rng.standard_normal((k, A.n)), device=dev)
        Zk = torch.empty_like(Rk)
        z1 = torch.empty(A.n, dtype=torch.float64, device=dev)

        def _per_call_us(fn, reps=20):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return 1e3 * e0.elapsed_time(e1) / reps

        us_block = _per_call_us(lambda: ctx.ic_apply_multi(Rk, Zk))
        us_single = _per_call_us(lambda: ctx.ic_apply(Rk[0], z1))
        nnz_l = (A.nnz - A.n) // 2
        by_block = 2 * (12 * nnz_l + 12 * A.n + 4) + 32 * A.n * k
        by_single = 2 * (12 * nnz_l + 28 * A.n + 4)
        out["multi_rhs"]["ic_apply"] = {
            "block_us": round(us_block, 1), "single_us": round(us_single, 1),
            "per_column_us": round(us_block / k, 1),
            "block_GBps": round(by_block / us_block / 1e3, 1),
            "single_GBps": round(by_single / us_single / 1e3, 1),
            "block_frac": round(by_block / us_block / 1e3 / HBM_PEAK_GBS, 4),
            "single_frac": round(by_single / us_single / 1e3 / HBM_PEAK_GBS, 4),
            "bytes_block": int(by_block), "bytes_single": int(by_single)}
        log(f"[bench] multi-RHS: {out['multi_rhs']}")

    if not args.no_leiden and not args.no_studies:
        # Leiden seed sensitivity (Table 4) and the CPM resolution (Table 10,
        # Fig. 5) on the timed matrix
        seeds = []
        for sd in [int(v) for v in args.leiden_seeds.split(",") if v]:
            tb = time.time()
            o = iccg.iccg_order_leiden(A, "cpm", 0.05, seed=sd)
            tb = time.time() - tb
            e, _ = B.entry(A, b, o, f"Leiden-CPM gamma=0.05 seed={sd}", timed=1, phases=False, blocking_s=tb)
            seeds.append(e)
        def rng_of(key):
            v = [e[key] for e in seeds]
            return [min(v), max(v)]
        out["leiden_seed_study"] = {"ordering": "Leiden-CPM gamma=0.05", "entries": seeds,
                                    "n_b_range": rng_of("n_b"), "n_c_range": rng_of("n_c"),
                                    "iters_range": rng_of("iters"), "ms_range": rng_of("ms")}
        cpm = []
        for g in [float(v) for v in args.cpm_gammas.split(",") if v]:
            tb = time.time()
            o = iccg.iccg_order_leiden(A, "cpm", g)
            tb = time.time() - tb
            cpm.append(B.entry(A, b, o, f"Leiden-CPM gamma={g:g}", timed=1, phases=False, blocking_s=tb)[0])
        out["leiden_cpm_gamma_study"] = cpm

    if not args.no_other_matrices:
        out["other_matrices"] = other_matrices(B, args, synth)

    if not args.no_learned:
        from paper_2609_00561_amd import learned
        tl0 = time.time()
        ctxs = []
        for kk in range(args.learned_matrices):
            Ak, _ = synth.workload("lognormal7_32", kk)
            ctxs.append(learned.build_context(Ak, 64)[0])
        t_setup = time.time() - tl0
        evals = []
        with iccg.Network(learned.init_params(0)) as net:
            tt = time.time()
            hist = learned.train(net, ctxs, args.learned_epochs, lr=1e-3, seed=0, log=log)
            torch.cuda.synchronize()
            t_train = time.time() - tt
            for c_ in ctxs:
                c_.close()
            # unseen seeds (10,000 and up) at sigma 0.5, 1, 2 on 64^3 and 128^3
            for m in (64, 128):
                for sigma in (0.5, 1.0, 2.0):
                    for j in range(args.learned_seeds):
                        seed = 10000 + 100 * int(2 * sigma) + j
                        Ae = synth.grid3d_7pt_lognormal(m, m, m, sigma, 1e-6, np.random.default_rng(seed))
                        be = synth.uniform_rhs(Ae.n, np.random.default_rng(seed + 1))
                        ce, oe = learned.build_context(Ae, 64)
                        with ce:
                            ev = learned.solve_both(net, ce, torch.tensor(be[oe.perm], device=dev), tol=args.tol)
                        ev["matrix"] = f"{m}^3 sigma={sigma:g} seed {seed} (unseen), ABMC s=64"
                        evals.append(ev)
                        log(f"[bench] learned form on {ev['matrix']}: {ev}")
            ev = learned.solve_both(net, ctx, torch.tensor(bp, device=dev), tol=args.tol)
            ev["matrix"] = f"{args.workload} (timed matrix), ABMC s={s_best}"
            evals.append(ev)

        def _fmt(ev):
            return {
                "matrix": ev["matrix"],
                "plain_iters": ev["plain_iters"], "plain_ms": round(ev["plain_ms"], 3),
                "learned_iters": ev.get("learned_iters"),
                "iters_delta": (ev["learned_iters"] - ev["plain_iters"]) if "learned_iters" in ev else None,
                "learned_ms": round(ev["learned_ms"], 3) if "learned_ms" in ev else None,
                "inference_ms": round(ev["infer_ms"], 3), "feature_setup_ms": round(ev["setup_ms"], 3),
                "pivot_ok": ev["pivot_ok"],
                "kept": ev["kept"], "x_rel_diff_vs_plain": ev.get("x_rel_diff"),
                "speedup_vs_fp64_incl_inference": (round(ev["plain_ms"] / (ev["learned_ms"] + ev["infer_ms"]), 3)
                                                   if "learned_ms" in ev else None),
            }
        ev_out = [_fmt(ev) for ev in evals]
        deltas = [e["iters_delta"] for e in ev_out if e["iters_delta"] is not None]
        out["learned"] = {
            "train": {"matrices": args.learned_matrices, "grid": "32^3", "epochs": args.learned_epochs,
                      "probes": "8 per step, IC(0)-smoothed Gaussian",
                      "probe_loss_by_epoch": [round(v, 5) for v in hist],
                      "train_s": round(t_train, 2), "setup_s": round(t_setup, 2)},
            "eval": ev_out,
            "iters_delta_summary": {"min": min(deltas), "max": max(deltas),
                                    "mean": round(float(np.mean(deltas)), 2), "n": len(deltas)},
        }
        log(f"[bench] learned form: {out['learned']['iters_delta_summary']}")

    if not args.no_cpu:
        import oracle
        model, avail, total_cpus = cpu_info()
        Ap = oracle.permute(A, order.perm)
        lval, _ = oracle.ic0(Ap)
        kit = args.cpu_iters
        tc = time.perf_counter()
        r = oracle.pcg(Ap, lval, bp, tol=0.0, maxit=kit)
        tc = time.perf_counter() - tc
        per_iter = tc / max(r.iters, 1)
        est_ms = per_iter * res["iters"] * 1e3
        out["cpu_baseline"] = {
            "value": round(est_ms, 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"{r.iters} PCG iterations of the serial FP64 oracle on the same permuted "
                      f"matrix ({tc:.1f} s), scaled to the GPU solve's {res['iters']} iterations",
            "cpu_model": model, "nproc": avail, "cpus_on_host": total_cpus,
            "phase_s": [round(v, 3) for v in r.phase_s.tolist()],
        }
        # the 64x64 Laplacian: whole oracle solves, ten timed runs
        A1, b1 = synth.workload("laplace2d_64", args.seed)
        o1 = oracle.order_abmc(A1, 64)
        A1p = oracle.permute(A1, o1.perm)
        l1, _ = oracle.ic0(A1p)
        b1p = np.ascontiguousarray(b1[o1.perm])
        t1s = []
        for _ in range(10):
            t1 = time.perf_counter()
            r1 = oracle.pcg(A1p, l1, b1p, tol=args.tol, maxit=10000)
            t1s.append(1e3 * (time.perf_counter() - t1))
        out["cpu_baseline"]["laplace2d_64_solve_ms"] = {
            "mean": round(float(np.mean(t1s)), 3), "sd": round(float(np.std(t1s, ddof=1)), 3),
            "median": round(float(np.median(t1s)), 3), "runs": 10, "iters": int(r1.iters)}
        log(f"[bench] CPU oracle: {per_iter * 1e3:.1f} ms/iter -> {est_ms / 1e3:.1f} s estimated")
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
