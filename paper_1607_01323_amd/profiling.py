"""Summaries of rocprofv3 output for the committed profiles (host-side helper).

``python -m paper_1607_01323_amd.profiling stats <kernel_stats.csv> <out.md> --cmd "..."``
    writes the per-kernel duration table of a --kernel-trace --stats run.
``python -m paper_1607_01323_amd.profiling trace <kernel_trace.csv> <out.md> --cmd "..."``
    writes per-configuration rows (kernel, grid size, workgroup size) of a
    --kernel-trace run, so launches of one kernel on different meshes are not
    averaged together.
``python -m paper_1607_01323_amd.profiling counters <out.md> <counter_collection.csv>... --trace <kernel_trace.csv> --cmd "..."``
    per-configuration means of SQ_* counters (per dispatch), with the fp64 /
    fp32 operation counts they imply and, from the durations of the trace run,
    the achieved FLOP rates against the chip's peaks.
``python -m paper_1607_01323_amd.profiling window <kernel_trace.csv> <out.md> --kernel K --grid G --skip S --count C --cmd "..."``
    durations of launches S .. S+C-1 of one kernel and grid size, in launch
    order (the timed loop of a benchmark, apart from other uses of the kernel).
``python -m paper_1607_01323_amd.profiling pmc <fetch_csv> <write_csv> <out.json> --cmd-fetch ... --cmd-write ...``
    reduces FETCH_SIZE / WRITE_SIZE counter collections (KiB per dispatch) to
    a per-kernel average and the copy-kernel calibration factor, tagged with
    the hash of the kernel sources they were taken on.
"""
import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["sipg_cart.hip", "conv.hip", "sipg_metric.hip"]


def kernel_hash(name):
    p = os.path.join(HERE, "csrc", name)
    if not os.path.exists(p):
        return None
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def short_name(k):
    k = k.replace("void ", "").replace("dgmf::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    return k.split("(")[0]


def stats_table(csv_path, out_md, cmd):
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{cmd}`", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short_name(r['Name'])[:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    return ""


def _grid(row):
    """Total work-items of the launch (counter files give the total, trace files
    the three extents), as a string, so that both files key alike."""
    g = _col(row, "Grid_Size")
    if g:
        return str(int(float(g)))
    t = 1
    for a in "XYZ":
        t *= int(float(_col(row, f"Grid_Size_{a}") or "1"))
    return str(t)


def _wg(row):
    g = _col(row, "Workgroup_Size")
    if g:
        return g
    return "x".join(_col(row, f"Workgroup_Size_{a}") or "1" for a in "XYZ")


def trace_durations(csv_path):
    """{(kernel, grid): [durations in ns]} from a kernel_trace.csv."""
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        k = short_name(_col(r, "Kernel_Name"))
        d = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        agg[(k, _grid(r), _wg(r))].append(d)
    return agg


def trace_table(csv_path, out_md, cmd):
    agg = trace_durations(csv_path)
    total = sum(sum(v) for v in agg.values()) or 1.0
    rows = sorted(agg.items(), key=lambda kv: -sum(kv[1]))
    lines = ["# rocprofv3 kernel trace, per configuration", "", f"Command: `{cmd}`", "",
             "One row per kernel and launch shape (grid size = total work-items), so launches on "
             "different meshes are listed apart.", "",
             "| kernel | grid | workgroup | calls | avg (us) | median (us) | min (us) | max (us) | share % |",
             "|---|---|---|---|---|---|---|---|---|"]
    for (k, g, wg), v in rows:
        v = sorted(v)
        lines.append(f"| `{k[:80]}` | {g} | {wg} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | "
                     f"{v[len(v) // 2] / 1e3:.2f} | {v[0] / 1e3:.2f} | {v[-1] / 1e3:.2f} | "
                     f"{100.0 * sum(v) / total:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def window_table(csv_path, out_md, kernel, grid, skip, count, cmd):
    rows = [r for r in csv.DictReader(open(csv_path))
            if short_name(_col(r, "Kernel_Name")) == kernel and _grid(r) == str(grid)]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    sel = rows[skip:skip + count]
    d = sorted((float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3 for r in sel)
    if not d:
        raise SystemExit("no launches of %s with grid %s" % (kernel, grid))
    period = (float(sel[-1]["Start_Timestamp"]) - float(sel[0]["Start_Timestamp"])) / 1e3 / max(1, len(sel) - 1)
    lines = ["# rocprofv3 kernel trace, one timed loop", "", f"Command: `{cmd}`", "",
             f"Launches {skip} to {skip + len(sel) - 1} (in launch order) of `{kernel}` with grid {grid} "
             f"({len(rows)} launches of that kernel and grid in the run).", "",
             "| launches | mean (us) | median (us) | min (us) | max (us) | start-to-start (us) |", "|---|---|---|---|---|---|",
             f"| {len(d)} | {sum(d) / len(d):.2f} | {d[len(d) // 2]:.2f} | {d[0]:.2f} | {d[-1]:.2f} | {period:.2f} |"]
    open(out_md, "w").write("\n".join(lines) + "\n")


FLOP_F64 = {"SQ_INSTS_VALU_ADD_F64": 1, "SQ_INSTS_VALU_MUL_F64": 1, "SQ_INSTS_VALU_FMA_F64": 2,
            "SQ_INSTS_VALU_TRANS_F64": 1}
FLOP_F32 = {"SQ_INSTS_VALU_ADD_F32": 1, "SQ_INSTS_VALU_MUL_F32": 1, "SQ_INSTS_VALU_FMA_F32": 2,
            "SQ_INSTS_VALU_TRANS_F32": 1}


def counters_table(out_md, csv_paths, trace_csv, cmd, peaks=(78.6, 157.3)):
    """Mean counter value per dispatch for each (kernel, grid); FLOPs per dispatch as
    64 lanes x the weighted VALU instruction counts (the counters count wavefront
    instructions); rates from the trace run's median durations."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    regs = {}
    for p in csv_paths:
        for r in csv.DictReader(open(p)):
            key = (short_name(_col(r, "Kernel_Name")), _grid(r))
            vals[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
            regs[key] = (_col(r, "VGPR_Count", "Arch_VGPR_Count"), _col(r, "Accum_VGPR_Count"),
                         _col(r, "SGPR_Count"), _col(r, "LDS_Block_Size", "Group_Segment_Size"),
                         _col(r, "Scratch_Size", "Private_Segment_Size"))
    dur = {}
    if trace_csv:
        for (k, g, _), v in trace_durations(trace_csv).items():
            v = sorted(v)
            dur[(k, g)] = v[len(v) // 2]
    names = sorted({c for d in vals.values() for c in d})
    lines = ["# rocprofv3 counters, per configuration", "", f"Command: `{cmd}`", "",
             "Mean value per dispatch.  fp64 / fp32 FLOP = 64 x (ADD + MUL + TRANS + 2 FMA) of the "
             "wavefront instruction counts (every lane counted as active); the rate uses the median "
             "duration of the same kernel and grid in the kernel-trace run.", ""]
    hdr = ["kernel", "grid", "VGPR", "AGPR", "SGPR", "LDS", "scratch"] + names + \
          ["fp64 GFLOP", "fp64 TFLOP/s", "fp64 frac", "fp32 GFLOP", "fp32 TFLOP/s", "fp32 frac"]
    lines.append("| " + " | ".join(hdr) + " |")
    lines.append("|" + "---|" * len(hdr))
    for key in sorted(vals):
        d = {c: sum(v) / len(v) for c, v in vals[key].items()}
        f64 = 64.0 * sum(w * d.get(c, 0.0) for c, w in FLOP_F64.items())
        f32 = 64.0 * sum(w * d.get(c, 0.0) for c, w in FLOP_F32.items())
        t = dur.get(key)
        r64 = f"{f64 / t / 1e3:.2f}" if t and f64 else ""
        r32 = f"{f32 / t / 1e3:.2f}" if t and f32 else ""
        fr64 = f"{f64 / t / 1e3 / peaks[0]:.3f}" if t and f64 else ""
        fr32 = f"{f32 / t / 1e3 / peaks[1]:.3f}" if t and f32 else ""
        row = [f"`{key[0][:70]}`", key[1], *regs.get(key, ("",) * 5)] + [f"{d.get(c, float('nan')):.4g}" for c in names]
        row += [f"{f64 / 1e9:.4g}", r64, fr64, f"{f32 / 1e9:.4g}", r32, fr32]
        lines.append("| " + " | ".join(str(x) for x in row) + " |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_kernel(csv_path, counter):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter:
            agg[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def pmc_summary(fetch_csv, write_csv, out_json, cmd_fetch, cmd_write, copy_bytes):
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")
    # calibration kernels of known traffic: torch's uniform_ fill writes copy_bytes,
    # torch's sum reads copy_bytes (the largest dispatch of each kind)
    kr = [k for k in f if "reduce" in k.lower()]
    f = {k: max(v, 0.0) for k, v in f.items()}
    kw_ = [k for k in w if "distribution" in k.lower()]
    cal = {}
    if kr and kw_:
        kf = max(kr, key=lambda k: f[k])
        kw = max(kw_, key=lambda k: w[k])
        cal = {"read_kernel": kf, "write_kernel": kw, "bytes": copy_bytes,
               "fetch_factor": copy_bytes / (f[kf] * 1024.0), "write_factor": copy_bytes / (w[kw] * 1024.0)}
    out = {"fetch_kib_per_dispatch": f, "write_kib_per_dispatch": w, "calibration": cal,
           "kernel_hashes": {s: kernel_hash(s) for s in KERNEL_SOURCES},
           "commands": {"fetch": cmd_fetch, "write": cmd_write}}
    json.dump(out, open(out_json, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("out")
    a.add_argument("--cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("out")
    t.add_argument("--cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("csvs", nargs="+")
    c.add_argument("--trace", default=None)
    c.add_argument("--cmd", required=True)
    wdw = sub.add_parser("window")
    wdw.add_argument("csv")
    wdw.add_argument("out")
    wdw.add_argument("--kernel", required=True)
    wdw.add_argument("--grid", required=True)
    wdw.add_argument("--skip", type=int, default=0)
    wdw.add_argument("--count", type=int, required=True)
    wdw.add_argument("--cmd", required=True)
    b = sub.add_parser("pmc")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("out")
    b.add_argument("--cmd-fetch", required=True)
    b.add_argument("--cmd-write", required=True)
    b.add_argument("--copy-bytes", type=float, required=True)
    args = ap.parse_args()
    if args.what == "stats":
        stats_table(args.csv, args.out, args.cmd)
    elif args.what == "trace":
        trace_table(args.csv, args.out, args.cmd)
    elif args.what == "window":
        window_table(args.csv, args.out, args.kernel, args.grid, args.skip, args.count, args.cmd)
    elif args.what == "counters":
        counters_table(args.out, args.csvs, args.trace, args.cmd)
    else:
        pmc_summary(args.fetch_csv, args.write_csv, args.out, args.cmd_fetch, args.cmd_write, args.copy_bytes)
