"""Summaries of rocprofv3 output for the committed profiles (host-side helper).

``python -m paper_1607_01323_amd.profiling stats <kernel_stats.csv> <out.md> --cmd "..."``
    writes the per-kernel duration table of a --kernel-trace --stats run.
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
    else:
        pmc_summary(args.fetch_csv, args.write_csv, args.out, args.cmd_fetch, args.cmd_write, args.copy_bytes)
