"""Build libdgmf.so (HIP kernels + C-ABI) in-tree for gfx950 with hipcc.

Usage: python paper_1607_01323_amd/build.py [--jobs N] [--debug]
(standalone: it does not import the package, whose import needs the library)
"""
import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libdgmf.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]
# gfx950 only; packed fp32 instructions are disabled for every device pass.
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def compile_one(src, opt):
    obj = os.path.join(OBJDIR, src + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE, opt, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r.returncode, r.stdout + r.stderr, cmd


def build(jobs=8, debug=False, verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    opt = "-O1" if debug else "-O3"
    srcs = sources()
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        results = list(ex.map(lambda s: compile_one(s, opt), srcs))
    failed = [r for r in results if r[2] != 0]
    for src, _, rc, out, cmd in results:
        msgs = [l for l in out.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l]
        if rc != 0 or (verbose and msgs):
            print(f"== {src} (rc={rc})\n" + "\n".join(msgs), file=sys.stderr)
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(r[0] for r in failed))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, *DEVICE, "-shared", "-fPIC", "-o", tmp, *[r[1] for r in results]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.debug, a.verbose))
