"""Build libtk.so (hand-written HIP for gfx950) in-tree.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection switched off, hardware floating-point atomics enabled for LDS
accumulation, and no fast-math (FP64 division and square root stay IEEE).
The sources compile to objects in parallel (under _build/) and are linked
into one shared library.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtk.so")
OBJ = os.path.join(ROOT, "_build", "tk")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-function"]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _filter(text):
    # the host pass does not know the packed-FP32 feature; that note is harmless
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def _compile(src, extra):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, *extra, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, obj, res.returncode, _filter(res.stdout + res.stderr)


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = max(1, min(len(srcs), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as pool:
        results = list(pool.map(lambda s: _compile(s, list(extra)), srcs))
    failed = False
    for cmd, obj, rc, out in results:
        if verbose:
            print(" ".join(cmd), flush=True)
        if out.strip() and (verbose or rc):
            print(out, file=sys.stderr)
        failed |= rc != 0
    if failed:
        raise RuntimeError("hipcc failed")
    link = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp",
            *[r[1] for r in results]]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, capture_output=True, text=True)
    out = _filter(res.stdout + res.stderr)
    if out.strip() and (verbose or res.returncode):
        print(out, file=sys.stderr)
    if res.returncode:
        raise RuntimeError("hipcc link failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
