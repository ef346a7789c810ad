"""Build the HIP library ``libhelmsep.so`` in-tree for gfx950.

Usage: ``python -m paper_1909_01299_amd.build`` (or ``build()`` from Python).
Every call compiles every source from scratch: one hipcc process per source
file (in parallel, objects under ``_build/``), then one link.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhelmsep.so")
OBJ = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off for every device function
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".cpp", ".hip")):
            out.append(os.path.join(CSRC, name))
    return out


def _filter(text: str):
    return [l for l in text.splitlines() if "packed-fp32-ops" not in l]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = []
    for src in sources():
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        if os.path.exists(obj):
            os.remove(obj)
        jobs.append((src, obj, [hipcc, *HIPCC_FLAGS, *inc, "-c", "-o", obj, src]))

    def run(job):
        src, obj, cmd = job
        if verbose:
            print(" ".join(cmd), flush=True)
        return src, subprocess.run(cmd, capture_output=True, text=True)

    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        results = list(pool.map(run, jobs))
    msgs = []
    failed = False
    for src, res in results:
        lines = _filter(res.stdout + res.stderr)
        if res.returncode != 0:
            failed = True
        if lines:
            msgs.append(f"--- {os.path.basename(src)}\n" + "\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[j[1] for j in jobs]]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + "\n".join(_filter(res.stdout + res.stderr)))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
