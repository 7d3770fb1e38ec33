"""Build the HIP library librhipm.so in-tree for gfx950 with hipcc.

Usage: python -m paper_2203_11875_amd.build  (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librhipm.so")
SOURCES = ["analysis.cpp", "kernels.hip", "chol.hip", "ipm.hip", "redlin.hip", "rhipm.cpp"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build librhipm.so)")


def _flags() -> list:
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source for gfx950 (one hipcc process per source, in
    parallel) and link librhipm.so next to this file. incremental: keep the
    objects that are newer than their source and every header (for
    development; the default compiles everything)."""
    from concurrent.futures import ThreadPoolExecutor
    odir = os.path.join(HERE, "_build")
    os.makedirs(odir, exist_ok=True)
    cc = hipcc()

    headers = [os.path.join(d, f) for d in (CSRC, os.path.join(ROOT, "include"))
               for f in os.listdir(d) if f.endswith((".h", ".hpp"))]
    newest_header = max(os.path.getmtime(h) for h in headers)

    def compile_one(src):
        obj = os.path.join(odir, os.path.splitext(src)[0] + ".o")
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(
                newest_header, os.path.getmtime(os.path.join(CSRC, src))):
            return obj, subprocess.CompletedProcess([], 0, "", "")
        cmd = [cc] + _flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return obj, subprocess.run(cmd, capture_output=True, text=True)

    workers = max(1, min(len(SOURCES), os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [r for _, r in results if r.returncode != 0]
    if failed:
        for r in failed:
            sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building librhipm.so")
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for o, _ in results] + \
        ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking librhipm.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
