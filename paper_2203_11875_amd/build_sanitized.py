"""Host-sanitised build of the library, for checking the host code on a CPU.

Compiles every source like build.py, with AddressSanitizer and
UndefinedBehaviorSanitizer on the host side only (the device code is built as
usual), into librhipm_san.so next to this file. run_host_tests() then runs
tests/test_host_symbolic.py (the symbolic analysis, the host refactorisation
and sweeps, the condensation-record emulation, the rh_symbolic_* entry points)
against that library in a fresh Python process with the sanitiser runtime
preloaded; any report fails the run.

Usage: python -m paper_2203_11875_amd.build_sanitized
"""
from __future__ import annotations

import os
import subprocess
import sys

from .build import CSRC, HERE, ROOT, SOURCES, _flags, hipcc

LIB = os.path.join(HERE, "librhipm_san.so")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def build() -> str:
    from concurrent.futures import ThreadPoolExecutor
    odir = os.path.join(HERE, "_build_san")
    os.makedirs(odir, exist_ok=True)
    cc = hipcc()

    def one(src):
        obj = os.path.join(odir, os.path.splitext(src)[0] + ".o")
        cmd = [cc] + _flags() + SAN + ["-O1", "-g", "-c", os.path.join(CSRC, src), "-o", obj]
        return obj, subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        res = list(ex.map(one, SOURCES))
    bad = [r for _, r in res if r.returncode != 0]
    if bad:
        for r in bad:
            sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("sanitised build failed")
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN + [o for o, _ in res] + \
        ["-o", LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("sanitised link failed")
    return LIB


def _runtime(name: str) -> str:
    out = subprocess.run([os.path.join(os.path.dirname(hipcc()), "..", "lib", "llvm", "bin",
                                       "clang++"), f"-print-file-name={name}"],
                         capture_output=True, text=True).stdout.strip()
    if not out or not os.path.exists(out):
        raise RuntimeError(f"{name} not found")
    return out


def run_host_tests() -> int:
    """tests/test_host_symbolic.py against librhipm_san.so; returns pytest's
    exit status."""
    env = dict(os.environ)
    env["LD_PRELOAD"] = _runtime("libclang_rt.asan-x86_64.so")
    env["RHIPM_LIB"] = LIB
    # Python's own allocations are not leak-checked; any other report aborts
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_host_symbolic.py")]
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    print(build(), flush=True)
    sys.exit(run_host_tests())
