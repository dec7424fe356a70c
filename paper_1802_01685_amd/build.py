"""Builds libbfly.so (the HIP kernels and the C-ABI runtime) for gfx950, in-tree.

    python -m paper_1802_01685_amd.build

Compiles csrc/bfly_kernels.hip, csrc/bfly_api.cpp and csrc/bfly_server.cpp with hipcc and
links them into
paper_1802_01685_amd/libbfly.so next to this file.  Always recompiles.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libbfly.so")

ARCH = "gfx950"
SOURCES = ["bfly_kernels.hip", "bfly_fft.hip", "bfly_tails.hip", "bfly_coinc.hip",
           "bfly_noalloc.hip", "bfly_api.cpp", "bfly_server.cpp"]
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-ffp-contract=off",
    f"-I{INCLUDE}", f"-I{CSRC}",
]
# Packed FP32 arithmetic is kept off in all device code.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if out.strip():
        print(out, file=sys.stderr)


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    with tempfile.TemporaryDirectory(prefix="bfly_build_") as tmp:
        objs = [os.path.join(tmp, os.path.basename(src) + ".o") for src in SOURCES]
        cmds = [[hipcc, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj]
                for src, obj in zip(SOURCES, objs)]
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0") or 0) or
                          (os.cpu_count() or 1)))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_run, c) for c in cmds]:
                f.result()
        tmp_lib = os.path.join(tmp, "libbfly.so")
        _run([hipcc, *DEVICE, "-shared", "-fPIC", *objs, "-lpthread", "-o", tmp_lib])
        shutil.copyfile(tmp_lib, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
