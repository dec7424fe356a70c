"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the library with the host half of every source instrumented (each -fsanitize= after
-Xarch_host: the device code is compiled as in the product build), links the C driver
tests/host/sanitize_driver.c against it, and runs the driver: descriptor validation over
valid, invalid and extreme descriptors, and every entry point with missing arguments.
Those calls never reach the device, so this runs without a GPU; the device-facing paths are
exercised by the GPU tests on the uninstrumented build.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    import sys
    sys.path.insert(0, ROOT)
    from paper_1802_01685_amd import build as B
    hipcc = _hipcc()
    if hipcc is None or not os.path.exists(CLANG):
        pytest.skip("no ROCm toolchain")
    out = tmp_path_factory.mktemp("asan")
    common = [c for c in B.COMMON if c != "-O3"] + ["-O1", "-g", "-fno-omit-frame-pointer"]
    objs, cmds = [], []
    for src in B.SOURCES:
        obj = str(out / (src + ".o"))
        objs.append(obj)
        cmds.append([hipcc, *common, *B.DEVICE, *SAN, "-c", os.path.join(B.CSRC, src), "-o", obj])

    def run(cmd):
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        for r in ex.map(run, cmds):
            assert r.returncode == 0, r.stderr[-3000:]
    lib = str(out / "libbfly.so")
    r = run([hipcc, *B.DEVICE, *SAN, "-shared-libsan", "-shared", "-fPIC", *objs, "-lpthread",
             "-o", lib])
    assert r.returncode == 0, r.stderr[-3000:]
    return out, lib


def test_host_abi_under_asan_and_ubsan(sanitized_lib):
    out, lib = sanitized_lib
    exe = str(out / "driver")
    rt = subprocess.run([CLANG, "-print-resource-dir"], capture_output=True,
                        text=True).stdout.strip()
    rtdir = os.path.join(rt, "lib", "linux")       # the shared sanitizer runtimes
    r = subprocess.run([CLANG, "-std=c99", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-shared-libsan",
                        "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "host", "sanitize_driver.c"),
                        lib, f"-Wl,-rpath,{out}", f"-Wl,-rpath,{rtdir}", "-lm", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ)
    # the HIP runtime keeps allocations until exit; memory errors and UB still abort
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    assert "0 failures" in run.stdout
