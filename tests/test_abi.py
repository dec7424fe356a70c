"""CPU checks of the C-ABI library: it loads, exports every entry point include/bfly.h
declares, and its host-side validation answers without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfly.h")
LIB = os.path.join(ROOT, "paper_1802_01685_amd", "libbfly.so")


def declared_symbols():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:bf_status|const char\*)\s+(bf_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libbfly.so is not built (run `python -m paper_1802_01685_amd.build`)")
    from paper_1802_01685_amd import bfly
    return bfly


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("bf_bank_bytes", "bf_bank_create", "bf_bank_info", "bf_bank_destroy",
              "bf_workspace_bytes", "bf_search_segment", "bf_search_batch", "bf_plan",
              "bf_set_timing", "bf_kernel_times", "bf_last_error", "bf_server_create",
              "bf_server_request_bytes", "bf_submit", "bf_poll", "bf_fetch", "bf_cancel",
              "bf_server_stats", "bf_server_destroy"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    L = ctypes.CDLL(LIB)
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert sorted(lib.EXPORTED) == declared_symbols()


def test_bank_bytes_and_validation_on_host(lib):
    from synth import bank_params
    d = lib.make_desc(bank_params("strain"), "bf16x3")
    # K_pad * L_pad * 4 bytes + a 256-byte status word
    assert lib.bank_bytes(d) == 65536 * 4096 * 4 + 256
    d3 = lib.make_desc(bank_params("light_curve_share"), "fp32")
    assert lib.bank_bytes(d3) == 720000 * 2016 * 4 + 256   # L_pad = 2016 (multiple of 32)
    d8 = lib.make_desc(bank_params("strain"), "fp8")
    # one byte per tap, then an int32 exponent and a float template sum per template, then
    # the status word
    assert lib.bank_bytes(d8) == 65536 * 4096 + 65536 * 8 + 256
    # FFT form: a float32 complex spectrum of N/2 + 1 bins per template (rows of N/2 + 2),
    # N = 8192 for L = 4096
    df = lib.make_desc(bank_params("strain"), "fft")
    assert lib.bank_bytes(df) == 65536 * (4096 + 2) * 8 + 256
    # N = 8192 for every template length; BF_FFT_POINTS = N picks a shorter transform where
    # it holds a template (the small strain-like bank: 256 templates of L = 512)
    ds = lib.make_desc(bank_params("small_strain"), "fft")
    assert lib.bank_bytes(ds) == 256 * (4096 + 2) * 8 + 256
    import os
    try:
        os.environ["BF_FFT_POINTS"] = "2048"
        assert lib.bank_bytes(ds) == 256 * (1024 + 2) * 8 + 256
        os.environ["BF_FFT_POINTS"] = "1024"
        assert lib.bank_bytes(ds) == 256 * (512 + 2) * 8 + 256
        os.environ["BF_FFT_POINTS"] = "1024"
        assert lib.bank_bytes(df) == 65536 * (4096 + 2) * 8 + 256   # L = 4096: too short
    finally:
        os.environ.pop("BF_FFT_POINTS", None)
    df.L = 4097
    with pytest.raises(lib.BflyError):
        lib.bank_bytes(df)
    # F16F8: four bytes per tap (fp16 + two e4m3 codes), the FP8 side tables; L_pad = 2048
    # (multiple of 64) for L = 2000; L is capped by the strip's LDS footprint
    dm = lib.make_desc(bank_params("light_curve_share"), "f16f8")
    assert lib.bank_bytes(dm) == 720000 * 2048 * 4 + 720000 * 8 + 256
    dm.L = 4225
    with pytest.raises(lib.BflyError):
        lib.bank_bytes(dm)
    dm.L = 4224
    assert lib.bank_bytes(dm) == 720000 * 4224 * 4 + 720000 * 8 + 256
    # F16F6: fp16 (2 bytes) + two 6-bit codes per tap = 3.5 bytes, the same side tables
    d6 = lib.make_desc(bank_params("light_curve_share"), "f16f6")
    assert lib.bank_bytes(d6) == 720000 * 2048 * 7 // 2 + 720000 * 8 + 256
    d6.L = 4225
    with pytest.raises(lib.BflyError):
        lib.bank_bytes(d6)
    for bad in ({"L": 0}, {"L": 9000}, {"n_f0": 0}, {"fs": -1.0}, {"shard_index": 12},
                {"f0_max": 1.0}, {"precision": 7}):
        q = lib.make_desc(bank_params("strain"), "fp32")
        for k, v in bad.items():
            setattr(q, k, v)
        with pytest.raises(lib.BflyError) as e:
            lib.bank_bytes(q)
        assert e.value.status == lib.BF_EINVAL
        assert lib.last_error() != ""


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The binding has no fallback: with the shared library absent it raises, and no module
    of the package imports the oracle."""
    import os
    import subprocess
    import sys
    code = (
        "import sys\n"
        "from paper_1802_01685_amd import bfly\n"
        f"bfly.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
        "bfly._lib = None\n"
        "try:\n"
        "    bfly.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(1)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True)
    assert r.returncode == 0 and "raised" in r.stdout, r.stdout + r.stderr
    pkg = os.path.join(root, "paper_1802_01685_amd")
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            assert "oracle" not in open(os.path.join(pkg, name)).read(), name


C_PROGRAM = r"""
#include <stdio.h>
#include "bfly.h"

int main(void) {
  bf_bank_desc d = {0};
  d.fs = 4096.0; d.L = 4096; d.n_f0 = 256; d.n_fdot = 256;
  d.shard_index = 0; d.shard_count = 1; d.precision = BF_BF16X3;
  d.f0_min = 50.0; d.f0_max = 2000.0; d.fdot_min = -2000.0; d.fdot_max = 2000.0;
  size_t bytes = 0;
  if (bf_bank_bytes(&d, &bytes) != BF_OK) return 2;
  d.L = 0;
  size_t ignored = 0;
  const bf_status st = bf_bank_bytes(&d, &ignored);
  printf("%zu %d %s\n", bytes, (int)st, bf_last_error());
  return st == BF_EINVAL ? 0 : 3;
}
"""


def test_header_is_plain_c_and_links(lib, tmp_path):
    """A C99 program includes bfly.h, links libbfly.so and calls host-side entry points."""
    import os
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "abi.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "abi"
    libdir = os.path.join(root, "paper_1802_01685_amd")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(root, "include"),
                        str(src), "-L", libdir, "-lbfly", f"-Wl,-rpath,{libdir}", "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0 and "-lbfly" in r.stderr:
        pytest.skip("libbfly.so is not built")
    assert r.returncode == 0, r.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True)
    assert run.returncode == 0, run.stdout + run.stderr
    bytes_, status = run.stdout.split()[:2]
    assert int(bytes_) == 65536 * 4096 * 4 + 256 and int(status) == lib.BF_EINVAL
