"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU.

Two programs are built with both sanitizers and run here, without a GPU:

* the library's host code (every source compiled host-only: no device code
  of the library is built) linked with `tests/sanitize/abi_driver.c`, which drives every
  entry point through its validation and error paths: null pointers, bad
  shapes and bends, workspaces too small or misaligned, option and pin
  ranges, batch jobs, plans, the tuning-rule list (its limit, replacement and
  read-back) and the timing brackets.  None of these calls reaches a kernel.
* the CPU oracle linked with `tests/sanitize/oracle_driver.c`, which runs
  every oracle function on small seeded images of both pixel types and on
  invalid arguments.

A test passes when its program exits 0 and neither sanitizer reported.
Sanitizers apply to host code only: the device side is never built with them.
"""

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1912_01884_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HERE = os.path.join(ROOT, "tests", "sanitize")
LIB_SOURCES = ["fhtp_api.cpp", "fhtp_timing.cpp", "fhtp_fht.hip", "fhtp_dp.hip",
               "fhtp_prep.hip", "fhtp_small.hip"]

ENV = dict(os.environ,
           ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        pytest.skip("hipcc not found")
    return path


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def _clean(r):
    text = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in text, text
    assert "runtime error:" not in text, text


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    # Host-only objects still register a device binary at start-up; each one
    # embeds that of an empty kernel (the library's kernels are never launched
    # here), which spares the minutes a full device build would take.
    empty = tmp_path / "empty.hip"
    empty.write_text("__global__ void fhtp_sanitize_empty() {}\n")
    fatbin = str(tmp_path / "empty.hipfb")
    _run([hipcc, "-x", "hip", "--cuda-device-only", "--offload-arch=gfx950", "-c", str(empty),
          "-o", fatbin])
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-Xclang", "-fcuda-include-gpubinary",
             "-Xclang", fatbin, "-Xarch_host", "-fsanitize=address,undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", f"-I{INCLUDE}", f"-I{CSRC}"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        _run([hipcc, "-x", "hip", "--cuda-host-only", "-c", os.path.join(CSRC, src), "-o", obj]
             + flags)
        return obj

    with ThreadPoolExecutor(max_workers=len(LIB_SOURCES)) as ex:
        objs = list(ex.map(compile_one, LIB_SOURCES))
    drv = str(tmp_path / "abi_driver.o")
    _run([hipcc, "-x", "c", "-std=c11", "-O1", "-g", "-Xarch_host", "-fsanitize=address,undefined",
          f"-I{INCLUDE}", "-c", os.path.join(HERE, "abi_driver.c"), "-o", drv])
    exe = str(tmp_path / "abi_driver")
    _run([hipcc, "-Xarch_host", "-fsanitize=address,undefined", "-o", exe, drv] + objs)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=120)
    _clean(r)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-omit-frame-pointer", "-o", exe, os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "fhtp_oracle.c"), "-lm"])
    r = subprocess.run([exe], capture_output=True, text=True,
                       env=dict(ENV, OMP_NUM_THREADS="2"), timeout=300)
    _clean(r)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
