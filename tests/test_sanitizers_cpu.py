"""AddressSanitizer and UndefinedBehaviorSanitizer on the host code (CPU only):

* the oracle, driven through every entry point on ragged boxes by
  oracle/sanitize_check.c (built with gcc, sanitizers on);
* the host side of the C ABI: libmts built with the host pass of api.hip
  sanitized (the device code and the other sources as usual), loaded through
  the Python binding with the sanitizer runtime preloaded, running the host
  ABI tests (argument checks, error paths, struct layout, exports).

Any sanitizer report aborts the child process, which fails the test.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2208_01525_amd", "csrc")
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# host pass only: the device code is built as usual
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
            "-fno-sanitize=vptr,function", "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host",
            "-fno-omit-frame-pointer"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_check")
    src = os.path.join(ROOT, "oracle", "sanitize_check.c")
    subprocess.run(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fcx-limited-range",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-Wall", "-Wextra", "-I" + os.path.join(ROOT, "oracle"), src, "-o", exe, "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env={**os.environ, **SAN_ENV,
                                                                   "ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitize_check: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


@pytest.mark.skipif(shutil.which("hipcc") is None or _asan_runtime() is None, reason="needs hipcc and clang's asan")
def test_host_abi_under_asan_ubsan(tmp_path):
    def compile_one(name):
        extra = HOST_SAN if name == "api.hip" else []
        obj = str(tmp_path / name.replace(".hip", ".o"))
        r = subprocess.run(["hipcc", *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, name), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    from paper_2208_01525_amd import build as B

    with cf.ThreadPoolExecutor(max_workers=min(len(B.SOURCES), 8)) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    lib = str(tmp_path / "libmts.so")
    # the sanitizer runtime comes from the preload; the link needs no sanitizer flag
    subprocess.run(["hipcc", "-shared", "--offload-arch=gfx950", *objs, "-o", lib], check=True)
    nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report" in nm and "__ubsan_handle" in nm
    env = {**os.environ, **SAN_ENV, "LD_PRELOAD": _asan_runtime(), "MTS_LIBRARY": lib}
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout and "failed" not in r.stdout
