"""The library's host code under AddressSanitizer and UBSan.

Every source is compiled as for the product (gfx950 device code unchanged)
with the sanitizers on its host part only (each -fsanitize= after
-Xarch_host), linked into a separate library, and driven by a C program
(host_sanitize/host_check.c) through the C ABI: argument validation,
workspace and checkpoint sizes, the batch table writer and the zero-work
early returns, none of which touches a device.  The objects are rebuilt
only when a source is newer than the library.
"""

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1703_06116_amd", "csrc")
INC = os.path.join(ROOT, "include")
HERE = os.path.join(ROOT, "tests", "host_sanitize")
OUT = os.path.join(HERE, "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", INC, "-I", CSRC]


def _stale(target, deps):
    return not os.path.exists(target) or any(os.path.getmtime(d) > os.path.getmtime(target) for d in deps)


def _build():
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    deps = srcs + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(INC, "shgb.h")]
    lib = os.path.join(OUT, "libshgb_san.so")
    if _stale(lib, deps):
        def compile_one(src):
            obj = os.path.join(OUT, os.path.basename(src) + ".o")
            r = subprocess.run([HIPCC, *FLAGS, *SAN_HOST, "-c", src, "-o", obj], capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-4000:]
            return obj
        with ThreadPoolExecutor(min(8, os.cpu_count() or 4)) as ex:
            objs = list(ex.map(compile_one, srcs))
        r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
    exe = os.path.join(OUT, "host_check")
    src = os.path.join(HERE, "host_check.c")
    if _stale(exe, [src, lib]):
        r = subprocess.run([CLANG, "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                            "-I", INC, src, "-o", exe, "-L", OUT, "-lshgb_san", f"-Wl,-rpath,{OUT}",
                            "-Wl,-rpath,/opt/rocm/lib", "-lm"], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs the ROCm toolchain")
def test_host_code_is_clean_under_asan_and_ubsan():
    exe = _build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
