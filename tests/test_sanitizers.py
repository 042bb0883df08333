"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code
(CPU only, no GPU needed).

* The FP64 oracle (oracle/hh_oracle.c) is compiled with gcc under both
  sanitizers together with tests/san/oracle_check.c, which calls every
  exported routine on buffers of exactly the documented sizes.
* The library's host code (argument validation, workspace and record size
  arithmetic of the C ABI) is compiled with the sanitizers on the host side
  only and linked with tests/san/abi_check.c, which sweeps the size queries
  and a table of invalid calls; every call there is refused or only sizes a
  buffer, so no device work is attempted.

Both drivers exit non-zero on a sanitizer report (no recovery) or a wrong
status.  Build products go to _build/san/ and are reused while the sources
are unchanged.
"""
import glob
import hashlib
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "_build", "san")
CSRC = os.path.join(ROOT, "paper_1811_07624_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/lib/llvm/bin/clang"

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")


def _digest(paths):
    h = hashlib.sha256()
    for p in sorted(paths):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    return r.returncode, r.stdout


def test_oracle_under_asan_ubsan():
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    os.makedirs(SAN, exist_ok=True)
    exe = os.path.join(SAN, "oracle_check")
    src = [os.path.join(ROOT, "tests", "san", "oracle_check.c"),
           os.path.join(ROOT, "oracle", "hh_oracle.c")]
    rc, out = _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe, *src, "-lm"])
    assert rc == 0, out
    rc, out = _run([exe], env=ENV, timeout=300)
    assert rc == 0 and "0 failure(s)" in out, out


def _compile_host_sanitized(src):
    obj = os.path.join(SAN, os.path.basename(src) + ".o")
    # host side instrumented, device side built unoptimised (only to satisfy
    # the link: no kernel runs here)
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-g0", "-std=c++17",
           "-fPIC", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", obj]
    rc, out = _run(cmd)
    if rc != 0:
        raise RuntimeError(f"sanitized build of {src} failed:\n{out}")
    return obj


def test_host_abi_under_asan_ubsan():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not available")
    os.makedirs(SAN, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    deps = srcs + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(ROOT, "include", "hh.h")]
    stamp = os.path.join(SAN, "objs.stamp")
    key = _digest(deps)
    objs = [os.path.join(SAN, os.path.basename(s) + ".o") for s in srcs]
    if not (os.path.exists(stamp) and open(stamp).read() == key and all(map(os.path.exists, objs))):
        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
            objs = list(ex.map(_compile_host_sanitized, srcs))
        with open(stamp, "w") as f:
            f.write(key)
    drv = os.path.join(SAN, "abi_check.o")
    rc, out = _run([CLANG, "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                    "-I", os.path.join(ROOT, "include"),
                    "-c", os.path.join(ROOT, "tests", "san", "abi_check.c"), "-o", drv])
    assert rc == 0, out
    exe = os.path.join(SAN, "abi_check")
    rc, out = _run([HIPCC, "--offload-arch=gfx950",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-o", exe, drv, *objs])
    assert rc == 0, out
    rc, out = _run([exe], env=ENV, timeout=300)
    assert rc == 0 and "0 failure(s)" in out, out
