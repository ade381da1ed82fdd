"""The oracle and the library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer, run on this CPU host (no GPU needed).  The
library's sources are compiled as usual for gfx950, each sanitizer flag
passed to the host compilation alone (the device code is not sanitized and
never runs here)."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2502_04189_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off"] + SAN +
         ["-I" + os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"])
    r = _run([exe], env=ENV, timeout=600)
    assert "0 failures" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_library_host_code_under_sanitizers(tmp_path):
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        _run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-Xarch_host", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host_san +
             ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    srcs = ("pcx_kernels.hip", "pcx_host.cpp", "pcx_batch.cpp", "pcx_tune.cpp", "pcx_noalloc.cpp")
    with ThreadPoolExecutor(max_workers=5) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "host_driver.o")
    _run([CLANG, "-O1", "-g", "-std=c++17"] + SAN + ["-I" + os.path.join(ROOT, "include"), "-c",
                                                      os.path.join(HERE, "host_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "host_san")
    _run([CLANG] + SAN + [drv] + objs + ["-o", exe, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64"])
    r = _run([exe], env=ENV, timeout=600)
    assert "0 failures" in r.stdout
