"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU).

The CPU oracle (plain C) and the library's host-only entry points (frame planning, ID prefix,
texture sizes, status strings) are built with `-fsanitize=address,undefined` and driven over small
scenes, edge cases and invalid arguments (tests/sanitize/*.c).  The sanitizers abort on any
out-of-bounds access, use after free, leak or undefined operation; the drivers exit non-zero on an
inconsistent result.  The library's kernels are not part of this build: the planning code is
compiled with sanitized host code only, and the kernel launchers it references are replaced by
stubs generated from their declarations (they are never called on these paths).
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ORACLE = os.path.join(ROOT, "oracle")
CSRC = os.path.join(ROOT, "paper_2604_21749_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


def test_oracle_under_address_and_undefined_sanitizers():
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    sources = [os.path.join(ORACLE, s) for s in ("raster.c", "brute.c", "resolve.c", "compress.c", "texture.c")]
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_driver")
        flags = ["-std=c11", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer", "-ffp-contract=off", "-mfma", "-msse4.1", "-pthread"]
        _run(["gcc"] + flags + ["-I", ORACLE, os.path.join(SAN, "oracle_driver.c")] + sources + ["-lm", "-o", exe])
        r = _run([exe], env=ENV, timeout=300)
    assert "oracle driver: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def _launcher_stubs(path):
    """Definitions, returning an error, for the kernel launchers runtime.hip declares."""
    src = open(os.path.join(CSRC, "runtime.hip")).read()
    start = src.index("namespace curast {\nhipError_t launch_")
    block = src[start:src.index("}  // namespace curast", start)]
    decls = re.findall(r"hipError_t\s+launch_\w+\([^;]*\);", block, flags=re.S)
    assert len(decls) >= 10, "launcher declarations not found in runtime.hip"
    body = ["#include <hip/hip_runtime.h>", '#include "curast.h"', '#include "common.h"', "namespace curast {"]
    body += [dcl[:-1] + " { return hipErrorInvalidValue; }" for dcl in decls]
    body.append("}  // namespace curast")
    open(path, "w").write("\n".join(body) + "\n")


def test_host_planning_under_address_and_undefined_sanitizers():
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not available")
    # host code only is sanitized (-Xarch_host before every sanitizer option)
    hip_flags = ["--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-fPIC",
                 "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-Wno-unused-value", "-Wno-unused-result", "-Wno-unused-parameter",
                 "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory() as d:
        stubs = os.path.join(d, "stubs.hip")
        _launcher_stubs(stubs)
        objs = []
        for src in (os.path.join(CSRC, "runtime.hip"), os.path.join(CSRC, "autotune.hip"), stubs):
            obj = os.path.join(d, os.path.basename(src) + ".o")
            _run([hipcc] + hip_flags + ["-c", src, "-o", obj])
            objs.append(obj)
        drv = os.path.join(d, "plan_driver.o")
        _run([clang, "-std=c11", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-I", os.path.join(ROOT, "include"), "-c", os.path.join(SAN, "plan_driver.c"), "-o", drv])
        exe = os.path.join(d, "plan_driver")
        _run([clang + "++", "-fsanitize=address,undefined", "-o", exe, drv] + objs +
             ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
        r = _run([exe], env=ENV, timeout=300)
    assert "plan driver: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
