"""The CPU oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only, no GPU needed).

  oracle   tests/sanitize/oracle_driver.c runs every system, boundary rule,
           limiter and splitting on small ragged grids through the oracle
           built with gcc -fsanitize=address,undefined;
  runtime  tests/sanitize/runtime_driver.cpp runs the host paths of the
           library that finish before any device work (descriptor
           validation, workspace plans, size limits, the static entry
           point's size refusal, batch and learned-correction sizing, error
           strings) against the library's sources built with the sanitizers
           on the host side only (-Xarch_host), the device code unchanged.

A planted heap overflow, built with the same flags, must be reported, so the
sanitizer set-up itself is checked.
"""
import os
import shutil
import subprocess

import pytest

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1805_08846_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
GCC_SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)


def test_sanitizers_report_a_planted_overflow(tmp_path):
    src = tmp_path / "bad.c"
    src.write_text("#include <stdlib.h>\nint main(void){int*p=malloc(4*sizeof(int));int s=p[4];"
                   "free(p);return s;}\n")
    exe = tmp_path / "bad"
    r = _run(["gcc"] + GCC_SAN + ["-o", str(exe), str(src)])
    assert r.returncode == 0, r.stderr
    r = _run([str(exe)], env=ENV)
    assert r.returncode != 0 and ("AddressSanitizer" in r.stderr or "runtime error" in r.stderr)


def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_driver"
    r = _run(["gcc"] + GCC_SAN + ["-std=c99", "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas", "-o",
                                   str(exe), os.path.join(SAN, "oracle_driver.c"),
                                   os.path.join(ROOT, "oracle", "claw_oracle.c"), "-lm"])
    assert r.returncode == 0, r.stderr
    r = _run([str(exe)], env=ENV)
    print(r.stdout)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm toolchain")
def test_runtime_host_paths_under_asan_ubsan(tmp_path):
    srcs = ["sweeps", "fused", "batch", "control", "learned", "runtime", "stream"]
    procs = []
    for f in srcs:
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=on",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-omit-frame-pointer",
               "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, f + ".hip"),
               "-o", str(tmp_path / (f + ".o"))]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err[-4000:]
    drv = tmp_path / "drv.o"
    r = _run([CLANG, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
              "-I", os.path.join(ROOT, "include"), "-c", os.path.join(SAN, "runtime_driver.cpp"), "-o", str(drv)])
    assert r.returncode == 0, r.stderr
    exe = tmp_path / "runtime_driver"
    r = _run([CLANG, "-fsanitize=address,undefined", "-o", str(exe), str(drv)]
             + [str(tmp_path / (f + ".o")) for f in srcs]
             + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    assert r.returncode == 0, r.stderr[-4000:]
    r = _run([str(exe)], env=ENV)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)
