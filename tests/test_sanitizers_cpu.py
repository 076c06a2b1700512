"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer.

* The FP64 oracle (plain C) with gcc, driven through every entry point and
  its edge cases by oracle/sanitize_check.c.
* The library's host code (parameter validation, the E4M3 host encoder,
  null-context handling) with hipcc, sanitizers on the host pass only (the
  GPU code is compiled as usual), driven by tests/abi_sanitize_check.c,
  which needs no GPU.

Any sanitizer report fails the run (halt on the first error, no recovery).
"""

import os
import shutil
import subprocess

import pytest

from paper_2412_18271_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          os.path.join(ROOT, "oracle", "nnp_oracle.c"), os.path.join(ROOT, "oracle", "sanitize_check.c"),
          "-o", exe, "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "sanitize_check ok" in r.stdout
    assert "runtime error" not in r.stderr


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="hipcc / clang not found")
def test_library_host_code_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2412_18271_amd", "csrc")
    lib = str(tmp_path / "libnnp_san.so")
    san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", f]
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san +
         ["-I", os.path.join(ROOT, "include"), "-shared"] + [os.path.join(csrc, f) for f in build.SOURCES] +
         ["-o", lib], timeout=900)
    exe = str(tmp_path / "abi_check")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_sanitize_check.c"),
          "-o", exe, "-L", str(tmp_path), "-lnnp_san", "-Wl,-rpath," + str(tmp_path), "-lm"])
    # the HIP runtime's own allocations outlive main: leak checking off here
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    r = _run([exe], env=env, timeout=300)
    assert "abi_sanitize_check ok" in r.stdout
    assert "runtime error" not in r.stderr
