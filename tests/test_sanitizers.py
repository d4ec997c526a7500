"""CPU runs under AddressSanitizer and UndefinedBehaviorSanitizer.

- The oracle (plain C, gcc -fsanitize=address,undefined): every case kind for a few steps, its
  state and flux reads and its building blocks (tests/sanitize/oracle_cases.c).
- The host side of the library (hipcc, sanitizers on the host pass only; the device code is
  built as usual): workspace sizing and every argument check, which return before any device
  work, so no GPU is needed (tests/sanitize/host_checks.c).
Both programs are built into a temporary directory and must exit 0 with no sanitizer report.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_address_and_undefined_sanitizers():
    if not shutil.which("gcc"):
        pytest.skip("gcc missing")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_cases")
        _run(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-fno-omit-frame-pointer",
              "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
              "-I" + os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_cases.c"),
              os.path.join(ROOT, "oracle", "ugks_oracle.c"), "-o", exe, "-lm"], timeout=300)
        r = _run([exe], env=ENV, timeout=300)
        assert r.stdout.strip().endswith("ok")
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_library_host_code_under_address_and_undefined_sanitizers():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain missing")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")]
    csrc = os.path.join(ROOT, "paper_1810_08137_amd", "csrc")
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for src in ("ugks_kernels.hip", "ugks_capi.hip"):
            obj = os.path.join(d, src + ".o")
            _run([HIPCC, *flags, *san, "-c", os.path.join(csrc, src), "-o", obj], timeout=600)
            objs.append(obj)
        lib = os.path.join(d, "libugks_asan.so")
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *san, "-shared-libsan", *objs,
              "-o", lib], timeout=300)
        exe = os.path.join(d, "host_checks")
        rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                            capture_output=True, text=True).stdout.strip()
        rtdir = os.path.dirname(rt) if os.path.isabs(rt) else os.path.join(
            subprocess.run([CLANG, "-print-resource-dir"], capture_output=True,
                           text=True).stdout.strip(), "lib", "linux")
        _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-shared-libsan",
              "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"),
              os.path.join(HERE, "host_checks.c"), lib, "-Wl,-rpath," + d,
              "-Wl,-rpath," + rtdir, "-o", exe, "-lm"], timeout=300)
        r = _run([exe], env=ENV, timeout=300)
        assert r.stdout.strip().startswith("ok")
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
