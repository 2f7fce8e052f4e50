"""Sanitizer runs on the CPU (no GPU needed).

* The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
  (gcc; every report aborts) runs its whole pin suite, tests/test_oracle.py.
* The library's host-side code -- the C-ABI layer with argument validation,
  the uneven-batch layout, the Pauli-string plan and the tune-file parser --
  built with the same sanitizers (hipcc, host side only; the device objects
  of the normal build are linked unchanged) is driven by
  tests/host_planner_driver.py with seeded random and damaged inputs and
  fake device pointers: every call fails with its documented status before
  any device call, and the plans stay within their published bounds.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_2401_16378_amd", "_build")
CLANG_ASAN = "/opt/rocm/lib/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"


def sanitizer_env(runtime, **extra):
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.update(extra)
    return env


def clean(r):
    text = r.stdout + r.stderr
    return r.returncode == 0 and "AddressSanitizer" not in text and "runtime error" not in text


def test_oracle_pins_under_asan_ubsan(tmp_path):
    import oracle
    runtime = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(runtime) or not os.path.exists(runtime):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle.py", "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=sanitizer_env(runtime, PAULI_ORACLE_LIB=lib), capture_output=True, text=True,
                       timeout=900)
    assert clean(r), r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout


def test_host_code_under_asan_ubsan(tmp_path):
    sys.path.insert(0, os.path.join(ROOT, "paper_2401_16378_amd"))
    import build as b
    objs = [os.path.join(BUILD, s.split(".")[0] + ".o") for s in b.SOURCES if s != "api.cpp"]
    if not all(os.path.exists(o) for o in objs) or not os.path.exists(CLANG_ASAN):
        pytest.skip("needs the normal build's device objects and clang's AddressSanitizer runtime")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in b.FLAGS if f != "-O3"] + ["-O1", "-g"]
    api_o = str(tmp_path / "api_asan.o")
    lib = str(tmp_path / "libpauli_asan.so")
    subprocess.check_call(["hipcc", *flags, *san, "-x", "hip", "-c", os.path.join(b.CSRC, "api.cpp"), "-o", api_o],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    subprocess.check_call(["hipcc", "-shared", "-fPIC", "--offload-arch=" + b.ARCH, *san[:4], "-shared-libsan",
                           "-o", lib, api_o, *objs])
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host_planner_driver.py"), lib,
                        str(tmp_path / "tune.txt")], cwd=ROOT, env=sanitizer_env(CLANG_ASAN), capture_output=True,
                       text=True, timeout=600)
    assert clean(r), r.stdout[-3000:] + r.stderr[-3000:]
    assert "host planner driver: ok" in r.stdout
