"""CPU AddressSanitizer / UndefinedBehaviorSanitizer runs (no GPU).

1. The FP64 oracle (oracle/islbm_oracle.c) is built with
   -fsanitize=address,undefined and the oracle pins (tests/test_oracle_pins.py)
   and the network-reference pins run against that build in a child process
   with the sanitizer runtime preloaded.
2. The host side of the C-ABI (islbm_capi.cpp: argument and mesh validation,
   parameter derivation, interpolation tables, reduction coefficients) is
   built with the same flags, with host-only stand-ins for the device
   launchers (tests/sanitize/stub_launch.cpp), and driven through every
   host-side path by tests/sanitize/abi_host_driver.cpp.
Both must finish with no sanitizer report.  The GPU code is not instrumented
(GPU sanitizers are not available here)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _have(tool):
    return shutil.which(tool) is not None


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(not _have("gcc") or _runtime("libasan.so") is None, reason="gcc with ASan needed")
def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call(["gcc", "-std=gnu99", *SAN, "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", lib, os.path.join(ROOT, "oracle", "islbm_oracle.c"), "-lm"])
    env = dict(os.environ, **ENV_SAN, ISLBM_ORACLE_LIB=lib, LD_PRELOAD=_runtime("libasan.so"),
               OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow", "tests/test_oracle_pins.py",
                        "tests/test_mlp_oracle.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail


@pytest.mark.skipif(not _have("g++") or not os.path.exists("/opt/rocm/lib/libamdhip64.so"),
                    reason="g++ and the HIP runtime library needed")
def test_capi_host_paths_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "abi_host_asan")
    csrc = os.path.join(ROOT, "paper_2509_01099_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++20", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(csrc, "islbm_capi.cpp"),
                           os.path.join(ROOT, "tests", "sanitize", "stub_launch.cpp"),
                           os.path.join(ROOT, "tests", "sanitize", "abi_host_driver.cpp"),
                           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    env = dict(os.environ, **ENV_SAN)
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "0 failure(s)" in r.stdout, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
