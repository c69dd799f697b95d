"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU (every report fatal, leaks checked):

* the CPU oracle, built with gcc and driven through each of its entry points
  by tests/oracle_sanitize_driver.c: dense and selective memory, both step
  schedules, the local-update period, learned candidate weights, the local
  search with and without 3-opt moves, colony exchange and the argument
  checks;
* the host side of libacs (the C ABI, the argument checks, the workspace
  layout and the no-device error path), built with hipcc with the
  sanitizers on the host compilation only and driven by
  tests/abi_sanitize_driver.c, linked with the same clang runtime.

A report from either sanitizer fails the test."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1605_02669_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    cmd = [gcc, "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wextra", "-Werror",
           os.path.join(HERE, "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "acs_oracle.c"), "-o", exe, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    _run(exe)


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/lib/llvm/bin/clang"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not found")
    lib = str(tmp_path / "libacs_san.so")
    srcs = [os.path.join(CSRC, f) for f in
            ("acs_kernels.hip", "acs_prior.hip", "acs_static.hip", "acs_api.cpp")]
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), *srcs, "-o", lib]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    rt = subprocess.run([clang, "-print-resource-dir"], capture_output=True,
                        text=True).stdout.strip()
    rtlib = os.path.join(rt, "lib", "linux")
    exe = str(tmp_path / "abi_driver")
    cmd = [clang, "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-Wextra",
           "-Werror", os.path.join(HERE, "abi_sanitize_driver.c"), "-o", exe,
           "-L", str(tmp_path), "-lacs_san", f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{rtlib}",
           "-lpthread", "-shared-libsan"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    _run(exe)
