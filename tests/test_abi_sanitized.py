"""The library's host-side argument validation under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

A copy of the library is built with the sanitizers on its host code only (device code
is untouched), and tests/abi_validation_driver.c calls every entry point with invalid
arguments, sizes and workspaces; each call must return its status code before any
device work, with no sanitizer report (any report aborts the driver)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm")
def test_validation_paths_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2412_11554_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    lib = tmp_path / "libaccord_san.so"
    build = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-disable-promote-alloca-to-lds", "-I", inc, "-I", csrc, "-o", str(lib),
             os.path.join(csrc, "accord_api.hip"), os.path.join(csrc, "accord_kernels.hip")]
    r = subprocess.run(build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = tmp_path / "driver"
    link = [CLANG, "-g", "-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer",
            "-I", inc, os.path.join(ROOT, "tests", "abi_validation_driver.c"),
            f"-L{tmp_path}", "-laccord_san", f"-Wl,-rpath,{tmp_path}", "-lm", "-o", str(exe)]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "validation OK" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)
