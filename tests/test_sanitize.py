"""The serial oracle built with AddressSanitizer and UndefinedBehavior-
Sanitizer (gcc, host code only) and driven through every path by
tests/sanitize/oracle_driver.c: square lattices of several partitions, the
ring, the time-slice variant, the score, the bookkeeping check, the
generators and rejected descriptors.  Any memory error, leak or undefined
operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    exe = tmp_path / "oracle_driver"
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer"]
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off"] + flags + [
        "-I", os.path.join(ROOT, "oracle"),
        os.path.join(ROOT, "oracle", "kmco.c"),
        os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "oracle driver: ok" in p.stdout


def test_host_library_under_asan_and_ubsan(tmp_path):
    """libkmc's host code built with -fsanitize=address,undefined (host side
    only; the device code is built as usual) and driven through the paths
    that need no GPU by tests/sanitize/host_driver.py, in a process with the
    sanitizer runtime preloaded.  Skipped where a preload is already set."""
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("a preload is already set in this environment")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("no ROCm compiler")
    rt = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True, check=True).stdout.strip()
    if not os.path.exists(rt):
        pytest.skip("no sanitizer runtime")
    lib = tmp_path / "libkmc_san.so"
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1403_4674_amd", "csrc"),
           "-o", str(lib), os.path.join(ROOT, "paper_1403_4674_amd", "csrc", "kmc.hip")]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run(["python3", os.path.join(ROOT, "tests", "sanitize", "host_driver.py"),
                        str(lib)], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "host driver: ok" in p.stdout
