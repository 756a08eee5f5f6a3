"""The library's host code (plan creation and validation, the integer tables, options,
the tuning report) under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

mpbp_host.cpp is compiled again with the sanitizers on its host compilation only (each
flag behind -Xarch_host; the device code is unchanged), linked with the regular kernel
objects into a separate library, and driven by tests/host_sanitize/host_driver.c, itself
built with the sanitizers, on host-only plans.  Any sanitizer report fails the run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
       "-g")


@pytest.mark.skipif(not os.path.exists(CLANG) or shutil.which("hipcc") is None and not os.path.exists(
    "/opt/rocm/bin/hipcc"), reason="needs the ROCm toolchain")
def test_host_code_under_sanitizers(tmp_path):
    from paper_2312_14907_amd import build as B
    if not all(os.path.exists(os.path.join(B.PKG, "_build", s + ".o")) for s in B.SOURCES):
        B.build()
    lib = B.build(out=str(tmp_path / "libmpbp_san.so"), objdir=str(tmp_path / "obj"), host_flags=SAN,
                  rebuild=("mpbp_host.cpp",))
    exe = tmp_path / "host_driver"
    r = subprocess.run([CLANG, *SAN, "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "host_sanitize", "host_driver.c"), "-o", str(exe), lib,
                        f"-Wl,-rpath,{tmp_path}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
