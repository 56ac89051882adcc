"""The runtime's host code (validation, planning, footprint, the reserved-block
allocator) built with
AddressSanitizer and UndefinedBehaviorSanitizer and driven over edge cases and
seeded random requests (tests/host/sanitize_driver.cpp).  CPU only: the device
launch wrappers are stubs in the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not installed")
def test_runtime_host_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    # the runtime holds a device array (the scratch search's working memory),
    # so it is compiled as HIP for gfx950; the sanitizers instrument host code only
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"),
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-x", "c++", os.path.join(ROOT, "tests", "host", "sanitize_driver.cpp"),
           "-x", "hip", "--offload-arch=gfx950",
           os.path.join(ROOT, "paper_2209_09848_amd", "csrc", "tno_runtime.cpp"),
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "valid" in r.stdout and "offset pool checked" in r.stdout
