"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code
(no GPU needed): the 2D and 3D oracles (gcc) and the library's host side
(hipcc, sanitizers on the host pass only, kernel launchers stubbed), each run
by a driver in tests/sanitize/ through every entry point that needs no
device.  Any invalid access, leak or undefined operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2311_05091_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
GCC_SAN = "-fsanitize=address,undefined -fno-sanitize-recover=all -fno-omit-frame-pointer".split()
HOST_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-sanitize-recover=all -Xarch_host -fno-omit-frame-pointer").split()
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


@pytest.mark.parametrize("driver", ["oracle2_driver.c", "oracle3_driver.c"])
def test_oracle_under_sanitizers(tmp_path, driver):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "drv")
    subprocess.check_call(["gcc", "-std=gnu11", "-O1", "-g", *GCC_SAN, os.path.join(SAN, driver), "-o", exe, "-lm"])
    assert "sanitized run ok" in _run(exe)


def test_library_host_code_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
           "-I" + CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
           os.path.join(CSRC, "tpf_api.hip"), os.path.join(CSRC, "tpf3_api.hip"),
           os.path.join(SAN, "launch_stubs.cpp"), os.path.join(SAN, "host_driver.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=900)
    assert "host sanitized run ok" in _run(exe)
