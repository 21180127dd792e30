"""The host MPO builders under AddressSanitizer and UndefinedBehaviorSanitizer.

mpo.cpp and subham.cpp (host only: no GPU code) are compiled with g++
-fsanitize=address,undefined together with tests/sanitize/host_driver.cpp,
which builds every recursion basis (exact and compressed), both stacked
sub-Hamiltonian MPOs and the affine transform for K = 2..6 and feeds the
argument checks malformed input; any sanitizer report fails the run.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1605_02611_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_mpo_builders_are_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_driver")
    cmd = ["g++", "-std=c++17", "-O0", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
           "-I" + os.path.join(ROOT, "include"), os.path.join(CSRC, "mpo.cpp"), os.path.join(CSRC, "subham.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "MPOs built" in r.stdout
