"""Host code of the library under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU (no device needed).

The library is rebuilt with host-side sanitizers (build_library(sanitize=True):
the device code is compiled as usual), a C++ driver (tests/sanitize/
host_checks.cpp) is linked against it with the sanitizer runtimes, and run:
workspace planning over extreme and invalid shapes (signed overflow in the
size arithmetic is undefined behaviour and stops the run), the host
generator of the test tensor, the pseudoinverse cut-off and the argument
checks of every entry point.  No call reaches the device."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.timeout(900)
@pytest.mark.skipif(not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")) or not os.path.exists(CLANG),
                    reason="needs hipcc and ROCm's clang++")
def test_host_code_under_asan_ubsan():
    from paper_2504_04989_amd.build import build_library
    lib = build_library(sanitize=True)
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "host_checks")
        cmd = [CLANG, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"), lib,
               f"-Wl,-rpath,{os.path.dirname(lib)}", "-Wl,-rpath,/opt/rocm/lib", "-L/opt/rocm/lib", "-lamdhip64",
               "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        out = r.stdout + r.stderr
        assert r.returncode == 0, out[-4000:]
        assert "host checks ok" in r.stdout
        assert "runtime error" not in out and "AddressSanitizer" not in out
