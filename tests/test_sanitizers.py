"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code
(CPU only): the FP64 oracle stepped through every boundary set, reading of
Eqs. 26-27 and collision operator in 2D and 3D (tests/sanitize/oracle_driver.c),
and the library's validation, layout and workspace code behind the C ABI
(tests/sanitize/api_driver.cpp, the kernel launchers stubbed out).  Each
driver must exit 0 with no sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(exe, leaks):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={int(leaks)}", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    print(out)
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", *SAN, os.path.join(ROOT, "oracle", "lbm_oracle.c"),
                    os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe], check=True)
    _run(exe, leaks=True)


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not available")
def test_host_runtime_validation_under_sanitizers(tmp_path):
    exe = str(tmp_path / "api_san")
    subprocess.run([CLANG, "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *SAN,
                    os.path.join(ROOT, "paper_2111_08666_amd", "csrc", "lbm_api.cpp"),
                    os.path.join(ROOT, "tests", "sanitize", "api_driver.cpp"),
                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe], check=True)
    # the HIP runtime's own start-up allocations are not this code's leaks
    _run(exe, leaks=False)
