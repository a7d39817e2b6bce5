"""The host runtime's C++ (lens validation and storage, paraxial optics,
path ids, ghost indexing, trace-table construction: paper_2605_04017_amd/csrc/
lt_api.cpp) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and driven by tests/host_sanitize.cpp over seeded
random prescriptions, valid and malformed.  CPU only: these functions make
no device calls."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_runtime_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{ROOT}/include",
           f"-I{ROOT}/paper_2605_04017_amd/csrc",
           os.path.join(ROOT, "tests", "host_sanitize.cpp"),
           os.path.join(ROOT, "paper_2605_04017_amd", "csrc", "lt_api.cpp"),
           f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "lenses stored" in r.stdout, r.stdout
    print(r.stdout.strip())
