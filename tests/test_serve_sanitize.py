"""The serving loop's host bookkeeping (paper_2605_04017_amd/csrc/
lt_serve.cpp: admission by memory budget, chunking, round-robin launches over
the stream pool, reaping by event query, completion reports, argument
checks, teardown with requests in flight) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and driven by
tests/serve_sanitize.cpp over 400 seeded random request streams.  The device
is a fake HIP runtime and fake launches (tests/serve_sanitize.cpp), so this
runs on the CPU; the same loop on the GPU is tests/test_gpu_serve.py."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_serving_loop_under_sanitizers(tmp_path):
    exe = str(tmp_path / "serve_sanitize")
    csrc = os.path.join(ROOT, "paper_2605_04017_amd", "csrc")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{ROOT}/include", f"-I{csrc}",
           os.path.join(ROOT, "tests", "serve_sanitize.cpp"), os.path.join(csrc, "lt_serve.cpp"),
           os.path.join(csrc, "lt_api.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "scenarios" in r.stdout, r.stdout
    print(r.stdout.strip())
