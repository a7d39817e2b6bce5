"""Error budget of the compensated tracer on the CPU: a host build of the
arithmetic the trace kernels run (trace_one_ff, tests/trace_budget.cpp),
traced along the transmit path and every two-reflection ghost of the
benchmark lenses and the serving lenses, against the FP64 oracle at the GPU
parity tolerances.  Three builds: the host's correctly rounded reciprocal and
square root, and both moved one ulp up or down, which bounds the one-ulp
error of the hardware instructions the device code uses in their place.
The device kernels themselves are compared in tests/test_gpu_trace.py."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth
from parity import compare_trace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
FIELDS = ("mask", "x", "y", "dx", "dy", "dz", "throughput")


def _build(tmp, ulp):
    exe = os.path.join(tmp, f"trace_budget_{ulp}")
    cmd = ["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{ROOT}/include",
           f"-I{ROOT}/paper_2605_04017_amd/csrc", os.path.join(ROOT, "tests", "trace_budget.cpp"),
           os.path.join(ROOT, "paper_2605_04017_amd", "csrc", "lt_api.cpp"),
           f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", exe]
    if ulp:
        cmd.insert(3, f"-DLT_HOST_APPROX_ULP={ulp}")
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _write_lens(path, L):
    with open(path, "w") as f:
        f.write(f"{len(L.surfaces)} {len(L.glasses)}\n")
        for s in L.surfaces:
            f.write(f"{s.radius!r} {s.thickness!r} {s.semi_diameter!r} {s.glass_after} {s.is_stop}\n")
        for g in L.glasses:
            f.write(f"{g.kind} " + " ".join(repr(float(c)) for c in g.coef) + "\n")


@pytest.fixture(scope="module")
def exes(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    tmp = str(tmp_path_factory.mktemp("budget"))
    return tmp, {u: _build(tmp, u) for u in (0, 1, -1)}


CASES = [("C1 doublet", synth.config_lens, 1, 4000), ("C2/C3 double Gauss", synth.config_lens, 2, 4000)] + \
        [(f"serving lens {i}", None, i, 1500) for i in range(len(synth.SERVE_SURFACES))]


@pytest.mark.parametrize("name,make,arg,n", CASES, ids=[c[0] for c in CASES])
def test_compensated_tracer_budget(exes, name, make, arg, n):
    tmp, builds = exes
    L = make(arg) if make is not None else synth.serve_lenses()[arg]
    rays = synth.make_rays(L, n, 7100 + arg)
    lens_txt = os.path.join(tmp, "lens.txt")
    rays_bin = os.path.join(tmp, "rays.bin")
    _write_lens(lens_txt, L)
    np.stack([rays[k].astype(np.float32) for k in ("x", "y", "dx", "dy", "dz", "lambda_nm")]).tofile(rays_bin)
    nr = L.n_refracting
    paths = [(0, 0, 0)] + [(1, j, i) for j in range(1, nr + 1) for i in range(j + 1, nr + 1)]
    ora = [oracle.trace(L, rays, p, diag=True) for p in paths]
    worst = {}
    for ulp, exe in builds.items():
        out_bin = os.path.join(tmp, f"out_{ulp}.bin")
        subprocess.run([exe, lens_txt, rays_bin, out_bin], check=True, capture_output=True, text=True)
        out = np.fromfile(out_bin, np.float32).reshape(len(paths), 7, n)
        # the lens's ghost order: lt_ghost_path enumerates j outer, i inner
        for q, p in enumerate(paths):
            got = {k: out[q, f] for f, k in enumerate(FIELDS)}
            got["mask"] = got["mask"].astype(np.uint8)
            st = compare_trace(got, ora[q])
            for k in ("pos_max", "ang_max", "thr_max"):
                worst[k] = max(worst.get(k, 0.0), st.get(k, 0.0))
    print(f"[budget] {name}: {len(paths)} paths x {n} rays, worst over three builds {worst}", flush=True)
