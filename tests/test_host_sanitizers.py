"""The host C++ of the library under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The DLR builder (`csrc/dlr_host.cpp`: composite Chebyshev sampling, pivoted QR, LU solves for the maps) is the
host code with the most index arithmetic; `tests/host/dlr_host_check.cpp` drives it over cutoffs from 1 to 4000 and
accuracies from 1e-6 to 1e-12.  It is built with g++ (host code only, no device compilation) with both sanitizers
and aborts on the first report; the test also checks that the maps carry single poles on the DLR frequencies (data
the basis represents exactly) to rounding, the ranks of the benchmark cutoffs, and that a rank cap below the
needed rank is an error.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_22223_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC), reason="needs g++ and HIP headers")
def test_dlr_host_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "dlr_host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC, "-I", CSRC,
           "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "dlr_host.cpp"),
           os.path.join(ROOT, "tests", "host", "dlr_host_check.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr[-4000:]
    cases = [l for l in run.stdout.splitlines() if l.startswith("case ")]
    assert len(cases) == 5, run.stdout
    ranks = {}
    for line in cases:
        vals = dict(re.findall(r"(\w+)=([-+0-9.e]+)", line))
        ranks[(float(vals["lambda"]), float(vals["eps"]))] = int(vals["rank"])
        # single poles on the DLR frequencies are represented exactly: the maps carry them to rounding
        assert float(vals["fermion_defect"]) < 1e-12, line
        assert float(vals["boson_defect"]) < 1e-12, line
        assert abs(float(vals["row_l1"]) - 1.0) < 1e-2, line
    # the ranks of the benchmark workloads (24 x 24 at beta = 50, 48 x 48 and 8^3 at beta = 100; omega_max = 25 eV)
    assert ranks[(1250.0, 1e-10)] == 53 and ranks[(2500.0, 1e-10)] == 59
    assert "capped rank=-" in run.stdout and "error=reported" in run.stdout
