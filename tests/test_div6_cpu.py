"""The sweep's division by 6 (paper_2102_12416_amd/csrc/jc_div6.h) equals
the IEEE quotient s / 6 for every input, checked on the host.

The helpers are __host__ __device__; tests/div6_check.hip compiles them
host-only and compares them with the host's division over all 2^32
binary32 patterns (NaN and +-inf included) and over binary64 edge sets and
random patterns of every exponent.  The GPU parity tests then show the
device computes the same bits (test_division_edge_values_bitwise).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def _has_fma():
    try:
        return " fma " in open("/proc/cpuinfo").read().replace("\n", " ")
    except OSError:
        return False


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
@pytest.mark.skipif(not _has_fma(), reason="the check is built for a host with FMA instructions")
def test_div6_equals_ieee_division_everywhere(tmp_path):
    exe = str(tmp_path / "div6_check")
    cmd = [HIPCC, "--offload-host-only", "-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-I", os.path.join(ROOT, "paper_2102_12416_amd", "csrc"), "-o", exe,
           os.path.join(ROOT, "tests", "div6_check.hip")]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ)
    env.setdefault("OMP_NUM_THREADS", str(min(16, len(os.sched_getaffinity(0)))))
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr[-2000:]
    words = out.stdout.split()
    assert words[0] == "checked" and int(words[1]) == 1 << 32 and int(words[2]) > 10 ** 7, out.stdout
    assert words[-1] == "0", out.stdout
    shutil.rmtree(str(tmp_path), ignore_errors=True)
