"""The library's reduced-argument FP64 exp and sincos (device helpers of the
influence factors, built here for the host from the same header): within a
few ulp of the C library over the argument range they serve, with the
quadrant signs right.  No GPU is used."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_reduced_exp_and_sincos_accuracy(tmp_path):
    from paper_2506_03127_amd import _build
    try:
        hipcc = _build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "math_accuracy")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-ffp-contract=off",
                           "-I", os.path.join(ROOT, "paper_2506_03127_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"), "-o", exe,
                           os.path.join(ROOT, "tests", "native", "math_accuracy.cpp")],
                          stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
