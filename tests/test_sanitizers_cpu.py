"""Host-only sanitizer runs (AddressSanitizer + UndefinedBehaviorSanitizer):

* the oracle, built with g++ into a driver that calls every exported entry
  point on small cases (``tests/sanitize/oracle_driver.cpp``);
* the library's host code -- the host tables, the argument validation of the
  create calls, the error strings and the null-context guards -- built with
  hipcc, sanitizers on the host pass only, into a driver that never launches
  a kernel (``tests/sanitize/library_host_driver.cpp``).

Any sanitizer report aborts the driver with a non-zero status.  No GPU is used.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2506_03127_amd", "csrc")


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "ok" in r.stdout


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
                           os.path.join(SAN, "oracle_driver.cpp")])
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1"})


def test_library_host_paths_under_sanitizers(tmp_path):
    from paper_2506_03127_amd import _build
    try:
        hipcc = _build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "library_host_driver")
    srcs = [os.path.join(CSRC, s) for s in _build.SOURCES]
    cmd = [hipcc, f"--offload-arch={_build.ARCH}", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-o", exe, os.path.join(SAN, "library_host_driver.cpp")] + srcs
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    # the HIP runtime keeps its own allocations until exit: leak checking is off here
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1"})
