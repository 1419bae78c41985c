"""The direct-mapped store's tagged occupancy bytes and clear schedule, built
for the host from the library's header and run over 5000 steps of seeded
random occupancies: the planner's count is exactly the occupied slots at every
step, and a schedule that never clears fails the same check.  No GPU is used."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tagged_occupancy_counts_exactly_the_occupied_slots(tmp_path):
    from paper_2506_03127_amd import _build
    try:
        hipcc = _build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "occupancy_tags")
    subprocess.check_call([hipcc, "-O2", "-std=c++17",
                           "-I", os.path.join(ROOT, "paper_2506_03127_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"), "-o", exe,
                           os.path.join(ROOT, "tests", "native", "occupancy_tags.cpp")],
                          stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
