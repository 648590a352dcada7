"""The plan's host code on its own (no GPU): a C++ check, compiled here
with g++ against plan.cpp, that the point lists own every sample once in
index order inside the right band, that spread lists hold each sample in
exactly the bands its stencil reaches, and that chunks tile the lists."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_point_lists_host_check(tmp_path):
    exe = str(tmp_path / "plan_lists_check")
    csrc = os.path.join(ROOT, "paper_1604_07651_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-pthread",
                    "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(csrc, "plan.cpp"),
                    os.path.join(ROOT, "tests", "host", "plan_lists_check.cpp"), "-o", exe],
                   check=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
