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


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_point_lists_host_check_under_sanitizers(tmp_path):
    """The same check with the host plan built under AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only; any report aborts the run):
    no out-of-bounds access, overflow or other undefined behaviour while the
    plan places the samples, builds the band lists, chunks and spans."""
    exe = str(tmp_path / "plan_lists_check_asan")
    csrc = os.path.join(ROOT, "paper_1604_07651_amd", "csrc")
    try:
        subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-pthread",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer",
                        "-I", os.path.join(ROOT, "include"), "-I", csrc,
                        os.path.join(csrc, "plan.cpp"),
                        os.path.join(ROOT, "tests", "host", "plan_lists_check.cpp"), "-o", exe],
                       check=True, timeout=300, capture_output=True)
    except subprocess.CalledProcessError as e:
        if b"asan" in e.stderr.lower() or b"ubsan" in e.stderr.lower():
            pytest.skip("sanitizer runtime not available")
        raise
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr
