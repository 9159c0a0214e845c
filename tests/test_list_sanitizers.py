"""The host list construction (csrc/lists.h, which the plan calls) built for the
CPU with the address and undefined-behaviour sanitizers and run on node sets up
to N = 512 (1024 oversampled points per axis, where the 10-bit start codes are
tightest), every list entry checked against a brute-force enumeration of the
(node, tile) pairs whose footprints meet, and the threaded build against the
serial one (tests/sanitize/list_harness.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_list_construction_under_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.fail("g++ is needed to build the sanitizer harness")
    exe = str(tmp_path / "list_harness")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-pthread", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_1311_4120_amd", "csrc"),
           os.path.join(ROOT, "tests", "sanitize", "list_harness.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    # verify_asan_link_order=0: the runtime need not come first among the
    # libraries the environment loads
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip() == "ok"
