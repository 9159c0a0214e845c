"""The host list construction (csrc/lists.h) and radial rule (csrc/radial.h),
which the plan calls, built for the CPU with the address and
undefined-behaviour sanitizers (tests/sanitize/list_harness.cpp):

  * the lists on node sets up to N = 512 (1024 oversampled points per axis,
    where the 10-bit start codes are tightest), every entry checked against a
    brute-force enumeration of the (node, tile) pairs whose footprints meet,
    and the threaded build against the serial one;
  * the per-line ranges of the spreading grid that footprints reach, and of
    the spectrum that the interpolation by tiles reads (every point of every
    listed tile, or its mirror image, inside its line's range; both ends of a
    range points that are read; unread lines empty);
  * the generalized Gaussian radial rule against the oracle's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("sanitize"))


def _build(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.fail("g++ is needed to build the sanitizer harness")
    exe = str(tmp_path / "list_harness")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-pthread", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_1311_4120_amd", "csrc"),
           os.path.join(ROOT, "tests", "sanitize", "list_harness.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def _env():
    # verify_asan_link_order=0: the runtime need not come first among the
    # libraries the environment loads
    return dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
                UBSAN_OPTIONS="print_stacktrace=1")


def test_list_construction_under_sanitizers(harness):
    exe = harness
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=_env())
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip() == "ok"


@pytest.mark.parametrize("c,n", [(30.7247761521, 44), (3.5, 24), (116.6, 96)])
def test_host_radial_rule_matches_the_oracle(harness, c, n):
    """The plan's generalized Gaussian radial rule (Sturm bisection and inverse
    iteration for the prolate functions, bisection for their roots) against the
    oracle's (scipy's tridiagonal eigensolver and root finder)."""
    from oracle.ggq import prolate_rule
    exe = harness
    r = subprocess.run([exe, "radial", repr(c), str(n)], capture_output=True, text=True, timeout=300, env=_env())
    assert r.returncode == 0, r.stderr[-2000:]
    got = np.array([[float(v) for v in line.split()] for line in r.stdout.strip().splitlines()])
    x, w = prolate_rule(c, n)
    assert got.shape == (n, 2)
    assert np.max(np.abs(got[:, 0] - x)) < 1e-13 and np.max(np.abs(got[:, 1] - w)) < 1e-13
