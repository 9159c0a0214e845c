"""Multiply-shift division by launch-time divisors (csrc/fastdiv.h), which the
FFT passes use for all their index arithmetic: checked against plain integer
division on the host over every divisor up to 4096, the low range of
numerators exhaustively, and random and edge numerators below 2^31."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1311_4120_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdint>
#include <random>
#include "fastdiv.h"
int main() {
  std::mt19937 rng(12345);
  const uint32_t edge[] = {0u, 1u, 2u, 0x3fffffffu, 0x40000000u, 0x7ffffffeu, 0x7fffffffu};
  for (uint32_t d = 1; d <= 4096; ++d) {
    jgb::FastDiv f(d);
    for (uint32_t n = 0; n < 20000; ++n)
      if (f.div(n) != n / d || f.mod(n) != n % d) { std::printf("FAIL %u %u\n", d, n); return 1; }
    for (uint32_t n : edge)
      if (f.div(n) != n / d) { std::printf("FAIL %u %u\n", d, n); return 1; }
    for (int i = 0; i < 2000; ++i) {
      uint32_t n = rng() & 0x7fffffffu;
      if (f.div(n) != n / d || f.mod(n) != n % d) { std::printf("FAIL %u %u\n", d, n); return 1; }
    }
  }
  const uint32_t big[] = {65536u, 262144u, 786432u, 1000003u, 134217728u, 0x7fffffffu};
  for (uint32_t d : big) {
    jgb::FastDiv f(d);
    for (int i = 0; i < 200000; ++i) {
      uint32_t n = rng() & 0x7fffffffu;
      if (f.div(n) != n / d) { std::printf("FAIL %u %u\n", d, n); return 1; }
    }
  }
  std::printf("ok\n");
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fastdiv_matches_integer_division(tmp_path):
    src = tmp_path / "fd.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "fd"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
