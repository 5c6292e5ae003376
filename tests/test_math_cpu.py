"""Accuracy of the kernel's own sine/cosine (paper_2302_01838_amd/csrc/vmap_math.h), compiled for
the host with g++ and compared with long-double sinl/cosl."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <cstdint>
#include "vmap_math.h"
int main() {
  double worst = 0.0, worst_x = 0.0;
  long n = 0;
  auto check = [&](float x) {
    float s, c;
    vmapi::vmap_sincosf(x, &s, &c);
    const long double xs = (long double)x;
    const double es = std::fabs((double)((long double)s - sinl(xs)));
    const double ec = std::fabs((double)((long double)c - cosl(xs)));
    const double e = es > ec ? es : ec;
    if (e > worst) { worst = e; worst_x = x; }
    ++n;
  };
  for (long i = -4000000; i <= 4000000; ++i) check((float)(i * (64.0 / 4000000.0)));
  uint32_t u = 12345u;
  for (long i = 0; i < 4000000; ++i) {  // xorshift32 points, |x| <= 64
    u ^= u << 13; u ^= u >> 17; u ^= u << 5;
    check((float)((u / 4294967296.0) * 128.0 - 64.0));
  }
  for (int q = -80; q <= 80; ++q) {  // multiples of pi/4 and their neighbours
    float x = (float)(q * 0.78539816339744830962);
    check(x); check(std::nextafter(x, 1e9f)); check(std::nextafter(x, -1e9f));
  }
  check(0.0f); check(-0.0f); check(1e-30f);
  std::printf("%.9e %.9e %ld\n", worst, worst_x, n);
  return 0;
}
"""


def test_sincos_accuracy(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2302_01838_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    worst, at, n = float(out[0]), float(out[1]), int(out[2])
    print(f"vmap_sincosf: max abs error {worst:.3e} at x = {at}, {n} points")
    assert n > 8_000_000
    assert worst < 2.5e-7
