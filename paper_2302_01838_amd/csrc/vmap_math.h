// Elementary functions of the step kernel that are written here rather than taken from a
// library, so that their cost and accuracy are known. Usable from host code (for tests) and
// device code.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define VMAP_HD __host__ __device__
#else
#define VMAP_HD
#endif

namespace vmapi {

// Sine and cosine of one FP32 argument with |x| < 6400 (|x| * 2/pi < 2^12).
//
// Range reduction (Cody and Waite, "Software Manual for the Elementary Functions", 1980):
// k = nearest integer to x * 2/pi, r = x - k * pi/2 with pi/2 = P1 + P2 + P3 split into FP32
// parts. P1 and P2 carry 12 significant bits each, so k * P1 and k * P2 are exact for
// |k| < 2^12; P3 is the FP32 rounding of the remainder (the split's own error is 5.7e-18).
// Then |r| <= pi/4 plus rounding.
//
// Polynomials: the Taylor series of sin through r^9 and of cos through r^8; on |r| <= pi/4 the
// first omitted terms are below 1.8e-9 (sin) and 2.5e-8 (cos), under half an FP32 ulp of 1.
// Horner's rule with fused multiply-adds. The quadrant k mod 4 selects the signs and the swap of
// sine and cosine.
//
// Error: below 2.5e-7 absolute for |x| <= 64 (tests/test_math_cpu.py).
VMAP_HD inline void vmap_sincosf(float x, float* sin_out, float* cos_out) {
  const float two_over_pi = 0.636619772367581343f;
  const float P1 = 0x1.922p+0f;
  const float P2 = -0x1.2aep-18f;
  const float P3 = -0x1.de973ep-31f;
  const float k = rintf(x * two_over_pi);
  float r = fmaf(-k, P1, x);
  r = fmaf(-k, P2, r);
  r = fmaf(-k, P3, r);
  const float r2 = r * r;
  // sin r = r (1 - r^2/3! + r^4/5! - r^6/7! + r^8/9!)
  float ps = 1.0f / 362880.0f;
  ps = fmaf(ps, r2, -1.0f / 5040.0f);
  ps = fmaf(ps, r2, 1.0f / 120.0f);
  ps = fmaf(ps, r2, -1.0f / 6.0f);
  const float sr = fmaf(ps * r2, r, r);
  // cos r = 1 - r^2/2! + r^4/4! - r^6/6! + r^8/8!
  float pc = 1.0f / 40320.0f;
  pc = fmaf(pc, r2, -1.0f / 720.0f);
  pc = fmaf(pc, r2, 1.0f / 24.0f);
  pc = fmaf(pc, r2, -0.5f);
  const float cr = fmaf(pc, r2, 1.0f);
  const int q = ((int)k) & 3;
  const float s = (q & 1) ? cr : sr;
  const float c = (q & 1) ? sr : cr;
  *sin_out = (q & 2) ? -s : s;
  *cos_out = ((q + 1) & 2) ? -c : c;
}

}  // namespace vmapi
