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
// Polynomials: sin r = r + r^3 (a0 + a1 r^2 + a2 r^4) and cos r = 1 + r^2 (b0 + b1 r^2 + b2 r^4),
// coefficients fitted toward the minimax absolute error on |r| <= pi/4 (sincos_fit.py beside
// this file: iteratively reweighted least squares on Chebyshev nodes) and rounded to FP32; fit
// errors 1.8e-9 (sin) and 3.2e-8 (cos). One term fewer each than the Taylor series through r^9
// and r^8 that they replace, at about the same final error. Horner's rule with fused
// multiply-adds. The quadrant k mod 4 selects the signs and the swap of sine and cosine.
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
  float ps = -0x1.98d88ap-13f;
  ps = fmaf(ps, r2, 0x1.1105aep-7f);
  ps = fmaf(ps, r2, -0x1.55554p-3f);
  const float sr = fmaf(ps * r2, r, r);
  float pc = -0x1.64737ep-10f;
  pc = fmaf(pc, r2, 0x1.553f8ap-5f);
  pc = fmaf(pc, r2, -0x1.ffffbap-2f);
  const float cr = fmaf(pc, r2, 1.0f);
  const int q = ((int)k) & 3;
  const float s = (q & 1) ? cr : sr;
  const float c = (q & 1) ? sr : cr;
  *sin_out = (q & 2) ? -s : s;
  *cos_out = ((q + 1) & 2) ? -c : c;
}

}  // namespace vmapi
