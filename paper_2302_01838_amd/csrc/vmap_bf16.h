// BF16 packing helpers of the tile kernels, host- and device-compilable (clang) so that they can
// be checked on the CPU.
#pragma once

#if defined(__HIPCC__)
#define VMAP_BF16_FN __host__ __device__ inline
#else
#define VMAP_BF16_FN inline
#endif

namespace vmapi {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Eight accumulator values rounded to BF16 (one MFMA operand's worth).
VMAP_BF16_FN bf16x8 round8(const f32x16& acc, int base) {
  bf16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (__bf16)acc[base + e];
  return v;
}

// ReLU' applied to eight BF16 deltas: h holds the layer's outputs, which are non-negative BF16
// with +0 for every inactive unit, so a unit is active exactly where h's bits are not zero.
VMAP_BF16_FN bf16x8 relu_mask(bf16x8 d, bf16x8 h) {
  typedef unsigned short u2 __attribute__((ext_vector_type(2)));
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 dw = __builtin_bit_cast(u4, d);
  const u4 hw = __builtin_bit_cast(u4, h);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned int hwi = hw[i];  // (a bit cast of the element expression itself misreads it)
    const u2 hv = __builtin_bit_cast(u2, hwi);
    const u2 m = (u2){0, 0} - __builtin_elementwise_min(hv, (u2){1, 1});
    const unsigned int mw = __builtin_bit_cast(unsigned int, m);
    dw[i] = dw[i] & mw;
  }
  return __builtin_bit_cast(bf16x8, dw);
}

// ReLU of eight accumulator values, rounded to BF16: each pair is rounded, then a signed 16-bit
// max with 0 keeps non-negative BF16 values and turns negative ones (and -0) into +0.
VMAP_BF16_FN bf16x8 relu_round8(const f32x16& acc, int base) {
  typedef short s2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  bf16x8 v;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const b2 pr = {(__bf16)acc[base + 2 * q], (__bf16)acc[base + 2 * q + 1]};
    s2 si = __builtin_bit_cast(s2, pr);
    si = __builtin_elementwise_max(si, (s2){0, 0});
    const b2 rl = __builtin_bit_cast(b2, si);
    v[2 * q] = rl[0];
    v[2 * q + 1] = rl[1];
  }
  return v;
}

}  // namespace vmapi
