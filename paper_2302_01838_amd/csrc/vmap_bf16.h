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
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

namespace bf16_detail {
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 b2 __attribute__((ext_vector_type(2)));
typedef short s2 __attribute__((ext_vector_type(2)));
typedef unsigned short u2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
}  // namespace bf16_detail

// Two FP32 values rounded to BF16 (nearest even) as one packed word, lo in bits 0-15. A vector
// conversion, so that the pair becomes one v_cvt_pk_bf16_f32 (element-wise conversions were
// converted one by one and then merged with v_perm_b32).
VMAP_BF16_FN unsigned int pack2(float lo, float hi) {
  using namespace bf16_detail;
  const f2 p = {lo, hi};
  return __builtin_bit_cast(unsigned int, __builtin_convertvector(p, b2));
}

// Eight accumulator values rounded to BF16 (one MFMA operand's worth).
VMAP_BF16_FN bf16x8 round8(const f32x16& acc, int base) {
  using namespace bf16_detail;
  u4 w;
#pragma unroll
  for (int q = 0; q < 4; ++q) w[q] = pack2(acc[base + 2 * q], acc[base + 2 * q + 1]);
  return __builtin_bit_cast(bf16x8, w);
}

// 1 where a 16-bit lane of w is not zero, else 0 (packed unsigned minimum with 1). On the device
// one v_pk_min_u16: written as such because the compiler turns the expression into two compares,
// two selects and a byte permute.
VMAP_BF16_FN unsigned int nonzero16(unsigned int w) {
#if defined(__HIP_DEVICE_COMPILE__)
  unsigned int t;
  asm("v_pk_min_u16 %0, %1, %2" : "=v"(t) : "v"(w), "s"(0x00010001u));
  return t;
#else
  using namespace bf16_detail;
  const u2 m = __builtin_elementwise_min(__builtin_bit_cast(u2, w), (u2){1, 1});
  return __builtin_bit_cast(unsigned int, m);
#endif
}

// ReLU' applied to eight BF16 deltas: h holds the layer's outputs, which are non-negative BF16
// with +0 for every inactive unit, so a unit is active exactly where h's bits are not zero. Each
// delta's bits are multiplied by that 0/1 (a packed 16-bit integer product).
VMAP_BF16_FN bf16x8 relu_mask(bf16x8 d, bf16x8 h) {
  using namespace bf16_detail;
  u4 dw = __builtin_bit_cast(u4, d);
  const u4 hw = __builtin_bit_cast(u4, h);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned int hwi = hw[i];  // (a bit cast of the element expression itself misreads it)
    const u2 t = __builtin_bit_cast(u2, nonzero16(hwi));
    const u2 dv = __builtin_bit_cast(u2, (unsigned int)dw[i]);
    dw[i] = __builtin_bit_cast(unsigned int, (u2)(dv * t));
  }
  return __builtin_bit_cast(bf16x8, dw);
}

// ReLU of eight accumulator values, rounded to BF16: each pair is rounded, then a signed 16-bit
// max with 0 keeps non-negative BF16 values and turns negative ones (and -0) into +0.
VMAP_BF16_FN bf16x8 relu_round8(const f32x16& acc, int base) {
  using namespace bf16_detail;
  u4 w;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    s2 si = __builtin_bit_cast(s2, pack2(acc[base + 2 * q], acc[base + 2 * q + 1]));
    si = __builtin_elementwise_max(si, (s2){0, 0});
    w[q] = __builtin_bit_cast(unsigned int, si);
  }
  return __builtin_bit_cast(bf16x8, w);
}

}  // namespace vmapi
