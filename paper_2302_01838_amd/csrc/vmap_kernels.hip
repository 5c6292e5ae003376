// HIP kernels for gfx950 (CDNA4) of the vectorised per-object training step.
//
// Work decomposition. A batch holds the rays of many objects, segmented by CSR offsets. Each
// object's rays are cut into tiles of `rays_per_tile` consecutive rays; a tile never straddles
// two objects and its boundaries are relative to the object's first ray, so an object's result
// does not depend on the other objects in the batch. One workgroup processes one tile at a time
// (grid-stride, so the launch may be persistent). Inside a tile, each 64-lane wave takes
// sub-tiles of floor(64 / S) whole rays: the S samples of a ray occupy S consecutive lanes.
//
// Per sub-tile a wave runs, without leaving registers except for two small LDS transposes:
//   1. point normalisation in FP64, rounded once to FP32, and Gaussian Fourier features
//      (object-level encoding, supplement Sec. B);
//   2. the MLP on MFMA, 32 samples per pass, features on the M axis and samples on the N axis,
//      so each layer's accumulator layout is directly the next layer's B operand (the K axis
//      is permuted consistently in the weights instead of moving data);
//   3. occupancy rendering of Eq. 3 with ray-segmented wavefront scans: an exclusive
//      multiplicative scan of (1 - o) and additive scans for the rendered sums;
//   4. the masked L1 losses of Eqs. 4-7;
//   5. the adjoint of rendering: with g_i the derivative of the loss with respect to the
//      termination probability T_i, dL/do_i = P_i g_i - R_i / (1 - o_i) where R_i = sum over the
//      ray's later samples of g_j T_j (a reverse scan); the logit's adjoint
//      o_i ((1 - o_i) g_i P_i - R_i) needs no division;
//   6. the MLP backward: dX products on MFMA from the accumulator layout, dW products on MFMA
//      after an LDS transpose, accumulated in registers across the wave's sub-tiles.
// The waves of a workgroup then add their gradients in a fixed order and write one partial
// per tile; a second kernel sums each object's tile partials in tile order (no float atomics,
// bitwise reproducible), and a third applies Adam per object.
//
// Precision. Both modes use the sine/cosine of vmap_math.h (error below 2.5e-7; the hardware
// v_sin/v_cos approximations were tried for BF16 and moved enough features across BF16 rounding
// boundaries to show in the gradients) and the hardware exp2 and reciprocal for the logistic.
// FP32 mode uses v_mfma_f32_32x32x2f32. BF16 mode rounds weights, activations and
// back-propagated deltas to BF16 (round to nearest even) where they enter a product and uses
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation; encoding, head activations, rendering,
// losses, reductions and Adam stay FP32.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "vmap_internal.h"
#include "vmap_math.h"
#include "vmap_bf16.h"

namespace vmapi {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Accumulator row held in register r (0..15) by lanes of half h (0, 1) of a 32x32 MFMA tile.
// The same map orders the K axis: K slot (h, r) of a block carries feature rowof(r, h).
__host__ __device__ constexpr int rowof(int r, int h) { return ((r >> 2) << 3) + (h << 2) + (r & 3); }
// Position of feature c (0..31) of a block in the permuted weight-column order.
__host__ __device__ constexpr int colpos(int c) { return (((c >> 2) & 1) << 4) + ((c >> 3) << 2) + (c & 3); }

__device__ __forceinline__ void wave_lds_sync() {
  // Orders this wave's LDS accesses across lanes: the compiler may not move LDS loads or stores
  // across it, and the wave waits until its own LDS operations have completed.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  asm volatile("" ::: "memory");
}

// BF16 operand tiles of the weight-gradient products are staged sample-major: row s (a sample)
// holds the tile's features, TR_STRIDE elements apart. A lane writes its accumulator-layout
// values as 8-byte runs of four consecutive features, and ds_read_b64_tr_b16 regroups them: in
// each group of 16 lanes, lane 4a + b receives element b of the 8-byte chunks addressed by lanes
// a, a + 4, a + 8 and a + 12 of its group (checked on the device), so four lanes that address
// four consecutive rows at the same feature offset hand each of their readers one feature's four
// consecutive samples.
constexpr int kTrStride = 36;  // BF16 elements per staged row (32 features + 4: 8-byte rows)

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef short v8i16 __attribute__((ext_vector_type(8)));

// Eight BF16 (two transposing reads, the second four rows further down) as one MFMA operand.
__device__ __forceinline__ bf16x8 tr_read8(const __bf16* p) {
  typedef __attribute__((address_space(3))) v4i16 lds_v4;
  const v4i16 a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4*)(p));
  const v4i16 b = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4*)(p + 4 * kTrStride));
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7));
}

// Elements 0-3 of v to p and elements 4-7 to p + 8 (two 8-byte stores).
__device__ __forceinline__ void write_runs(__bf16* p, bf16x8 v) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  typedef unsigned int u2w __attribute__((ext_vector_type(2)));
  const u4 w = __builtin_bit_cast(u4, v);
  *reinterpret_cast<u2w*>(p) = (u2w){w[0], w[1]};
  *reinterpret_cast<u2w*>(p + 8) = (u2w){w[2], w[3]};
}

// First tile of a workgroup. Workgroups are dealt to the eight XCDs in turn (workgroup b runs on
// XCD b mod 8, each with its own L2); when the grid has a workgroup per tile, the first n_tiles
// workgroups of one XCD take consecutive tiles, so that an object's tiles (its weights, rays and
// samples) share one L2 instead of being fetched into all eight. Workgroups past n_tiles (the
// last dispatched) stay without a tile. Otherwise tile = workgroup index. Only for launches whose
// tiles all do work: each XCD gets an equal share of tiles, not of work.
__device__ __forceinline__ int first_tile_of_block(int n_tiles) {
  constexpr int kXcds = 8;
  const int b = blockIdx.x;
  if ((int)gridDim.x < n_tiles || b >= n_tiles) return b;
  const int x = b % kXcds;
  int start = 0;
  for (int y = 0; y < x; ++y) start += (n_tiles - y + kXcds - 1) / kXcds;  // workgroups of XCD y
  return start + b / kXcds;
}

// Unit and block of this workgroup in a one-dimensional grid of 8 ceil(units / 8) nblk
// workgroups (workgroups are dealt to the eight XCDs in turn by index): unit u goes to XCD u mod 8,
// and each XCD takes its units' nblk blocks one unit after another, so that the blocks of a unit
// (which share its rows and its object's weights) share one L2, and the units that exist (the
// first ones of a bound with slack) are spread evenly over the XCDs.
__device__ __forceinline__ void xcd_unit_block(int nblk, int& unit, int& blk) {
  const int b = (int)blockIdx.x, x = b & 7, s = b >> 3;
  unit = x + 8 * (s / nblk);
  blk = s % nblk;
}

// Logistic sigmoid from the hardware exponential and reciprocal (about 1 ulp each; an IEEE
// division costs a dozen instructions). exp(-z) overflows to +inf for z < -88, giving 0.
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// sigma(z) and sigma(-z) = 1 - sigma(z) from one exponential e = exp(-z) (as 2^(-z log2 e), the
// hardware v_exp_f32): sigma(z) = 1 / (1 + e); sigma(-z) = e sigma(z) for z > 0 (e < 1) and
// 1 - sigma(z) for z <= 0 (sigma(z) <= 1/2, so no cancellation). e = inf for very negative z
// gives sigma(z) = 0 and sigma(-z) = 1.
__device__ __forceinline__ void sigm_pair(float z, float& sp, float& sn) {
  const float e = __builtin_amdgcn_exp2f(-z * 1.44269504088896341f);
  sp = __builtin_amdgcn_rcpf(1.0f + e);
  sn = (z > 0.f) ? e * sp : 1.0f - sp;
}

template <bool BF>
__device__ __forceinline__ float round_w(float x) {
  if constexpr (BF) return (float)(__bf16)x;
  return x;
}

// Reads of a wide object's weight image in device memory through a buffer resource: the lane
// part of an offset sits in one VGPR and the block's constant part in an SGPR or the immediate,
// so unrolled loops need no 64-bit address per load.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const unsigned char* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ bf16x8 img_b128(__amdgpu_buffer_rsrc_t r, int lane_off, int off) {
  return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, off, 0));
}
__device__ __forceinline__ f32x4 img_f4(__amdgpu_buffer_rsrc_t r, int lane_off, int off) {
  return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, off, 0));
}
__device__ __forceinline__ float img_f1(__amdgpu_buffer_rsrc_t r, int lane_off, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, off, 0));
}

// Activations of one 32-sample pass: NL + 1 layers (encoding first), H/32 blocks, D layout.
template <int H, bool BF>
struct Acts;
template <int H>
struct Acts<H, false> {
  float v[kLayers + 1][H / 32][16];
  __device__ __forceinline__ float get(int l, int b, int r) const { return v[l][b][r]; }
  __device__ __forceinline__ void set(int l, int b, int r, float x) { v[l][b][r] = x; }
  // registers r and r + 1 (r even)
  __device__ __forceinline__ void set2(int l, int b, int r, float x, float y) {
    v[l][b][r] = x;
    v[l][b][r + 1] = y;
  }
};
template <int H>
struct Acts<H, true> {
  bf16x8 v[kLayers + 1][H / 32][2];
  __device__ __forceinline__ float get(int l, int b, int r) const { return (float)v[l][b][r >> 3][r & 7]; }
  __device__ __forceinline__ void set(int l, int b, int r, float x) { v[l][b][r >> 3][r & 7] = (__bf16)x; }
  // registers r and r + 1 (r even), rounded as one packed pair
  __device__ __forceinline__ void set2(int l, int b, int r, float x, float y) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    u4 w = __builtin_bit_cast(u4, v[l][b][r >> 3]);
    w[(r & 7) >> 1] = pack2(x, y);
    v[l][b][r >> 3] = __builtin_bit_cast(bf16x8, w);
  }
};

// Back-propagated deltas of one 32-sample pass in the accumulator layout. In BF16 mode they only
// ever enter products and LDS staging rounded to BF16, so they are kept rounded.
template <int H, bool BF>
struct Deltas;
template <int H>
struct Deltas<H, false> {
  float v[H / 32][16];
  __device__ __forceinline__ void set(int b, int r, float x) { v[b][r] = x; }
};
template <int H>
struct Deltas<H, true> {
  bf16x8 v[H / 32][2];
  __device__ __forceinline__ void set(int b, int r, float x) { v[b][r >> 3][r & 7] = (__bf16)x; }
};

// ---------------------------------------------------------------------------------------------
// Weight staging: object k's parameters -> LDS (permuted columns; BF16 in BF16 mode, plus the
// transposed copies that the backward's input-gradient products read as A operands). Threads
// tid, tid + nt, ... of the caller share the work; the destination may also be a weight image in
// device memory (wide models).

// Where stage_weights puts parameter p (value w) of a width-H object: the same bytes, one
// parameter at a time (BF16: with its transposed copy, or its bias's three pieces). The
// optimiser kernels keep the weight images current with it after each update.
template <int H, bool BF>
__device__ __forceinline__ void place_param(unsigned char* img, int p, float w) {
  constexpr LdsLayout L = lds_layout(H, BF, 1);
  using WT = typename std::conditional<BF, __bf16, float>::type;
  int off = 0;
#pragma unroll
  for (int l = 0; l < kLayers; ++l) {
    const int K = (l == 0) ? kEnc : H;
    if (p < off + H * K) {
      const int e = p - off, row = e / K, col = e - row * K;
      reinterpret_cast<WT*>(img + L.w_off[l])[row * L.w_stride[l] + (col & ~31) + colpos(col & 31)] = (WT)w;
      if constexpr (BF) {
        if (l > 0)
          reinterpret_cast<__bf16*>(img + L.wt_off[l])[col * (H + 8) + (row & ~31) + colpos(row & 31)] = (__bf16)w;
      }
      return;
    }
    off += H * K;
    if (p < off + H) {
      const int row = p - off;
      reinterpret_cast<float*>(img + L.b_off)[l * H + row] = w;
      if constexpr (BF) {
        const __bf16 hi = (__bf16)w;
        const __bf16 mid = (__bf16)(w - (float)hi);
        const __bf16 lo = (__bf16)((w - (float)hi) - (float)mid);
        __bf16* dst = reinterpret_cast<__bf16*>(img + L.bA_off) + (size_t)(l * H + row) * 16;
        dst[0] = hi;
        dst[1] = mid;
        dst[2] = lo;
      }
      return;
    }
    off += H;
  }
  if (p < off + kOut * H) {
    const int e = p - off, c = e / H, col = e - c * H;
    if constexpr (BF) {
      reinterpret_cast<__bf16*>(img + L.whb_off)[c * (H + 8) + (col & ~31) + colpos(col & 31)] = (__bf16)w;
      reinterpret_cast<__bf16*>(img + L.whtb_off)[col * kOut + c] = (__bf16)w;
    } else {
      reinterpret_cast<float*>(img + L.wh_off)[c * (H + 4) + (col & ~31) + colpos(col & 31)] = w;
    }
    return;
  }
  off += kOut * H;
  reinterpret_cast<float*>(img + L.bh_off)[p - off] = w;
}

// A weight image fetched into LDS without registers: each wave's 64 lanes move 1 KiB blocks
// (global_load_lds_dwordx4: lane l's 16 bytes land at the wave-uniform LDS address + 16 l); the
// part past the last whole block goes through registers. The LDS writes complete under vmcnt, so
// readers wait for it (s_waitcnt) and a barrier.
__device__ __forceinline__ void fetch_image_lds(const unsigned char* src, unsigned char* dst, int bytes,
                                                int lane, int wave, int nw) {
  const int blocks = bytes >> 10;
  for (int b = wave; b < blocks; b += nw)
    __builtin_amdgcn_global_load_lds(src + (b << 10) + 16 * lane,
                                     (__attribute__((address_space(3))) void*)(dst + (b << 10)), 16, 0, 0);
  const int tail = (bytes - (blocks << 10)) >> 4;  // 16-byte pieces left
  if (wave == nw - 1 && lane < tail) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    *reinterpret_cast<u32x4*>(dst + (blocks << 10) + 16 * lane) =
        *reinterpret_cast<const u32x4*>(src + (blocks << 10) + 16 * lane);
  }
}

// src_hidden: the object's own width; an object of hidden 16 staged at H = 32 reads each slot of
// the width-32 layout from its own parameters (padded_index), zero for the padding.
template <int H, bool BF>
__device__ __forceinline__ void stage_weights(const float* __restrict__ th, unsigned char* smem, int tid, int nt,
                                              int src_hidden = H) {
  constexpr LdsLayout L = lds_layout(H, BF, 1);
  using WT = typename std::conditional<BF, __bf16, float>::type;
  const bool padded = (H == 32 && src_hidden == 16);
  auto param = [&](int q) -> float {
    if (padded) {
      const int p = unpadded_index16(q);
      return p >= 0 ? th[p] : 0.f;
    }
    return th[q];
  };
  int off = 0;
  float* bias = reinterpret_cast<float*>(smem + L.b_off);
#pragma unroll
  for (int l = 0; l < kLayers; ++l) {
    const int K = (l == 0) ? kEnc : H;
    WT* W = reinterpret_cast<WT*>(smem + L.w_off[l]);
    const int ws = L.w_stride[l];
    for (int e = tid; e < H * K; e += nt) {
      const int row = e / K, col = e - row * K;
      const WT w = (WT)param(off + e);
      W[row * ws + (col & ~31) + colpos(col & 31)] = w;
      if constexpr (BF) {
        if (l > 0) {  // W^T[col][row], rows of the transpose permuted like the forward's K axis
          __bf16* Wt = reinterpret_cast<__bf16*>(smem + L.wt_off[l]);
          Wt[col * (H + 8) + (row & ~31) + colpos(row & 31)] = w;
        }
      }
    }
    off += H * K;
    for (int e = tid; e < H; e += nt) bias[l * H + e] = param(off + e);
    off += H;
  }
  for (int e = tid; e < kOut * H; e += nt) {
    const int c = e / H, col = e - c * H;
    if constexpr (BF) {
      const __bf16 w = (__bf16)param(off + e);
      reinterpret_cast<__bf16*>(smem + L.whb_off)[c * (H + 8) + (col & ~31) + colpos(col & 31)] = w;
      reinterpret_cast<__bf16*>(smem + L.whtb_off)[col * kOut + c] = w;
    } else {
      reinterpret_cast<float*>(smem + L.wh_off)[c * (H + 4) + (col & ~31) + colpos(col & 31)] = param(off + e);
    }
  }
  off += kOut * H;
  float* bh = reinterpret_cast<float*>(smem + L.bh_off);
  for (int e = tid; e < kOut; e += nt) bh[e] = param(off + e);
  if constexpr (BF) {
    // bias as an MFMA operand: b = hi + mid + lo exactly (three BF16 pieces of 8 bits each)
    __bf16* bA = reinterpret_cast<__bf16*>(smem + L.bA_off);
    int boff[kLayers];
    int o2 = 0;
#pragma unroll
    for (int l = 0; l < kLayers; ++l) {
      const int K = (l == 0) ? kEnc : H;
      boff[l] = o2 + H * K;
      o2 += H * K + H;
    }
    for (int e = tid; e < kLayers * H; e += nt) {
      const int l = e / H, row = e - l * H;
      const float b = param(boff[l] + row);
      const __bf16 hi = (__bf16)b;
      const __bf16 mid = (__bf16)(b - (float)hi);
      const __bf16 lo = (__bf16)((b - (float)hi) - (float)mid);
      __bf16* dst = bA + (size_t)e * 16;
      dst[0] = hi;
      dst[1] = mid;
      dst[2] = lo;
      for (int q = 3; q < 16; ++q) dst[q] = (__bf16)0.0f;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Forward of one 32-sample pass for the calling wave. xt: this lane's normalised point (the
// sample of column n = lane & 31; both lane halves hold the same point); Bm: the encoding matrix.
// ENC = false: the encoding is already in A.v[0] (kept from an earlier pass; xt unused).
// ipe: xt[3] holds the sample's variance in the object frame; each feature is its expectation
// under the isotropic Gaussian (integrated positional encoding). Fills the activations
// and, with WITH_HEAD, returns the four output pre-activations z of sample n (valid in both lane
// halves).

template <int H, bool BF, bool WITH_HEAD, bool ENC = true>
__device__ __forceinline__ void forward_pass(const float xt[4], const unsigned char* smem,
                                             const float* Bm, Acts<H, BF>& A, float z[4],
                                             bool ipe = false) {
  constexpr int MT = H / 32;
  constexpr LdsLayout L = lds_layout(H, BF, 1);
  // Weights are re-read on every pass instead of being held in registers across passes. `smem`
  // is the weight base: the LDS staging, or a wide object's image in device memory.
  asm volatile("" ::: "memory");
  const int lane = threadIdx.x & 63, n = lane & 31, hf = lane >> 5;
  // Gaussian Fourier features: register r of block 0 holds feature rowof(r, hf):
  // r = 0..3 sin(phi[4hf + r]), 4..7 sin(phi[8 + 4hf + r - 4]), 8..15 the cosines.
  // Without ENC the caller has already placed them in A.v[0].
#pragma unroll
  for (int g = 0; g < (ENC ? 2 : 0); ++g) {
#pragma unroll
    for (int i = 0; i < 4; i += 2) {  // two features at a time: one packed pair per half
      float s[2], c[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int f = 8 * g + 4 * hf + i + u;
        const float phi = xt[0] * Bm[f] + xt[1] * Bm[kFeatures + f] + xt[2] * Bm[2 * kFeatures + f];
        vmap_sincosf(phi, &s[u], &c[u]);
        if (ipe) {  // expectation under N(x, v I): attenuation exp(-v |b_f|^2 / 2)
          const float nb = Bm[f] * Bm[f] + Bm[kFeatures + f] * Bm[kFeatures + f] +
                           Bm[2 * kFeatures + f] * Bm[2 * kFeatures + f];
          const float att = expf(-0.5f * xt[3] * nb);
          s[u] *= att;
          c[u] *= att;
        }
      }
      A.set2(0, 0, 4 * g + i, s[0], s[1]);
      A.set2(0, 0, 8 + 4 * g + i, c[0], c[1]);
    }
  }
  if constexpr (weights_global(H)) {
    static_assert(BF, "weights in device memory: BF16 only");
    const __amdgpu_buffer_rsrc_t rs = image_rsrc(smem, image_bytes(H, BF));
#pragma unroll
    for (int l = 0; l < kLayers; ++l) {
      const int KB = (l == 0) ? 1 : MT;
      const int ws = L.w_stride[l];
      const int lw = (n * ws + 16 * hf) * 2;
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            const bf16x8 wa = img_b128(rs, lw, L.w_off[l] + (mo * 32 * ws + kb * 32 + 8 * jj) * 2);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, A.v[l][kb][jj], acc, 0, 0, 0);
          }
#pragma unroll
        for (int g = 0; g < 4; ++g) {  // rows 8g + 4hf + i
          const f32x4 b4 = img_f4(rs, 16 * hf, L.b_off + (l * H + mo * 32 + 8 * g) * 4);
#pragma unroll
          for (int i = 0; i < 4; ++i) A.set(l + 1, mo, 4 * g + i, fmaxf(acc[4 * g + i] + b4[i], 0.0f));
        }
      }
    }
    if constexpr (!WITH_HEAD) return;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const int lw = (min(n, kOut - 1) * (H + 8) + 16 * hf) * 2;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        bf16x8 wa = img_b128(rs, lw, L.whb_off + (mt * 32 + 8 * jj) * 2);
        if (n >= kOut) wa = bf16x8{};
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, A.v[kLayers][mt][jj], acc, 0, 0, 0);
      }
#pragma unroll
    for (int c = 0; c < kOut; ++c) z[c] = __shfl(acc[c], n) + img_f1(rs, 0, L.bh_off + 4 * c);
    return;
  } else {
  const float* bias = reinterpret_cast<const float*>(smem + L.b_off);
#pragma unroll
  for (int l = 0; l < kLayers; ++l) {
    const int KB = (l == 0) ? 1 : MT;
    const int ws = L.w_stride[l];
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) {
      f32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.f;
      if constexpr (BF) {  // accumulator starts at the bias (one MFMA, exact)
        const bf16x8 ba = *reinterpret_cast<const bf16x8*>(
            reinterpret_cast<const __bf16*>(smem + L.bA_off) + (l * H + mo * 32 + n) * 16 + 8 * hf);
        const bf16x8 ones3 = {(__bf16)1.0f, (__bf16)1.0f, (__bf16)1.0f, (__bf16)0.0f,
                              (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f};
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ba, ones3, acc, 0, 0, 0);
      }
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        if constexpr (BF) {
          const __bf16* wrow = reinterpret_cast<const __bf16*>(smem + L.w_off[l]) +
                               (mo * 32 + n) * ws + kb * 32 + 16 * hf;
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            const bf16x8 wa = *reinterpret_cast<const bf16x8*>(wrow + 8 * jj);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, A.v[l][kb][jj], acc, 0, 0, 0);
          }
        } else {
          const float* wrow = reinterpret_cast<const float*>(smem + L.w_off[l]) +
                              (mo * 32 + n) * ws + kb * 32 + 16 * hf;
#pragma unroll
          for (int q = 0; q < 16; ++q)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wrow[q], A.v[l][kb][q], acc, 0, 0, 0);
        }
      }
      if constexpr (BF) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) A.v[l + 1][mo][jj] = relu_round8(acc, 8 * jj);
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r)
          A.set(l + 1, mo, r, fmaxf(acc[r] + bias[l * H + mo * 32 + rowof(r, hf)], 0.0f));
      }
    }
  }
  if constexpr (!WITH_HEAD) return;
  const float* bh = reinterpret_cast<const float*>(smem + L.bh_off);
  if constexpr (BF) {
    // output layer on MFMA: A = W_out with its four rows padded to 32 (zero rows held in
    // registers, not in LDS); sample n's outputs land in rows 0..3 of lane n (half 0)
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const __bf16* wh = reinterpret_cast<const __bf16*>(smem + L.whb_off);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        bf16x8 wa = {};
        if (n < kOut) wa = *reinterpret_cast<const bf16x8*>(wh + n * (H + 8) + mt * 32 + 16 * hf + 8 * jj);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, A.v[kLayers][mt][jj], acc, 0, 0, 0);
      }
#pragma unroll
    for (int c = 0; c < kOut; ++c) z[c] = __shfl(acc[c], n) + bh[c];
  } else {
    // output layer on the VALU: each half sums its 16 features per block, then the halves are
    // added (the same two addends in both halves, so both hold the same value)
    const float* Wh = reinterpret_cast<const float*>(smem + L.wh_off);
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
      float s = 0.f;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += Wh[c * (H + 4) + mt * 32 + 16 * hf + r] * A.get(kLayers, mt, r);
      s += __shfl_xor(s, 32);
      z[c] = s + bh[c];
    }
  }
  }  // weights in LDS
}

// ---------------------------------------------------------------------------------------------
// The step's tile kernel.

__device__ __forceinline__ void read_batch(StepArgs& a) {
  if (const BatchDev* b = a.bd) {
    a.n_objects = b->n_objects;
    a.n_rays = b->n_rays;
    a.S = b->S;
    a.object_ids = b->object_ids;
    a.ray_offsets = b->ray_offsets;
    a.rays_o = b->rays_o;
    a.rays_d = b->rays_d;
    a.t = b->t;
    a.depth = b->depth;
    a.rgb = b->rgb;
    a.mask = b->mask;
    a.var = b->var;
  }
}

__device__ __forceinline__ void read_batch(OptArgs& a) {
  if (const BatchDev* b = a.bd) {
    a.n_objects = b->n_objects;
    a.ids = b->object_ids;
    a.offs = b->ray_offsets;
    a.loss_out = b->loss_out;
  }
}

// Rendering (Eq. 3), the masked L1 losses (Eqs. 4-7) and, in training, their adjoint for one
// sub-tile of the calling wave: lane = sample slot, zs = the slot's head pre-activations (r, g, b,
// occupancy). Adds the sub-tile's loss to `loss`; forward mode writes the rendered outputs;
// training returns dL/dz of the slot in dzs (zero on slots at or past nslots).
// The rendering's per-sample inputs of a sub-tile (sample depth; the ray's depth, mask and colour
// targets), loaded before the forward pass so that their latency hides behind it.
struct RenderIn {
  float tt, D, M, rgb[3];
};

template <bool TRAIN>
__device__ __forceinline__ RenderIn render_inputs(const StepArgs& a, int r0, int nslots) {
  const int lane = threadIdx.x & 63;
  RenderIn in{0.f, 0.f, 0.f, {0.f, 0.f, 0.f}};
  if (lane < nslots) {
    const int ray = r0 + lane / a.S;
    in.tt = a.t[(size_t)r0 * a.S + lane];
    // rendering without targets (forward mode, NULL target buffers) evaluates the loss terms
    // against zero targets; that loss is not reported
    if (TRAIN || a.depth != nullptr) {
      in.D = a.depth[ray];
      in.M = a.mask[ray];
#pragma unroll
      for (int c = 0; c < 3; ++c) in.rgb[c] = a.rgb[3 * ray + c];
    }
  }
  return in;
}

// Cross-lane moves of the ray scans, by DPP (a VALU operand modifier, no LDS round trip). DPP
// controls: row_shr:n (lane l takes lane l - n of its row of 16), row_shl:n (lane l + n),
// wave_shr:1 / wave_shl:1 (lane l - 1 / l + 1 across the wave), row_bcast:15 (lane 15 of each row
// into the next row, rows 1 and 3 written), row_bcast:31 (lane 31 into rows 2 and 3). Lanes whose
// source does not exist keep 0; the scans below never use those lanes' results. A move reads its
// source lane's register only if that lane is active, so every move runs with the whole wave
// active (computed before any select that uses it, never in a conditional arm).
constexpr int kDppRowShr = 0x110, kDppRowShl = 0x100, kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138,
              kDppBcast15 = 0x142, kDppBcast31 = 0x143;

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                               ROW_MASK, 0xf, false));
}

// Inclusive scans within the rays of a sub-tile. A ray is a segment of S consecutive lanes from
// lane 0 (lanes past the last ray are segments of one lane); si = the lane's position in its
// segment, de = its distance to the segment's last lane. Forward: lane l combines lanes
// [segment start, l], by shifts of 1, 2, 4 and 8 within rows of 16 lanes (a step combines where
// the source lies in both the row and the segment), then lane 15 of each row into the next row
// and lane 31 into rows 2 and 3 (where no segment starts between the row's first lane and l).
// Reverse: lane l combines lanes [l, segment end], by shifts within rows, then the first lane of
// rows 3, 2 and 1 into the row before, in that order.
struct RayScan {
  bool f[6];  // forward steps
  bool r[4];  // reverse steps within rows
  int de, lr, row;

  __device__ __forceinline__ RayScan(int lane, int si, int de_) : de(de_) {
    lr = lane & 15;
    row = lane >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f[i] = si >= (1 << i) && lr >= (1 << i);
      r[i] = de >= (1 << i) && lr + (1 << i) <= 15;
    }
    f[4] = (row & 1) && si > lr;
    f[5] = lane >= 32 && si > lane - 32;
  }

  template <int N, class Op>
  __device__ __forceinline__ void forward(float (&v)[N], Op op) const {
    float u[N];
#define VMAP_SCAN_STEP(I, CTRL, RM)                                        \
  {                                                                        \
    _Pragma("unroll") for (int q = 0; q < N; ++q) u[q] = dpp_mov<CTRL, RM>(v[q]); \
    _Pragma("unroll") for (int q = 0; q < N; ++q) v[q] = f[I] ? op(v[q], u[q]) : v[q]; \
  }
    VMAP_SCAN_STEP(0, kDppRowShr + 1, 0xf)
    VMAP_SCAN_STEP(1, kDppRowShr + 2, 0xf)
    VMAP_SCAN_STEP(2, kDppRowShr + 4, 0xf)
    VMAP_SCAN_STEP(3, kDppRowShr + 8, 0xf)
    VMAP_SCAN_STEP(4, kDppBcast15, 0xa)
    VMAP_SCAN_STEP(5, kDppBcast31, 0xc)
#undef VMAP_SCAN_STEP
  }

  __device__ __forceinline__ float reverse_sum(float v) const {
    float u;
    u = dpp_mov<kDppRowShl + 1>(v); v = r[0] ? v + u : v;
    u = dpp_mov<kDppRowShl + 2>(v); v = r[1] ? v + u : v;
    u = dpp_mov<kDppRowShl + 4>(v); v = r[2] ? v + u : v;
    u = dpp_mov<kDppRowShl + 8>(v); v = r[3] ? v + u : v;
#pragma unroll
    for (int rr = 2; rr >= 0; --rr) {
      const float s = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16 * (rr + 1)));
      v = (row == rr && de > 15 - lr) ? v + s : v;
    }
    return v;
  }
};

template <bool TRAIN>
__device__ __forceinline__ void render_subtile(const StepArgs& a, int r0, int nslots, float wseed,
                                               const RenderIn& in, const float zs[kOut], float dzs[kOut],
                                               float& loss) {
  const int lane = threadIdx.x & 63;
  const int S = a.S;
  const float lc = a.lambda_c, lo = a.lambda_o;
  const bool valid = lane < nslots;
  const int jr = valid ? lane / S : 0;
  const int si = valid ? lane - jr * S : 0;
  const int de = valid ? S - 1 - si : 0;
  const int ray = r0 + jr;
  const RayScan sc(lane, si, de);
  float o = 0.f, q = 1.f, c3[3] = {0.f, 0.f, 0.f}, cq[3] = {0.f, 0.f, 0.f};
  const float tt = in.tt;
  if (valid) {
    sigm_pair(zs[3], o, q);  // q = 1 - o, without cancellation
#pragma unroll
    for (int c = 0; c < 3; ++c) sigm_pair(zs[c], c3[c], cq[c]);
  }
  // P_i = prod_{j<i} (1 - o_j): inclusive product scan within the ray, then shift by one lane
  float pin[1] = {q};
  sc.forward(pin, [](float x, float y) { return x * y; });
  const float Pin = pin[0];
  const float Pprev = dpp_mov<kDppWaveShr1>(Pin);  // outside the select: every lane must take part
  const float Pex = (si == 0) ? 1.f : Pprev;
  const float Tw = o * Pex;  // termination probability T_i
  // the ray's sums end up in its last lane
  float sums[5] = {Tw, Tw * tt, Tw * c3[0], Tw * c3[1], Tw * c3[2]};
  sc.forward(sums, [](float x, float y) { return x + y; });

  // the ray's outputs, loss and residual signs, in its last lane; the signs (each -1, 0 or 1)
  // travel packed to the other lanes of the ray
  int code = 0;
  if (valid && de == 0) {
    const float Oh = sums[0], Dh = sums[1];
    const float Ch[3] = {sums[2], sums[3], sums[4]};
    const float D = in.D, M = in.M;
    const float rD = Dh - D;
    float rC[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rC[c] = Ch[c] - in.rgb[c];
    const float rho = (M == 1.0f) ? -Pin : (Oh - M);
    loss += M * fabsf(rD) + lc * M * (fabsf(rC[0]) + fabsf(rC[1]) + fabsf(rC[2])) + lo * fabsf(rho);
    if constexpr (!TRAIN) {
      if (a.out_depth) a.out_depth[ray] = Dh;
      if (a.out_occ) a.out_occ[ray] = Oh;
      if (a.out_rgb) { a.out_rgb[3 * ray] = Ch[0]; a.out_rgb[3 * ray + 1] = Ch[1]; a.out_rgb[3 * ray + 2] = Ch[2]; }
    }
    auto sgn2 = [](float x) { return (x > 0.f) ? 2 : ((x < 0.f) ? 0 : 1); };
    code = sgn2(rD) | (sgn2(rho) << 2) | (sgn2(rC[0]) << 4) | (sgn2(rC[1]) << 6) | (sgn2(rC[2]) << 8);
  }
  if constexpr (!TRAIN) return;
  code = __shfl(code, jr * S + S - 1);
  auto sgn_of = [&](int i) { return (float)(((code >> (2 * i)) & 3) - 1); };

  float g = 0.f, aC[3] = {0.f, 0.f, 0.f};
  if (valid) {
    const float M = in.M;
    const float aD = wseed * M * sgn_of(0);
    const float aO = wseed * lo * sgn_of(1);
#pragma unroll
    for (int c = 0; c < 3; ++c) aC[c] = wseed * lc * M * sgn_of(2 + c);
    g = aD * tt + aC[0] * c3[0] + aC[1] * c3[1] + aC[2] * c3[2] + aO;
  }
  // adjoint of rendering: dL/dz_occ,i = o_i (q_i g_i P_i - R_i), R_i = sum over the later samples j
  // of the ray of g_j T_j (the exclusive suffix sum, a reverse scan shifted by one lane)
  const float Rin = sc.reverse_sum(g * Tw);
  const float Rnext = dpp_mov<kDppWaveShl1>(Rin);
  const float R = (de == 0) ? 0.f : Rnext;
  dzs[3] = valid ? o * (q * g * Pex - R) : 0.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) dzs[c] = valid ? Tw * aC[c] * c3[c] * cq[c] : 0.f;
}

// ---------------------------------------------------------------------------------------------
// Per-object gradient and optimiser. Tile partials are already unscaled by the tile kernel, which
// also flagged objects with a non-finite partial. Three kernels share the pieces below:
//   k_reduce      — loss and gradient per object (forward/backward split),
//   k_adam        — Adam from the stored gradient (after k_reduce),
//   k_reduce_adam — both in one pass (the training step when it is split into launches).
// The optimiser kernels take each object's next step count from the work-list kernel; block
// (0, j) writes it back; block (0, 0) of k_reduce and k_adam, and the extra last row of
// k_reduce_adam, update the loss scaler from the flags. No block reads what
// another block of the same launch writes, so no device-scope fence is needed. After a MODE_STEP
// tile launch (below) the table, step counts and cleared flags come from the tile kernel and the
// non-finite reports from its tiles.

// Sum of an object's tile partials at parameter p, in tile order; up to 32 loads are issued
// before the first add (objects here have at most a few tens of tiles).
__device__ __forceinline__ float tile_sum(const float* __restrict__ partial, int p_stride, int t0,
                                          int t1, int p) {
  float g = 0.f;
  for (int t = t0; t < t1; t += 32) {
    float x[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) x[u] = (t + u < t1) ? partial[(size_t)(t + u) * p_stride + p] : 0.f;
#pragma unroll
    for (int u = 0; u < 32; ++u)
      if (t + u < t1) g += x[u];
  }
  return g;
}


__device__ __forceinline__ bool obj_valid(const OptArgs& a, int k) {
  return k >= 0 && k < a.max_objects && a.desc[k].registered;
}

// Whether batch object j (id k) had a non-finite tile partial: bit 0 of its flag (set by the tiles;
// k_reduce_adam marks its own overflows in bit 1, which this test leaves out, so every workgroup
// of an object decides alike), or with per-tile reports the OR of its tiles' entries. Called by
// every thread of the workgroup.
__device__ __forceinline__ bool object_bad(const OptArgs& a, int j, int k) {
  if (!a.tile_bad) return __syncthreads_or((a.flags[k] & 1) != 0) != 0;
  int bad = 0;
  const TileRange tr = clamp_tile_range(a.tile_start[j], a.tile_start[j + 1], a.max_tiles);
  for (int t = tr.t0 + (int)threadIdx.x; t < tr.t1; t += blockDim.x) bad |= a.tile_bad[t];
  return __syncthreads_or(bad) != 0;
}

// OR of the non-finite reports of tiles [t0, t1); up to 32 loads are issued before the first use.
__device__ __forceinline__ int tile_or(const int32_t* __restrict__ bad, int t0, int t1) {
  int r = 0;
  for (int t = t0; t < t1; t += 32) {
    int x[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) x[u] = (t + u < t1) ? bad[t + u] : 0;
#pragma unroll
    for (int u = 0; u < 32; ++u) r |= x[u];
  }
  return r;
}

// One workgroup (any size): count the batch objects with rays whose gradient was not finite;
// BF16 loss scaler. (On the split path an overflow that k_reduce_adam finds while summing finite
// partials is flagged during this same launch, so it is counted only if its flag is already
// visible; the per-tile reports of the training step are complete before the launch.) Each thread loads its object's id, rays, tiles and descriptor at once (an id
// out of range reads object 0's descriptor and is then discarded), then its tiles' reports.
__device__ void scaler_update(const OptArgs& a) {
  __shared__ int count;
  if (!a.scaler->batch_ok) return;  // the batch did not run: the scaler stays as it is
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  int skipped = 0;
  for (int jj = threadIdx.x; jj < a.n_objects; jj += blockDim.x) {
    const int kk = a.ids[jj];
    const int r0 = a.offs[jj], r1 = a.offs[jj + 1];
    const TileRange tr = clamp_tile_range(a.tile_start[jj], a.tile_start[jj + 1], a.max_tiles);
    const int t0 = tr.t0, t1 = tr.t1;
    const bool in_range = kk >= 0 && kk < a.max_objects;
    const int kc = in_range ? kk : 0;
    const bool registered = a.desc[kc].registered != 0;
    // from the tiles: the objects' flags are being written by this launch
    const int bad = a.tile_bad ? tile_or(a.tile_bad, t0, t1) : a.flags[kc];
    if (in_range && registered && r1 > r0 && bad != 0) ++skipped;
  }
  if (skipped) atomicAdd(&count, skipped);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int total = count;
    a.scaler->skipped = total;
    if (a.bf16) {
      // the scale stays a power of two in [2^-125, 2^126], so that it and its inverse are normal
      const float sc = a.scaler->scale;
      if (total > 0) {
        if (sc >= 0x1p-124f) a.scaler->scale = sc * 0.5f;
        a.scaler->good_steps = 0;
      } else if (++a.scaler->good_steps >= a.growth) {
        if (sc <= 0x1p125f) a.scaler->scale = sc * 2.0f;
        a.scaler->good_steps = 0;
      }
    }
  }
}

struct AdamCoef {
  float step, rs, b1, c1, b2, c2, eps;
};

// Bias-corrected step size and 1/sqrt(bias correction of v) in FP64, then rounded once.
__device__ __forceinline__ void adam_coef_store(const OptArgs& a, int t, float* sh) {
  const double bc1 = 1.0 - pow(a.beta1, (double)t), bc2 = 1.0 - pow(a.beta2, (double)t);
  sh[0] = (float)(a.lr / bc1);
  sh[1] = (float)(1.0 / sqrt(bc2));
}

__device__ __forceinline__ AdamCoef adam_coef_load(const OptArgs& a, const float* sh) {
  return AdamCoef{sh[0], sh[1], (float)a.beta1, (float)(1.0 - a.beta1), (float)a.beta2,
                  (float)(1.0 - a.beta2), (float)a.eps};
}

__device__ AdamCoef adam_coef(const OptArgs& a, int t) {
  __shared__ float sh[2];
  if (threadIdx.x == 0) adam_coef_store(a, t, sh);
  __syncthreads();
  return adam_coef_load(a, sh);
}

// Parameter p of object k changed to th: its entry in the object's weight image (width 32, also
// for hidden 16, whose image is the zero-padded width-32 one; the BF16 image of hidden 128), or
// in its BF16 parameter copy (layered path, hidden 256 and up). WIDE = false leaves out the
// hidden-128 image, for k_reduce_adam: a stack that can hold hidden-128 objects has at least
// kReduceWide parameter slots per object and takes k_reduce_adam_wide (its launcher checks).
template <bool WIDE = true>
__device__ __forceinline__ void update_image(const OptArgs& a, int k, int hidden, int p, float th) {
  if (a.gimg && keeps_gimg(hidden)) {
    a.gimg[(size_t)k * a.p_stride + p] = (uint16_t)(pack2(th, 0.f) & 0xffffu);
    return;
  }
  if constexpr (WIDE) {
    if (hidden == 128) {
      if (a.wimage && a.bf16) place_param<128, true>(a.wimage + (size_t)k * a.wimage_stride, p, th);
      return;
    }
  }
  if (!a.img32 || kernel_width(hidden) != 32) return;
  const int q = padded_index(hidden, p);
  if (a.bf16) place_param<32, true>(a.img32 + (size_t)k * img32_bytes(true), q, th);
  else place_param<32, false>(a.img32 + (size_t)k * img32_bytes(false), q, th);
}

// One Adam update; the contractions are spelled out so that the rounding does not depend on how
// the compiler schedules the surrounding code.
__device__ __forceinline__ void adam_elem(const AdamCoef& c, float g, float& th, float& m, float& v) {
  m = fmaf(c.b1, m, c.c1 * g);
  v = fmaf(c.b2, v, c.c2 * (g * g));
  th = fmaf(-c.step, m / fmaf(sqrtf(v), c.rs, c.eps), th);
}

// ---------------------------------------------------------------------------------------------
// Training step without a work-list launch (MODE_STEP). Every workgroup of the tile kernel scans
// the batch's ray offsets into a tile table in LDS (what k_worklist writes to device memory);
// workgroup 0 also leaves in device memory what k_worklist leaves for the optimiser: the table,
// the next Adam step counts and cleared flags. Tiles then report a non-finite partial in their
// own tile_bad entry instead of the object's flag (which workgroup 0 may clear concurrently), and
// k_reduce_adam reads those entries.

// tbl[j] = first tile of batch object j, tbl[n_objects] = tiles: the exclusive scan of
// ceil(rays_j / rays_per_tile) over the batch (the launch's objects share one width, so one tile
// size); tray[j] = the batch's ray offsets (n_objects + 1 of them) and tk[j] = object ids, so that
// a tile finds its object and rays in LDS. Returns the tile count, or -1 when the offsets fail
// the check of segment_ok (ray_offsets[0] = 0, every segment inside [0, n_rays] and in order,
// ray_offsets[n] = n_rays); then no tile runs. Called by every thread of the workgroup.
__device__ int step_table(const StepArgs& a, int32_t* tbl, int32_t* tray, int32_t* tk) {
  __shared__ int wtot[8];  // up to eight waves
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int rpt = a.rays_per_tile;
  int carry = 0, bad = 0;
  for (int base = 0; base < a.n_objects; base += nt) {
    const int j = base + tid;
    int cnt = 0;
    if (j < a.n_objects) {
      const int o0 = a.ray_offsets[j], o1 = a.ray_offsets[j + 1];
      tray[j] = o0;
      tk[j] = a.object_ids[j];
      if (j == a.n_objects - 1) tray[j + 1] = o1;
      const bool ok = batch_segment_ok(j, a.n_objects, o0, o1, a.n_rays);
      bad |= !ok;
      cnt = ok ? tiles_of(o1 - o0, rpt) : 0;
    }
    // inclusive scan over the wave by DPP: shifts within rows of 16, then lane 15 of each row
    // into the next row and lane 31 into rows 2 and 3 (every move with the whole wave active)
    int x = cnt;
    const int lr = lane & 15;
    int y = __builtin_amdgcn_update_dpp(0, x, kDppRowShr + 1, 0xf, 0xf, false);
    x += (lr >= 1) ? y : 0;
    y = __builtin_amdgcn_update_dpp(0, x, kDppRowShr + 2, 0xf, 0xf, false);
    x += (lr >= 2) ? y : 0;
    y = __builtin_amdgcn_update_dpp(0, x, kDppRowShr + 4, 0xf, 0xf, false);
    x += (lr >= 4) ? y : 0;
    y = __builtin_amdgcn_update_dpp(0, x, kDppRowShr + 8, 0xf, 0xf, false);
    x += (lr >= 8) ? y : 0;
    y = __builtin_amdgcn_update_dpp(0, x, kDppBcast15, 0xa, 0xf, false);
    x += ((lane >> 4) & 1) ? y : 0;
    y = __builtin_amdgcn_update_dpp(0, x, kDppBcast31, 0xc, 0xf, false);
    x += (lane >= 32) ? y : 0;
    if (lane == kWave - 1) wtot[wave] = x;
    __syncthreads();
    int before = carry, total = 0;
    for (int w = 0; w < nw; ++w) {
      const int v = wtot[w];
      if (w < wave) before += v;
      total += v;
    }
    if (j < a.n_objects) tbl[j] = before + x - cnt;
    carry += total;
    __syncthreads();
  }
  if (tid == 0) tbl[a.n_objects] = carry;
  return __syncthreads_or(bad) ? -1 : carry;
}

template <int H, bool BF, int MODE>
// BF16 at width 32: up to eight waves per workgroup, 256 registers (two waves per SIMD).
__global__ void __launch_bounds__((BF && H == 32) ? 512 : 256, 1) k_step_tiles(const StepArgs a_in) {
  StepArgs a = a_in;
  read_batch(a);
  constexpr int MT = H / 32;
  constexpr bool TABLE = (MODE == MODE_STEP);  // tile table built here, not by k_worklist
  constexpr bool TRAIN = (MODE == MODE_TRAIN) || TABLE;
  constexpr bool KEEP = TRAIN && !BF;  // activations kept across the rendering (no recompute)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr LdsLayout L = lds_layout(H, BF, 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int n = lane & 31, hf = lane >> 5;
  const int S = a.S;
  const int rpw = kSlots / S;

  // first tile of every batch object: from the LDS table or from k_worklist
  // (and, with the LDS table, its ray offsets and object ids)
  const int tbl_words = round_up(a.n_objects + 1, 4);
  int32_t* tbl = reinterpret_cast<int32_t*>(smem + a.lds_table);
  int32_t* tray = tbl + tbl_words;
  int32_t* tk = tray + tbl_words;
  auto first_tile = [&](int j) { return TABLE ? tbl[j] : a.tile_start[j]; };
  int n_tiles;
  if constexpr (TABLE) {
    n_tiles = step_table(a, tbl, tray, tk);
    if (blockIdx.x == 0) {  // what k_worklist leaves for the optimiser
      if (tid == 0) {
        a.scaler->batch_ok = n_tiles >= 0;
        if (n_tiles < 0) atomicOr(&a.scaler->device_error, DERR_OFFSETS);
      }
      for (int j = tid; j <= a.n_objects; j += blockDim.x) a.tile_start_out[j] = n_tiles >= 0 ? tbl[j] : 0;
      for (int j = tid; j < a.n_objects; j += blockDim.x) {
        const int k = tk[j];
        const bool valid = k >= 0 && k < a.max_objects;
        if (valid) a.flags[k] = 0;
        a.t_next[j] = (valid && a.desc[k].registered) ? a.desc[k].step + 1 : 0;
      }
    }
  } else {
    n_tiles = a.tile_start[a.n_objects];
  }
  n_tiles = clamp_tiles(n_tiles, a.max_tiles);

  float* Bl = reinterpret_cast<float*>(smem + L.B_off);
  if (tid < 3 * kFeatures) Bl[tid] = a.B[tid];
  int staged = -1;

  // XCD-aware order only when every tile belongs to this launch (tiles of other widths would
  // crowd the XCDs that hold them)
  for (int tile = TABLE ? first_tile_of_block(n_tiles) : (int)blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    // object of this tile: the j with first_tile(j) <= tile < first_tile(j + 1) (objects without
    // rays have an empty range), 64 candidates per wave at a time
    int j = 0;
    for (int base = 0; base < a.n_objects; base += kWave) {
      const int jj = base + lane;
      const bool hit = jj < a.n_objects && first_tile(jj) <= tile && tile < first_tile(jj + 1);
      const unsigned long long m = __ballot(hit);
      if (m) {
        j = base + __ffsll((long long)m) - 1;
        break;
      }
    }
    const int k = TABLE ? tk[j] : a.object_ids[j];
    const int rpt = tile_rays(H, a.rays_per_tile, a.rays_per_tile_wide);
    const RayRange rr = tile_ray_range(TABLE ? tray[j] : a.ray_offsets[j],
                                       TABLE ? tray[j + 1] : a.ray_offsets[j + 1],
                                       tile - first_tile(j), rpt, a.n_rays);
    const int ray_lo = rr.lo, ray_hi = rr.hi;
    const int nrays = ray_hi - ray_lo;
    const int nsub = (nrays + rpw - 1) / rpw;
    // The object's weight image goes to LDS before its descriptor is checked, so that the two are
    // fetched together (an id out of range fetches object 0's image, which is then discarded).
    const bool k_ok = k >= 0 && k < a.max_objects;
    const int kc = k_ok ? k : 0;
    static_assert(H == 32 && L.B_off % 16 == 0, "weight images are kept for width 32");
    const unsigned char* img = a.img32 + (size_t)kc * img32_bytes(BF);
    const bool restage = (k != staged);
    if (restage) {  // the object's weight image, as it is, straight into LDS
      if (staged >= 0) __syncthreads();  // the previous object's weights are no longer read
      fetch_image_lds(img, smem, L.B_off, lane, wave, nw);
      staged = -1;
    }
    const ObjDesc& od = a.desc[kc];
    const int registered = od.registered, hidden = od.hidden;
    const double cx = od.centre[0], cy = od.centre[1], cz = od.centre[2];
    const double inv_s = od.inv_scale;
    float wseed = 1.0f;
    if constexpr (TRAIN) {
      if (a.dloss) wseed = a.dloss[j];
      if (a.use_scale) wseed *= a.scaler->scale;
    }
    if (!k_ok || !registered) {
      if (tid == 0) atomicOr(&a.scaler->device_error, 1);
      continue;
    }
    if (kernel_width(hidden) != H) continue;  // handled by the launch for that width
    if (restage) {
      __builtin_amdgcn_s_waitcnt(0);  // this thread's part of the image is in LDS
      staged = k;
    }
    __syncthreads();

    f32x16 accW[kLayers][MT][MT];
    f32x4 accWh[H / 16];  // BF16: output-layer weight gradient, 16x16 blocks (rows 0..3 used)
    float accH[kOut][MT];
    float accDb[kLayers][MT];
    float accDbH[kOut];
    if constexpr (TRAIN) {
#pragma unroll
      for (int l = 0; l < kLayers; ++l)
#pragma unroll
        for (int mo = 0; mo < MT; ++mo) {
          accDb[l][mo] = 0.f;
#pragma unroll
          for (int ki = 0; ki < MT; ++ki)
#pragma unroll
            for (int r = 0; r < 16; ++r) accW[l][mo][ki][r] = 0.f;
        }
#pragma unroll
      for (int c = 0; c < kOut; ++c) {
        accDbH[c] = 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) accH[c][mt] = 0.f;
      }
#pragma unroll
      for (int b = 0; b < H / 16; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) accWh[b][i] = 0.f;
    }
    float wave_loss = 0.f;

    unsigned char* scr = smem + L.scratch_off + wave * L.scratch_wave;
    unsigned char* encc = scr + dz_tile_bytes(BF) + 2 * tr_tile_bytes(H, BF);

    for (int sub = wave; sub < nsub; sub += nw) {
      asm volatile("" ::: "memory");
      const int r0 = ray_lo + sub * rpw;
      const int nr = min(rpw, ray_hi - r0);
      const int nslots = nr * S;
      const RenderIn rin = render_inputs<TRAIN>(a, r0, nslots);  // in flight during the forward

      // ---------------- forward of both passes for the head outputs only. Each pass's
      // activations are recomputed right before its backward (activation recomputation), so no
      // activation is held across the rendering.
      // the lane's sample: normalised point and (integrated encoding) normalised variance
      auto point = [&](int p, float xt[4]) {
        const int slot = 32 * p + n;
        xt[0] = xt[1] = xt[2] = xt[3] = 0.f;
        if (slot < nslots) {
          const int ray = r0 + slot / S;
          const double tt = (double)a.t[(size_t)r0 * S + slot];
          const float* o3 = a.rays_o + 3 * (size_t)ray;
          const float* d3 = a.rays_d + 3 * (size_t)ray;
          xt[0] = (float)(((double)o3[0] + tt * (double)d3[0] - cx) * inv_s);
          xt[1] = (float)(((double)o3[1] + tt * (double)d3[1] - cy) * inv_s);
          xt[2] = (float)(((double)o3[2] + tt * (double)d3[2] - cz) * inv_s);
          if (a.var) xt[3] = (float)((double)a.var[(size_t)r0 * S + slot] * inv_s * inv_s);
        }
      };
      float zs[kOut] = {0.f, 0.f, 0.f, 0.f};
      // FP32 (one wave per SIMD either way) keeps both passes' activations for the backward;
      // BF16 recomputes them there from the encodings kept in LDS (no sine/cosine twice), which
      // keeps it at two waves per SIMD (measured faster than keeping the activations).
      Acts<H, BF> keep0, keep1;
      if constexpr (KEEP) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          float xt[4], z[kOut];
          point(p, xt);
          forward_pass<H, BF, true>(xt, smem, Bl, p == 0 ? keep0 : keep1, z, a.var != nullptr);
#pragma unroll
          for (int c = 0; c < kOut; ++c) zs[c] = (hf == p) ? z[c] : zs[c];
        }
      } else {  // (unrolled: the two passes' chains interleave)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          Acts<H, BF> tmp;
          float xt[4], z[kOut];
          point(p, xt);
          forward_pass<H, BF, true>(xt, smem, Bl, tmp, z, a.var != nullptr);
#pragma unroll
          for (int c = 0; c < kOut; ++c) zs[c] = (hf == p) ? z[c] : zs[c];
          if constexpr (TRAIN && BF) {
            if (p == 1) {  // the last pass's activations stay for its backward, which runs first
              keep1 = tmp;
            } else {  // the first pass's encoding, for its recomputation
#pragma unroll
              for (int jj = 0; jj < 2; ++jj)
                *reinterpret_cast<bf16x8*>(encc + lane * 32 + 16 * jj) = tmp.v[0][0][jj];
            }
          }
        }
      }

      float dzs[kOut];
      render_subtile<TRAIN>(a, r0, nslots, wseed, rin, zs, dzs, wave_loss);
      if constexpr (!TRAIN) continue;
#pragma unroll
      for (int c = 0; c < kOut; ++c) accDbH[c] += dzs[c];

      // ---------------- MLP backward, one pass of 32 samples at a time
      unsigned char* dzt = scr;
      unsigned char* dtile = scr + dz_tile_bytes(BF);
      unsigned char* htile = dtile + tr_tile_bytes(H, BF);
      // one pass's backward (p: which 32 samples); BF16 runs the last pass first, on the
      // activations its forward left in registers, and recomputes only the first pass
      auto backward_pass = [&](const int p) {
        Acts<H, BF> act;
        if constexpr (KEEP) {
#pragma unroll
          for (int l = 0; l <= kLayers; ++l)
#pragma unroll
            for (int b = 0; b < H / 32; ++b)
#pragma unroll
              for (int q = 0; q < (int)(sizeof(act.v[0][0]) / sizeof(act.v[0][0][0])); ++q)
                act.v[l][b][q] = (p == 0) ? keep0.v[l][b][q] : keep1.v[l][b][q];
        } else if constexpr (BF) {
          if (p == 1) {
            act = keep1;
          } else {  // recompute from the pass's encoding kept in LDS
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
              act.v[0][0][jj] = *reinterpret_cast<const bf16x8*>(encc + lane * 32 + 16 * jj);
            float z[kOut];
            forward_pass<H, BF, false, false>(nullptr, smem, Bl, act, z);
          }
        } else {
          float xt[4], z[kOut];
          point(p, xt);
          forward_pass<H, BF, false>(xt, smem, Bl, act, z, a.var != nullptr);
        }
        // the pass's dL/dz sits in lanes 32p..32p+31; FP32 moves it to both halves
        float dz[kOut];
        if constexpr (!BF) {
#pragma unroll
          for (int c = 0; c < kOut; ++c) dz[c] = __shfl(dzs[c], 32 * p + n);
        }
        // stage dz and h_L, transposed for the output layer's weight gradient
        wave_lds_sync();
        if constexpr (BF) {  // written by the lanes that hold it (no cross-lane move)
          if (hf == p) {
            bf16x4 d4;
#pragma unroll
            for (int c = 0; c < kOut; ++c) {
              d4[c] = (__bf16)dzs[c];
              reinterpret_cast<__bf16*>(dzt)[c * 40 + n] = d4[c];
            }
            *reinterpret_cast<bf16x4*>(dzt + kDzRowsBytes + 8 * n) = d4;
          }
        } else if (hf == 0) {
#pragma unroll
          for (int c = 0; c < kOut; ++c) reinterpret_cast<float*>(dzt)[n * kOut + c] = dz[c];
        }
        if constexpr (BF) {  // sample-major runs (register block jj: features 16jj + 4hf + 0..3, + 8)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
              write_runs(reinterpret_cast<__bf16*>(htile) + n * kTrStride + mt * 32 + 16 * jj + 4 * hf,
                         act.v[kLayers][mt][jj]);
        } else {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r)
              reinterpret_cast<float*>(htile)[n * (H + 4) + mt * 32 + rowof(r, hf)] = act.v[kLayers][mt][r];
        }
        wave_lds_sync();
        Deltas<H, BF> dl;
        if constexpr (BF) {
          // output-layer weight gradient on MFMA 16x16x32: rows = the four outputs (padded to 16),
          // columns = 16 features, K = the pass's 32 samples
          const int m16 = lane & 15, kg = lane >> 4;
          bf16x8 da = {};
          if (m16 < kOut) da = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const __bf16*>(dzt) + m16 * 40 + 8 * kg);
          // B operand (feature 16b + m16, samples 8kg..8kg+7): lane x of group kg addresses row
          // 8kg + x/4 at feature 16b + 4(x mod 4)
          const __bf16* hq = reinterpret_cast<const __bf16*>(htile) + (8 * kg + (m16 >> 2)) * kTrStride + 4 * (m16 & 3);
#pragma unroll
          for (int b = 0; b < H / 16; ++b) {
            const bf16x8 hb = tr_read8(hq + 16 * b);
            accWh[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(da, hb, accWh[b], 0, 0, 0);
          }
          // delta of the last hidden layer: W_out^T dz on MFMA (K = 4 outputs padded to 16)
          bf16x8 dzb = {};
          if (hf == 0) {
            const bf16x4 d4 = *reinterpret_cast<const bf16x4*>(dzt + kDzRowsBytes + 8 * n);
#pragma unroll
            for (int c = 0; c < kOut; ++c) dzb[c] = d4[c];
          }
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            bf16x8 wa = {};
            if (hf == 0) {
              const __bf16* wt = reinterpret_cast<const __bf16*>(smem + L.whtb_off) + (mt * 32 + n) * kOut;
#pragma unroll
              for (int c = 0; c < kOut; ++c) wa[c] = wt[c];
            }
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.f;
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, dzb, acc, 0, 0, 0);
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) dl.v[mt][jj] = relu_mask(round8(acc, 8 * jj), act.v[kLayers][mt][jj]);
          }
        } else {
          // output-layer weight gradient: lane owns feature mt*32 + n, half hf takes 16 samples
          const float* dzl = reinterpret_cast<const float*>(dzt);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) {
              const int s = 16 * hf + s2;
              const float hv = reinterpret_cast<const float*>(htile)[s * (H + 4) + mt * 32 + n];
#pragma unroll
              for (int c = 0; c < kOut; ++c) accH[c][mt] += dzl[s * kOut + c] * hv;
            }
          }
          // delta of the last hidden layer: (W_out^T dz) masked by ReLU'
          const float* Wh = reinterpret_cast<const float*>(smem + L.wh_off);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              float s = 0.f;
#pragma unroll
              for (int c = 0; c < kOut; ++c) s += Wh[c * (H + 4) + mt * 32 + 16 * hf + r] * dz[c];
              const float hv = reinterpret_cast<const float*>(htile)[n * (H + 4) + mt * 32 + rowof(r, hf)];
              dl.set(mt, r, (hv > 0.f) ? s : 0.f);
            }
        }
#pragma unroll
        for (int l = kLayers - 1; l >= 0; --l) {
          const int KB = (l == 0) ? 1 : MT;
          // delta_{l-1} = (W_l^T delta_l) masked by ReLU' of layer l-1: its products first, so that
          // they run while this layer's operands are staged and its weight gradient accumulates
          const int ws = L.w_stride[l > 0 ? l : 1];
          f32x16 nacc[MT];
          if (l > 0) {
#pragma unroll
            for (int mi = 0; mi < MT; ++mi) {
              f32x16& acc = nacc[mi];
#pragma unroll
              for (int r = 0; r < 16; ++r) acc[r] = 0.f;
              const int col = mi * 32 + colpos(n);
#pragma unroll
              for (int ko = 0; ko < MT; ++ko) {
                if constexpr (BF) {
                  // A = W_l^T from its transposed copy: 8 consecutive BF16 per lane
                  const __bf16* Wt = reinterpret_cast<const __bf16*>(smem + L.wt_off[l]) +
                                     (mi * 32 + n) * (H + 8) + ko * 32 + 16 * hf;
#pragma unroll
                  for (int jj = 0; jj < 2; ++jj) {
                    const bf16x8 wa = *reinterpret_cast<const bf16x8*>(Wt + 8 * jj);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, dl.v[ko][jj], acc, 0, 0, 0);
                  }
                } else {
                  const float* W = reinterpret_cast<const float*>(smem + L.w_off[l]);
#pragma unroll
                  for (int qq = 0; qq < 16; ++qq)
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(W[(ko * 32 + rowof(qq, hf)) * ws + col],
                                                               dl.v[ko][qq], acc, 0, 0, 0);
                }
              }
            }
          }
          // stage delta_l (out features) and h_{l-1} (in features): BF16 sample-major runs, FP32
          // sample-major
          wave_lds_sync();
          if constexpr (BF) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
              for (int jj = 0; jj < 2; ++jj)
                write_runs(reinterpret_cast<__bf16*>(dtile) + n * kTrStride + mt * 32 + 16 * jj + 4 * hf,
                           dl.v[mt][jj]);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
#pragma unroll
              for (int jj = 0; jj < 2; ++jj)
                write_runs(reinterpret_cast<__bf16*>(htile) + n * kTrStride + kb * 32 + 16 * jj + 4 * hf,
                           act.v[l][kb][jj]);
          } else {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
              for (int r = 0; r < 16; ++r)
                reinterpret_cast<float*>(dtile)[n * (H + 4) + mt * 32 + rowof(r, hf)] = dl.v[mt][r];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
#pragma unroll
              for (int r = 0; r < 16; ++r)
                reinterpret_cast<float*>(htile)[n * (H + 4) + kb * 32 + rowof(r, hf)] = act.v[l][kb][r];
          }
          wave_lds_sync();
          // weight gradient dW_l += delta_l h_{l-1}^T over the pass's 32 samples
#pragma unroll
          for (int mo = 0; mo < MT; ++mo) {
#pragma unroll
            for (int ki = 0; ki < KB; ++ki) {
              if constexpr (BF) {
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) {
                  // A and B operands (feature row lane & 31, samples 16jj + 8hf + 0..7): lane x of
                  // group G = lane / 16 addresses row 16jj + 8(G / 2) + x/4 at feature
                  // 16(G mod 2) + 4(x mod 4)
                  const int lo = (16 * jj + 8 * hf + ((lane & 15) >> 2)) * kTrStride + 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
                  const bf16x8 da = tr_read8(reinterpret_cast<const __bf16*>(dtile) + lo + mo * 32);
                  const bf16x8 hb = tr_read8(reinterpret_cast<const __bf16*>(htile) + lo + ki * 32);
                  accW[l][mo][ki] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(da, hb, accW[l][mo][ki], 0, 0, 0);
                  if (ki == 0) {  // bias gradient: the 8 deltas' sum, two at a time (v_dot2)
                    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
                    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
                    const u4 dw = __builtin_bit_cast(u4, da);
                    const b2 ones = {(__bf16)1.0f, (__bf16)1.0f};
                    float s = 0.f;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                      s = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(b2, (unsigned int)dw[e]), ones, s, false);
                    accDb[l][mo] += s;
                  }
                }
              } else {
#pragma unroll
                for (int qq = 0; qq < 16; ++qq) {
                  const int s = 2 * qq + hf;
                  const float da = reinterpret_cast<const float*>(dtile)[s * (H + 4) + mo * 32 + n];
                  const float hb = reinterpret_cast<const float*>(htile)[s * (H + 4) + ki * 32 + n];
                  accW[l][mo][ki] = __builtin_amdgcn_mfma_f32_32x32x2f32(da, hb, accW[l][mo][ki], 0, 0, 0);
                  if (ki == 0) accDb[l][mo] += da;
                }
              }
            }
          }
          if (l == 0) break;
          Deltas<H, BF> nd;
#pragma unroll
          for (int mi = 0; mi < MT; ++mi) {
            const f32x16& acc = nacc[mi];
            if constexpr (BF) {
#pragma unroll
              for (int jj = 0; jj < 2; ++jj) nd.v[mi][jj] = relu_mask(round8(acc, 8 * jj), act.v[l][mi][jj]);
            } else {
#pragma unroll
              for (int r = 0; r < 16; ++r) {
                const float hv = reinterpret_cast<const float*>(htile)[n * (H + 4) + mi * 32 + rowof(r, hf)];
                nd.set(mi, r, (hv > 0.f) ? acc[r] : 0.f);
              }
            }
          }
          dl = nd;
        }
      };
      if constexpr (BF) {
        backward_pass(1);
        backward_pass(0);
      } else {
#pragma unroll 1
        for (int p = 0; p < 2; ++p) backward_pass(p);
      }
    }  // sub-tiles

    // ---------------- combine the waves of the workgroup in a fixed order
    // per-wave reductions in registers first
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) wave_loss += __shfl_xor(wave_loss, off);
    if constexpr (TRAIN) {
#pragma unroll
      for (int c = 0; c < kOut; ++c) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) accDbH[c] += __shfl_xor(accDbH[c], off);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) accH[c][mt] += __shfl_xor(accH[c][mt], 32);
      }
#pragma unroll
      for (int l = 0; l < kLayers; ++l)
#pragma unroll
        for (int mo = 0; mo < MT; ++mo) accDb[l][mo] += __shfl_xor(accDb[l][mo], 32);
    }
    __syncthreads();  // staging buffers are free: reuse them for the tile's gradient
    // nc copies of the tile's gradient and loss (two for two to seven waves, four for eight): the
    // first nc waves write them, the others then add theirs in turn (copy c = waves c, c + nc, ...,
    // in that order); the partial is the sum of the copies in order.
    constexpr int kRedWords = round_up(n_params_of(H), 4);
    const int nc = red_copies(nw);
    float* red0 = reinterpret_cast<float*>(smem + L.scratch_off);
    float* red = red0 + (wave % nc) * kRedWords;
    float* lsum = reinterpret_cast<float*>(smem + L.loss_off);
    int* any_bad = reinterpret_cast<int*>(smem + L.loss_off + 16);
    if (tid == 0) *any_bad = 0;  // read after the barriers below
    // lane, n and hf again, through an empty asm statement: the addresses below are then computed
    // here, not hoisted to the kernel's start and kept (spilled) across the sub-tiles
    int rl = lane;
    asm volatile("" : "+v"(rl));
    const int rn = rl & 31, rh = rl >> 5;
    for (int ph = 0; ph < (nw + nc - 1) / nc; ++ph) {
      if (wave / nc == ph) {
        const bool first = (ph == 0);
        if (rl == 0) lsum[wave % nc] = (first ? 0.f : lsum[wave % nc]) + wave_loss;
        if constexpr (TRAIN) {
          int off = 0;
#pragma unroll
          for (int l = 0; l < kLayers; ++l) {
            const int K = (l == 0) ? kEnc : H;
            const int KB = K / 32;
#pragma unroll
            for (int mo = 0; mo < MT; ++mo)
#pragma unroll
              for (int ki = 0; ki < KB; ++ki)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                  const int idx = off + (mo * 32 + rowof(r, rh)) * K + ki * 32 + rn;
                  red[idx] = (first ? 0.f : red[idx]) + accW[l][mo][ki][r];
                }
            off += H * K;
            if (rh == 0) {
#pragma unroll
              for (int mo = 0; mo < MT; ++mo) {
                const int idx = off + mo * 32 + rn;
                red[idx] = (first ? 0.f : red[idx]) + accDb[l][mo];
              }
            }
            off += H;
          }
          if constexpr (BF) {
            if (rl < 16) {
#pragma unroll
              for (int c = 0; c < kOut; ++c)
#pragma unroll
                for (int b = 0; b < H / 16; ++b) {
                  const int idx = off + c * H + b * 16 + rl;
                  red[idx] = (first ? 0.f : red[idx]) + accWh[b][c];
                }
            }
          } else if (rh == 0) {
#pragma unroll
            for (int c = 0; c < kOut; ++c)
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) {
                const int idx = off + c * H + mt * 32 + rn;
                red[idx] = (first ? 0.f : red[idx]) + accH[c][mt];
              }
          }
          off += kOut * H;
          if (lane == 0) {
#pragma unroll
            for (int c = 0; c < kOut; ++c) red[off + c] = (first ? 0.f : red[off + c]) + accDbH[c];
          }
        }
      }
      __syncthreads();
    }
    if constexpr (TRAIN) {
      // unscale (exact: the scale is a power of two) and report a partial that is not finite or
      // too large to be summed safely (partial_bad)
      const int P = n_params_of(H);
      const float inv = a.use_scale ? 1.0f / a.scaler->scale : 1.0f;
      float* dst = a.partial + (size_t)tile * a.p_stride;
      int bad = 0;
      for (int e = tid; e < P; e += blockDim.x) {
        float g = red0[e];
        for (int c = 1; c < nc; ++c) g += red0[c * kRedWords + e];
        g *= inv;
        bad |= partial_bad(g);
        __builtin_nontemporal_store(g, &dst[e]);  // read once, by the next kernel
      }
      if (bad) *any_bad = 1;  // every writer stores the same value
      __syncthreads();
      if (tid == 0) {
        if constexpr (TABLE) a.tile_bad[tile] = *any_bad;
        else if (*any_bad) atomicOr(&a.flags[k], 1);
      }
    }
    if (tid == 0) {
      float l = lsum[0];
      for (int c = 1; c < nc; ++c) l += lsum[c];
      a.tile_loss[tile] = l;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Tile kernel for wide models (H = 64, 128): the four waves of a workgroup split every weight
// gradient by rows. Each wave runs the forward, rendering, adjoint and delta chain of its own
// sub-tile as k_step_tiles does, stages delta_l and h_{l-1} in LDS, and after a workgroup barrier
// computes its quarter of the rows of dW_l (and db_l) over the 128 samples of all four waves, on
// v_mfma_f32_16x16x32_bf16 (BF16) or v_mfma_f32_16x16x4f32 (FP32). A wave thus holds a quarter of
// the weight-gradient accumulators, and the tile needs no cross-wave reduction: the waves' slices
// are disjoint. For H = 128 the weights and their BF16 transposes do not fit in LDS beside the
// staging tiles: they are read from the object's weight image in device memory (the byte layout
// of the LDS staging, staged when the parameters are set and kept current by the optimiser
// kernels), and each wave accumulates its
// gradient slice in the tile's partial in device memory, layer by layer, not in registers.

template <int H, bool BF, int MODE>
__global__ void __launch_bounds__(256, 1) k_step_coop(const StepArgs a_in) {
  static_assert(H == 64 || H == 128, "cooperative tile kernel: H = 64 or 128");
  StepArgs a = a_in;
  read_batch(a);
  constexpr int MT = H / 32;
  constexpr bool TRAIN = (MODE == MODE_TRAIN);
  constexpr bool GW = weights_global(H);
  constexpr bool RMW = GW;          // gradient slices accumulate in the partial
  constexpr LdsLayout L = lds_layout(H, BF, 1);
  constexpr CoopLayout C = coop_layout(H, BF);
  constexpr int RW = H / 4;         // weight-gradient rows of one wave
  constexpr int RB = RW / 16;       // ... in 16-row blocks
  constexpr int NBH = H / 16;       // 16-column blocks of a hidden layer's input
  constexpr int HB = H / 64;        // 16-column blocks of the output layer's dW of one wave
  constexpr int FW = H / 4;         // FP32 output layer: features of one wave
  constexpr int TB = dz_tile_bytes(BF), TT = tr_tile_bytes(H, BF);
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = lane & 31, hf = lane >> 5;
  const int m16 = lane & 15, kg = lane >> 4;
  const int S = a.S;
  const int rpw = kSlots / S;
  const int n_tiles = clamp_tiles(a.tile_start[a.n_objects], a.max_tiles);
  float* Bl = reinterpret_cast<float*>(smem + C.B_off);
  if (tid < 3 * kFeatures) Bl[tid] = a.B[tid];
  unsigned char* const scr0 = smem + C.scratch_off;
  int staged = -1;

  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    int jlo = 0, jhi = a.n_objects;
    while (jhi - jlo > 1) {
      const int mid = (jlo + jhi) >> 1;
      if (a.tile_start[mid] <= tile) jlo = mid; else jhi = mid;
    }
    const int j = jlo;
    // uniform by construction: the weight-image and partial buffer resources live in SGPRs
    const int k = __builtin_amdgcn_readfirstlane(a.object_ids[j]);
    if (k < 0 || k >= a.max_objects || !a.desc[k].registered) {
      if (tid == 0) atomicOr(&a.scaler->device_error, 1);
      continue;
    }
    if (kernel_width(a.desc[k].hidden) != H) continue;
    const int rpt = tile_rays(H, a.rays_per_tile, a.rays_per_tile_wide);
    const RayRange rr = tile_ray_range(a.ray_offsets[j], a.ray_offsets[j + 1], tile - a.tile_start[j],
                                       rpt, a.n_rays);
    const int ray_lo = rr.lo, ray_hi = rr.hi;
    const unsigned char* wb = smem;
    if constexpr (GW) {
      wb = a.wimage + (size_t)k * a.wimage_stride;
    } else if (k != staged) {
      __syncthreads();
      stage_weights<H, BF>(a.theta + (size_t)k * a.p_stride, smem, tid, blockDim.x);
      staged = k;
    }
    __syncthreads();
    const double cx = a.desc[k].centre[0], cy = a.desc[k].centre[1], cz = a.desc[k].centre[2];
    const double inv_s = a.desc[k].inv_scale;
    float wseed = 1.0f;
    if constexpr (TRAIN) {
      if (a.dloss) wseed = a.dloss[j];
      if (a.use_scale) wseed *= a.scaler->scale;
    }
    const float inv = (TRAIN && a.use_scale) ? 1.0f / a.scaler->scale : 1.0f;
    float* dst = a.partial + (size_t)tile * a.p_stride;
    // the tile's partial as a buffer: lane offsets in one VGPR, block offsets as constants
    const __amdgpu_buffer_rsrc_t prs =
        __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, n_params_of(H) * 4, 0x00020000);

    f32x4 accW[RMW ? 1 : kLayers][RB][NBH];  // this wave's rows of dW_l (16x16 blocks)
    float accDb[kLayers][RB];                // lane sums of this wave's rows of db_l
    f32x4 accWh[HB];                         // BF16: this wave's columns of the output layer's dW
    float accH[kOut];                        // FP32: the same, one feature per lane group
    float accDbH[kOut];
    if constexpr (TRAIN) {
      if constexpr (!RMW) {
#pragma unroll
        for (int l = 0; l < kLayers; ++l)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NBH; ++cb)
#pragma unroll
              for (int i = 0; i < 4; ++i) accW[l][rb][cb][i] = 0.f;
      }
#pragma unroll
      for (int l = 0; l < kLayers; ++l)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) accDb[l][rb] = 0.f;
#pragma unroll
      for (int bb = 0; bb < HB; ++bb)
#pragma unroll
        for (int i = 0; i < 4; ++i) accWh[bb][i] = 0.f;
#pragma unroll
      for (int c = 0; c < kOut; ++c) { accH[c] = 0.f; accDbH[c] = 0.f; }
    }
    float wave_loss = 0.f;
    int bad = 0;

    unsigned char* dzt = scr0 + wave * C.scratch_wave;
    unsigned char* dtile = dzt + TB;
    unsigned char* htile = dtile + TT;
    const int nrays = ray_hi - ray_lo;
    const int nsub = (nrays + rpw - 1) / rpw;
    const int rounds = (nsub + 3) / 4;

    // Every wave runs every round (a wave without a sub-tile carries zero seeds), since the
    // weight-gradient products of a round read all four waves' staging tiles.
    for (int rd = 0; rd < rounds; ++rd) {
      asm volatile("" ::: "memory");
      const int sub = rd * 4 + wave;
      const int r0 = ray_lo + sub * rpw;
      const int nr = (sub < nsub) ? min(rpw, ray_hi - r0) : 0;
      const int nslots = nr * S;
      const RenderIn rin = render_inputs<TRAIN>(a, r0, nslots);  // in flight during the forward

      // the lane's sample: normalised point and (integrated encoding) normalised variance
      auto point = [&](int p, float xt[4]) {
        const int slot = 32 * p + n;
        xt[0] = xt[1] = xt[2] = xt[3] = 0.f;
        if (slot < nslots) {
          const int ray = r0 + slot / S;
          const double tt = (double)a.t[(size_t)r0 * S + slot];
          const float* o3 = a.rays_o + 3 * (size_t)ray;
          const float* d3 = a.rays_d + 3 * (size_t)ray;
          xt[0] = (float)(((double)o3[0] + tt * (double)d3[0] - cx) * inv_s);
          xt[1] = (float)(((double)o3[1] + tt * (double)d3[1] - cy) * inv_s);
          xt[2] = (float)(((double)o3[2] + tt * (double)d3[2] - cz) * inv_s);
          if (a.var) xt[3] = (float)((double)a.var[(size_t)r0 * S + slot] * inv_s * inv_s);
        }
      };
      float zs[kOut] = {0.f, 0.f, 0.f, 0.f};
      if (nslots > 0) {
#pragma unroll 1
        for (int p = 0; p < 2; ++p) {
          Acts<H, BF> tmp;
          float xt[4], z[kOut];
          point(p, xt);
          forward_pass<H, BF, true>(xt, wb, Bl, tmp, z, a.var != nullptr);
#pragma unroll
          for (int c = 0; c < kOut; ++c) zs[c] = (hf == p) ? z[c] : zs[c];
        }
      }
      float dzs[kOut];
      render_subtile<TRAIN>(a, r0, nslots, wseed, rin, zs, dzs, wave_loss);
      if constexpr (!TRAIN) continue;
#pragma unroll
      for (int c = 0; c < kOut; ++c) accDbH[c] += dzs[c];

#pragma unroll 1
      for (int p = 0; p < 2; ++p) {
        const bool first = (rd == 0 && p == 0), last = (rd == rounds - 1 && p == 1);
        Acts<H, BF> act;
        {
          float xt[4], z[kOut];
          point(p, xt);
          forward_pass<H, BF, false>(xt, wb, Bl, act, z, a.var != nullptr);
        }
        float dz[kOut];
#pragma unroll
        for (int c = 0; c < kOut; ++c) dz[c] = __shfl(dzs[c], 32 * p + n);
        __syncthreads();  // every wave is done reading the staging tiles
        if (hf == 0) {
#pragma unroll
          for (int c = 0; c < kOut; ++c) {
            if constexpr (BF) reinterpret_cast<__bf16*>(dzt)[c * 40 + n] = (__bf16)dz[c];
            else reinterpret_cast<float*>(dzt)[n * kOut + c] = dz[c];
          }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int f = mt * 32 + rowof(r, hf);
            if constexpr (BF)
              reinterpret_cast<__bf16*>(htile)[f * 40 + n] = act.v[kLayers][mt][r >> 3][r & 7];
            else
              reinterpret_cast<float*>(htile)[n * (H + 4) + f] = act.v[kLayers][mt][r];
          }
        __syncthreads();
        // output layer: this wave's columns of dW over the four waves' samples
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2) {
          const unsigned char* dz2 = scr0 + w2 * C.scratch_wave;
          const unsigned char* h2 = dz2 + TB + TT;
          if constexpr (BF) {
            bf16x8 da = {};
            if (m16 < kOut)
              da = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const __bf16*>(dz2) + m16 * 40 + 8 * kg);
#pragma unroll
            for (int bb = 0; bb < HB; ++bb) {
              const int b = wave * HB + bb;
              const bf16x8 hb = *reinterpret_cast<const bf16x8*>(
                  reinterpret_cast<const __bf16*>(h2) + (b * 16 + m16) * 40 + 8 * kg);
              accWh[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(da, hb, accWh[bb], 0, 0, 0);
            }
          } else {
            constexpr int G = 64 / FW, SG = 32 / G;
            const int f = wave * FW + (lane % FW), g = lane / FW;
#pragma unroll
            for (int s2 = 0; s2 < SG; ++s2) {
              const int s = g * SG + s2;
              const float hv = reinterpret_cast<const float*>(h2)[s * (H + 4) + f];
#pragma unroll
              for (int c = 0; c < kOut; ++c) accH[c] += reinterpret_cast<const float*>(dz2)[s * kOut + c] * hv;
            }
          }
        }
        // delta of the last hidden layer, own samples: (W_out^T dz) masked by ReLU'
        Deltas<H, BF> dl;
        if constexpr (BF) {
          bf16x8 dzb = {};
          if (hf == 0) {
#pragma unroll
            for (int c = 0; c < kOut; ++c) dzb[c] = (__bf16)dz[c];
          }
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            bf16x8 wa = {};
            if constexpr (GW) {
              const uint2 w4 = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(
                  image_rsrc(wb, image_bytes(H, BF)), n * kOut * 2, L.whtb_off + mt * 32 * kOut * 2, 0));
              if (hf == 0) {
                wa[0] = __builtin_bit_cast(__bf16, (unsigned short)(w4.x & 0xffff));
                wa[1] = __builtin_bit_cast(__bf16, (unsigned short)(w4.x >> 16));
                wa[2] = __builtin_bit_cast(__bf16, (unsigned short)(w4.y & 0xffff));
                wa[3] = __builtin_bit_cast(__bf16, (unsigned short)(w4.y >> 16));
              }
            } else if (hf == 0) {
              const __bf16* wt = reinterpret_cast<const __bf16*>(wb + L.whtb_off) + (mt * 32 + n) * kOut;
#pragma unroll
              for (int c = 0; c < kOut; ++c) wa[c] = wt[c];
            }
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.f;
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, dzb, acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const float hv = (float)reinterpret_cast<const __bf16*>(htile)[(mt * 32 + rowof(r, hf)) * 40 + n];
              dl.set(mt, r, (hv > 0.f) ? acc[r] : 0.f);
            }
          }
        } else {
          const float* Wh = reinterpret_cast<const float*>(wb + L.wh_off);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              float s = 0.f;
#pragma unroll
              for (int c = 0; c < kOut; ++c) s += Wh[c * (H + 4) + mt * 32 + 16 * hf + r] * dz[c];
              const float hv = reinterpret_cast<const float*>(htile)[n * (H + 4) + mt * 32 + rowof(r, hf)];
              dl.set(mt, r, (hv > 0.f) ? s : 0.f);
            }
        }
#pragma unroll
        for (int l = kLayers - 1; l >= 0; --l) {
          const int K = (l == 0) ? kEnc : H;
          const int KB = K / 32, NB = K / 16;
          const int off = layer_param_off(H, l);
          __syncthreads();  // every wave is done reading the staging tiles
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int f = mt * 32 + rowof(r, hf);
              if constexpr (BF) reinterpret_cast<__bf16*>(dtile)[f * 40 + n] = dl.v[mt][r >> 3][r & 7];
              else reinterpret_cast<float*>(dtile)[n * (H + 4) + f] = dl.v[mt][r];
            }
#pragma unroll
          for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int f = kb * 32 + rowof(r, hf);
              if constexpr (BF)
                reinterpret_cast<__bf16*>(htile)[f * 40 + n] = act.v[l][kb][r >> 3][r & 7];
              else
                reinterpret_cast<float*>(htile)[n * (H + 4) + f] = act.v[l][kb][r];
            }
          // this wave's rows of dW_l: D lane holds row 16 rb + 4 kg + i, column 16 cb + m16
          f32x4 acc[RB][NBH];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NBH; ++cb) {
              if (cb >= NB) continue;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                if constexpr (RMW) {
                  // row wave RW + 16 rb + 4 kg + i, column 16 cb + m16
                  const int lo = ((wave * RW + 4 * kg) * K + m16) * 4;
                  const int co = (off + (rb * 16 + i) * K + cb * 16) * 4;
                  acc[rb][cb][i] =
                      first ? 0.f : __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(prs, lo, co, 0));
                } else {
                  acc[rb][cb][i] = accW[RMW ? 0 : l][rb][cb][i];
                }
              }
            }
          __syncthreads();  // every wave's tiles are staged
#pragma unroll
          for (int w2 = 0; w2 < 4; ++w2) {
            const unsigned char* d2 = scr0 + w2 * C.scratch_wave + TB;
            const unsigned char* h2 = d2 + TT;
            if constexpr (BF) {
              bf16x8 da[RB];
#pragma unroll
              for (int rb = 0; rb < RB; ++rb) {
                da[rb] = *reinterpret_cast<const bf16x8*>(
                    reinterpret_cast<const __bf16*>(d2) + (wave * RW + rb * 16 + m16) * 40 + 8 * kg);
                float s = 0.f;
#pragma unroll
                for (int e = 0; e < 8; ++e) s += (float)da[rb][e];
                accDb[l][rb] += s;
              }
#pragma unroll
              for (int cb = 0; cb < NBH; ++cb) {
                if (cb >= NB) continue;
                const bf16x8 hb = *reinterpret_cast<const bf16x8*>(
                    reinterpret_cast<const __bf16*>(h2) + (cb * 16 + m16) * 40 + 8 * kg);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                  acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(da[rb], hb, acc[rb][cb], 0, 0, 0);
              }
            } else {
#pragma unroll
              for (int kk = 0; kk < 8; ++kk) {
                const int s = 4 * kk + kg;
                float da[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                  da[rb] = reinterpret_cast<const float*>(d2)[s * (H + 4) + wave * RW + rb * 16 + m16];
                  accDb[l][rb] += da[rb];
                }
#pragma unroll
                for (int cb = 0; cb < NBH; ++cb) {
                  if (cb >= NB) continue;
                  const float hb = reinterpret_cast<const float*>(h2)[s * (H + 4) + cb * 16 + m16];
#pragma unroll
                  for (int rb = 0; rb < RB; ++rb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(da[rb], hb, acc[rb][cb], 0, 0, 0);
                }
              }
            }
          }
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NBH; ++cb) {
              if (cb >= NB) continue;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                if constexpr (RMW) {
                  const int lo = ((wave * RW + 4 * kg) * K + m16) * 4;
                  const int co = (off + (rb * 16 + i) * K + cb * 16) * 4;
                  float v = acc[rb][cb][i];
                  if (last) {
                    v *= inv;
                    bad |= partial_bad(v);
                  }
                  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), prs, lo, co, 0);
                } else {
                  accW[RMW ? 0 : l][rb][cb][i] = acc[rb][cb][i];
                }
              }
            }
          if (l == 0) break;
          // delta_{l-1} = (W_l^T delta_l) masked by ReLU' of layer l-1, own samples
          const int ws = L.w_stride[l];
          Deltas<H, BF> nd;
#pragma unroll
          for (int mi = 0; mi < MT; ++mi) {
            f32x16 acc2;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc2[r] = 0.f;
            const int col = mi * 32 + colpos(n);
#pragma unroll
            for (int ko = 0; ko < MT; ++ko) {
              if constexpr (BF) {
                const __bf16* Wt = reinterpret_cast<const __bf16*>(wb + L.wt_off[l]) +
                                   (mi * 32 + n) * (H + 8) + ko * 32 + 16 * hf;
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) {
                  bf16x8 wa;
                  if constexpr (GW)
                    wa = img_b128(image_rsrc(wb, image_bytes(H, BF)), (n * (H + 8) + 16 * hf) * 2,
                                  L.wt_off[l] + (mi * 32 * (H + 8) + ko * 32 + 8 * jj) * 2);
                  else
                    wa = *reinterpret_cast<const bf16x8*>(Wt + 8 * jj);
                  acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, dl.v[ko][jj], acc2, 0, 0, 0);
                }
              } else {
                const float* W = reinterpret_cast<const float*>(wb + L.w_off[l]);
#pragma unroll
                for (int qq = 0; qq < 16; ++qq)
                  acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(W[(ko * 32 + rowof(qq, hf)) * ws + col],
                                                              dl.v[ko][qq], acc2, 0, 0, 0);
              }
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              float hv;
              if constexpr (BF) hv = (float)reinterpret_cast<const __bf16*>(htile)[(mi * 32 + rowof(r, hf)) * 40 + n];
              else hv = reinterpret_cast<const float*>(htile)[n * (H + 4) + mi * 32 + rowof(r, hf)];
              nd.set(mi, r, (hv > 0.f) ? acc2[r] : 0.f);
            }
          }
          dl = nd;
        }
      }
    }  // rounds

    // ---------------- tile result: loss and output-layer bias combined in wave order, every
    // wave writes its own gradient slices
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) wave_loss += __shfl_xor(wave_loss, off);
    if constexpr (TRAIN) {
#pragma unroll
      for (int c = 0; c < kOut; ++c) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) accDbH[c] += __shfl_xor(accDbH[c], off);
        if constexpr (!BF) {
#pragma unroll
          for (int off = FW; off < 64; off <<= 1) accH[c] += __shfl_xor(accH[c], off);
        }
      }
#pragma unroll
      for (int l = 0; l < kLayers; ++l)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          accDb[l][rb] += __shfl_xor(accDb[l][rb], 16);
          accDb[l][rb] += __shfl_xor(accDb[l][rb], 32);
        }
    }
    float* lsum = reinterpret_cast<float*>(smem + C.loss_off);
    int* any_bad = reinterpret_cast<int*>(smem + C.loss_off + 20);
    __syncthreads();
    for (int w = 0; w < 4; ++w) {
      if (wave == w && lane == 0) {
        lsum[0] = (w == 0 ? 0.f : lsum[0]) + wave_loss;
        if constexpr (TRAIN) {
#pragma unroll
          for (int c = 0; c < kOut; ++c) lsum[1 + c] = (w == 0 ? 0.f : lsum[1 + c]) + accDbH[c];
          if (w == 0) *any_bad = 0;
        }
      }
      __syncthreads();
    }
    if constexpr (TRAIN) {
      auto put = [&](int idx, float g) {
        g *= inv;
        bad |= partial_bad(g);
        dst[idx] = g;
      };
#pragma unroll
      for (int l = 0; l < kLayers; ++l) {
        const int K = (l == 0) ? kEnc : H;
        const int NB = K / 16;
        const int off = layer_param_off(H, l);
        if constexpr (!RMW) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NBH; ++cb) {
              if (cb >= NB) continue;
#pragma unroll
              for (int i = 0; i < 4; ++i)
                put(off + (wave * RW + rb * 16 + 4 * kg + i) * K + cb * 16 + m16, accW[RMW ? 0 : l][rb][cb][i]);
            }
        }
        if (kg == 0) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) put(off + H * K + wave * RW + rb * 16 + m16, accDb[l][rb]);
        }
      }
      const int offh = layer_param_off(H, kLayers);
      if constexpr (BF) {
        if (lane < 16) {
#pragma unroll
          for (int bb = 0; bb < HB; ++bb)
#pragma unroll
            for (int c = 0; c < kOut; ++c) put(offh + c * H + (wave * HB + bb) * 16 + lane, accWh[bb][c]);
        }
      } else if (lane < FW) {
#pragma unroll
        for (int c = 0; c < kOut; ++c) put(offh + c * H + wave * FW + lane, accH[c]);
      }
      if (wave == 0 && lane < kOut) put(offh + kOut * H + lane, lsum[1 + lane]);
      if (bad) *any_bad = 1;  // every writer stores the same value
      __syncthreads();
      if (tid == 0 && *any_bad) atomicOr(&a.flags[k], 1);
    }
    if (tid == 0) a.tile_loss[tile] = lsum[0];
    __syncthreads();
  }
}

// Weight image of object `single` (width 32, or hidden 128 in BF16) from its parameters, when they
// are set (added, or written through vmap_set_state); the optimiser kernels keep it current after
// that. With single < 0, block (x, j) stages a share of batch object j's image.
template <int H, bool BF>
__global__ void __launch_bounds__(256) k_stage_image(const StepArgs a_in, int single) {
  StepArgs a = a_in;
  read_batch(a);
  int k = single;
  if (single < 0) {
    if ((int)blockIdx.y >= a.n_objects) return;
    k = a.object_ids[blockIdx.y];
  }
  if (k < 0 || k >= a.max_objects || !a.desc[k].registered || kernel_width(a.desc[k].hidden) != H) return;
  unsigned char* dst = (H == 32) ? a.img32 + (size_t)k * img32_bytes(BF)
                                 : a.wimage + (size_t)k * a.wimage_stride;
  stage_weights<H, BF>(a.theta + (size_t)k * a.p_stride, dst, blockIdx.x * blockDim.x + threadIdx.x,
                       gridDim.x * blockDim.x, a.desc[k].hidden);
}

// ---------------------------------------------------------------------------------------------
// Shape query of one object: forward only, 64 points per wave iteration.

template <int H, bool BF>
__global__ void __launch_bounds__(256) k_query(const QueryArgs qa) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr bool GW = weights_global(H);
  constexpr int B_off = GW ? coop_layout(H, BF).B_off : lds_layout(H, BF, 1).B_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int n = lane & 31, hf = lane >> 5;
  float* Bl = reinterpret_cast<float*>(smem + B_off);
  if (tid < 3 * kFeatures) Bl[tid] = qa.B[tid];
  const unsigned char* wb = smem;
  if constexpr (GW) wb = qa.wimage + (size_t)qa.k * qa.wimage_stride;
  else stage_weights<H, BF>(qa.theta + (size_t)qa.k * qa.p_stride, smem, tid, blockDim.x, qa.desc[qa.k].hidden);
  __syncthreads();
  const ObjDesc d = qa.desc[qa.k];
  for (int64_t chunk = (int64_t)blockIdx.x * nw + wave; chunk * kSlots < qa.n; chunk += (int64_t)gridDim.x * nw) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int64_t i = chunk * kSlots + 32 * p + n;
      float xt[4] = {0.f, 0.f, 0.f, 0.f};
      if (i < qa.n) {
#pragma unroll
        for (int c = 0; c < 3; ++c) xt[c] = (float)(((double)qa.pts[3 * i + c] - d.centre[c]) * d.inv_scale);
      }
      Acts<H, BF> act;
      float z[kOut];
      forward_pass<H, BF, true>(xt, wb, Bl, act, z);
      if (i < qa.n && hf == 0) {
        qa.occ[i] = sigm(z[3]);
        if (qa.rgb) {
#pragma unroll
          for (int c = 0; c < 3; ++c) qa.rgb[3 * i + c] = sigm(z[c]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Tile offsets per batch object (exclusive scan of ceil(rays / rays_per_tile)); clears the
// non-finite flags of the batch's objects and records each object's next Adam step count, so
// that the optimiser kernels read it from here while one of their blocks advances the count.
// Checks the ray offsets as step_table does: a batch that fails gets no tiles, and the optimiser
// kernels leave every object unchanged (ScalerState::batch_ok).

__global__ void __launch_bounds__(1024) k_worklist(int n_objects, int n_rays, const int32_t* ids,
                                                   const int32_t* offs, int rpt, int rpt_wide, int rpt_gen,
                                                   int max_objects, const ObjDesc* __restrict__ desc,
                                                   ScalerState* __restrict__ scaler,
                                                   int32_t* __restrict__ tile_start,
                                                   int32_t* __restrict__ flags,
                                                   int32_t* __restrict__ t_next,
                                                   const BatchDev* __restrict__ bd) {
  __shared__ int part[1024];
  if (bd) {
    n_objects = bd->n_objects;
    n_rays = bd->n_rays;
    ids = bd->object_ids;
    offs = bd->ray_offsets;
  }
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (n_objects + nt - 1) / nt;
  const int j0 = min(tid * per, n_objects), j1 = min(j0 + per, n_objects);
  int local = 0, bad = 0;
  // rays per tile of batch object j (by its width; invalid ids take the narrow size)
  auto rpt_of = [&](int j) {
    const int k = ids[j];
    if (k < 0 || k >= max_objects || !desc[k].registered) return rpt;
    const int h = desc[k].hidden;
    return generic_width(h) ? rpt_gen : tile_rays(h, rpt, rpt_wide);
  };
  auto seg_ok = [&](int j, int o0, int o1) { return batch_segment_ok(j, n_objects, o0, o1, n_rays); };
  for (int j = j0; j < j1; ++j) {
    const int o0 = offs[j], o1 = offs[j + 1];
    const bool ok = seg_ok(j, o0, o1);
    bad |= !ok;
    local += ok ? tiles_of(o1 - o0, rpt_of(j)) : 0;
    const int k = ids[j];
    const bool valid = k >= 0 && k < max_objects;
    if (valid) flags[k] = 0;
    // step count after this batch's update, read by the optimiser kernels
    t_next[j] = (valid && desc[k].registered) ? desc[k].step + 1 : 0;
  }
  part[tid] = local;
  const bool any_bad = __syncthreads_or(bad) != 0;
  for (int off = 1; off < nt; off <<= 1) {
    const int v = (tid >= off) ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - local;
  for (int j = j0; j < j1; ++j) {
    tile_start[j] = any_bad ? 0 : run;
    const int o0 = offs[j], o1 = offs[j + 1];
    run += seg_ok(j, o0, o1) ? tiles_of(o1 - o0, rpt_of(j)) : 0;
  }
  if (tid == nt - 1) {
    tile_start[n_objects] = any_bad ? 0 : part[nt - 1];
    scaler->batch_ok = !any_bad;
    if (any_bad) atomicOr(&scaler->device_error, DERR_OFFSETS);
  }
}

__global__ void __launch_bounds__(256) k_reduce(const OptArgs a_in, int want_grad) {
  OptArgs a = a_in;
  read_batch(a);
  const int j = blockIdx.y;
  const int k = a.ids[j];
  const bool valid = obj_valid(a, k) && a.scaler->batch_ok;
  const TileRange tr = clamp_tile_range(a.tile_start[j], a.tile_start[j + 1], a.max_tiles);
  const int t0 = tr.t0, t1 = tr.t1;
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.loss_out) {
    float s = 0.f;
    if (valid)
      for (int t = t0; t < t1; ++t) s += a.tile_loss[t];
    a.loss_out[j] = s;
  }
  if (!want_grad || !valid) return;
  const int P = a.desc[k].n_params;
  bool bad = false;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < a.p_stride) {
    const float g = (p < P) ? tile_sum(a.partial, a.p_stride, t0, t1, padded_index(a.desc[k].hidden, p)) : 0.f;
    bad = !isfinite(g);
    a.grad[(size_t)k * a.p_stride + p] = g;
    if (a.grad_out) a.grad_out[(size_t)j * a.p_stride + p] = g;
  }
  if (bad) atomicOr(&a.flags[k], 1);
}

__global__ void __launch_bounds__(256) k_adam(const OptArgs a_in) {
  OptArgs a = a_in;
  read_batch(a);
  const int j = blockIdx.y;
  if (blockIdx.x == 0 && j == 0) scaler_update(a);
  const int k = a.ids[j];
  if (!a.scaler->batch_ok || !obj_valid(a, k) || a.offs[j + 1] <= a.offs[j] || a.flags[k]) return;
  const int t = a.t_next[j];
  const AdamCoef c = adam_coef(a, t);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < a.desc[k].n_params) {
    const size_t i = (size_t)k * a.p_stride + p;
    float th = a.theta[i], m = a.m[i], v = a.v[i];
    adam_elem(c, a.grad[i], th, m, v);
    a.theta[i] = th;
    a.m[i] = m;
    a.v[i] = v;
    update_image(a, k, a.desc[k].hidden, p, th);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.desc[k].step = t;
}

// Training step: gradient and update in one pass. The tiles report a partial holding an element
// that is not finite or reaches 2^64 in magnitude (partial_bad), so an object none of whose tiles
// reported has a finite summed gradient and its skip is decided, for the whole object, before any
// store; the element test below is a guard that this bound makes unreachable. Every load of a thread depends on at most the batch object's id, ray
// range and tile range, so a workgroup waits for device memory twice (those, then the object's
// data); the validity checks only decide what is stored. Thread 0 works out the Adam
// coefficients while the loads are in flight. The grid has one row of workgroups per batch object
// and a last row whose first workgroup updates the loss scaler (its own chain of loads).
__global__ void __launch_bounds__(256) k_reduce_adam(const OptArgs a_in) {
  OptArgs a = a_in;
  read_batch(a);
  const int j = blockIdx.y;
  if (j == (int)gridDim.y - 1) {
    if (blockIdx.x == 0) scaler_update(a);
    return;
  }
  const int k = a.ids[j];
  const TileRange tr = clamp_tile_range(a.tile_start[j], a.tile_start[j + 1], a.max_tiles);
  const int t0 = tr.t0, t1 = tr.t1;
  const int r0 = a.offs[j], r1 = a.offs[j + 1];
  const int t = a.t_next[j];
  const int batch_ok = a.scaler->batch_ok;
  const bool in_range = k >= 0 && k < a.max_objects;
  const int kc = in_range ? k : 0;  // loads of an id out of range are discarded
  const ObjDesc& d = a.desc[kc];
  const int registered = d.registered, n_params = d.n_params, hidden = d.hidden;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t i = (size_t)kc * a.p_stride + p;
  float th = 0.f, m = 0.f, v = 0.f, g = 0.f;
  if (p < a.p_stride) {
    th = a.theta[i];
    m = a.m[i];
    v = a.v[i];
    // the partials hold the kernel width's layout (hidden 16: padded to 32)
    g = tile_sum(a.partial, a.p_stride, t0, t1, (hidden == 16 && p < n_params) ? padded_index(16, p) : p);
  }
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  float loss = 0.f;
  if (lead && a.loss_out) loss = tile_sum(a.tile_loss, 1, t0, t1, 0);
  __shared__ float sh[2];
  if (threadIdx.x == 0) adam_coef_store(a, t, sh);
  const bool valid = in_range && registered != 0 && batch_ok;
  if (lead && a.loss_out) a.loss_out[j] = valid ? loss : 0.f;
  if (!valid || r1 <= r0) return;
  // the barrier of object_bad also publishes the coefficients
  if (object_bad(a, j, k)) {
    if (a.tile_bad && lead) a.flags[k] = 1;
    return;
  }
  const AdamCoef c = adam_coef_load(a, sh);
  if (p < n_params) {
    a.grad[i] = g;
    if (isfinite(g)) {
      adam_elem(c, g, th, m, v);
      a.theta[i] = th;
      a.m[i] = m;
      a.v[i] = v;
    } else {
      atomicOr(&a.flags[k], 2);  // for the skip count (bit 1: see object_bad)
    }
    update_image<false>(a, k, hidden, p, th);
  }
  if (lead) a.desc[k].step = t;
}

// k_reduce_adam for objects of many parameters: a row of workgroups per batch object (its width
// capped by the launch) walks the object's parameters four at a time per thread, so that the
// object's descriptor, tile range, skip test and Adam coefficients are settled once per workgroup
// rather than once per 256 parameters. Per parameter the same arithmetic in the same order:
// the tiles' partials summed in tile order from zero, then one Adam update.
__global__ void __launch_bounds__(256) k_reduce_adam_wide(const OptArgs a_in) {
  OptArgs a = a_in;
  read_batch(a);
  const int j = blockIdx.y;
  if (j == (int)gridDim.y - 1) {
    if (blockIdx.x == 0) scaler_update(a);
    return;
  }
  const int k = a.ids[j];
  const TileRange tr = clamp_tile_range(a.tile_start[j], a.tile_start[j + 1], a.max_tiles);
  const int t0 = tr.t0, t1 = tr.t1;
  const int r0 = a.offs[j], r1 = a.offs[j + 1];
  const int t = a.t_next[j];
  const int batch_ok = a.scaler->batch_ok;
  const bool in_range = k >= 0 && k < a.max_objects;
  const int kc = in_range ? k : 0;
  const ObjDesc& d = a.desc[kc];
  const int registered = d.registered, n_params = d.n_params, hidden = d.hidden;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  float loss = 0.f;
  if (lead && a.loss_out) loss = tile_sum(a.tile_loss, 1, t0, t1, 0);
  __shared__ float sh[2];
  if (threadIdx.x == 0) adam_coef_store(a, t, sh);
  const bool valid = in_range && registered != 0 && batch_ok;
  if (lead && a.loss_out) a.loss_out[j] = valid ? loss : 0.f;
  if (!valid || r1 <= r0) return;
  if (object_bad(a, j, k)) {
    if (a.tile_bad && lead) a.flags[k] = 1;
    return;
  }
  const AdamCoef c = adam_coef_load(a, sh);
  const size_t base = (size_t)k * a.p_stride;
  // p_stride is a multiple of 4, so p + 3 < p_stride for every p taken
  for (int p = (blockIdx.x * blockDim.x + threadIdx.x) * 4; p < n_params; p += gridDim.x * blockDim.x * 4) {
    const size_t i = base + p;
    const float4 x = *reinterpret_cast<const float4*>(a.theta + i);
    const float4 y = *reinterpret_cast<const float4*>(a.m + i);
    const float4 z = *reinterpret_cast<const float4*>(a.v + i);
    float th[4] = {x.x, x.y, x.z, x.w}, m[4] = {y.x, y.y, y.z, y.w}, v[4] = {z.x, z.y, z.z, z.w};
    float g[4] = {0.f, 0.f, 0.f, 0.f};
    // slot of p in the partials (hidden 16: the width-32 layout, where four parameters p..p+3
    // with p a multiple of 4 stay four consecutive slots)
    const int pq = padded_index(hidden, p);
    for (int tt = t0; tt < t1; tt += 8) {
      float4 q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        q[u] = (tt + u < t1) ? *reinterpret_cast<const float4*>(a.partial + (size_t)(tt + u) * a.p_stride + pq)
                             : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (tt + u < t1) {
          g[0] += q[u].x;
          g[1] += q[u].y;
          g[2] += q[u].z;
          g[3] += q[u].w;
        }
    }
    if (p + 3 < n_params && isfinite(g[0]) && isfinite(g[1]) && isfinite(g[2]) && isfinite(g[3])) {
#pragma unroll
      for (int e = 0; e < 4; ++e) adam_elem(c, g[e], th[e], m[e], v[e]);
      *reinterpret_cast<float4*>(a.grad + i) = make_float4(g[0], g[1], g[2], g[3]);
      *reinterpret_cast<float4*>(a.theta + i) = make_float4(th[0], th[1], th[2], th[3]);
      *reinterpret_cast<float4*>(a.m + i) = make_float4(m[0], m[1], m[2], m[3]);
      *reinterpret_cast<float4*>(a.v + i) = make_float4(v[0], v[1], v[2], v[3]);
      if (a.gimg && keeps_gimg(hidden)) {  // the four BF16 copies in one store (i is a multiple of 4)
        typedef unsigned int u2w __attribute__((ext_vector_type(2)));
        *reinterpret_cast<u2w*>(a.gimg + i) = u2w{pack2(th[0], th[1]), pack2(th[2], th[3])};
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) update_image(a, k, hidden, p + e, th[e]);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (p + e >= n_params) continue;
        a.grad[i + e] = g[e];
        if (isfinite(g[e])) {
          adam_elem(c, g[e], th[e], m[e], v[e]);
          a.theta[i + e] = th[e];
          a.m[i + e] = m[e];
          a.v[i + e] = v[e];
        } else {
          atomicOr(&a.flags[k], 2);
        }
        update_image(a, k, hidden, p + e, th[e]);
      }
    }
  }
  if (lead) a.desc[k].step = t;
}

// ---------------------------------------------------------------------------------------------
// Object initialisation: Xavier-uniform weights from SplitMix64 in counter mode, zero biases,
// zero Adam moments and gradient; also writes the object's descriptor.

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t index) {
  uint64_t z = seed + (index + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct InitBounds {
  double bound[kLayers + 1];
  int w_end[kLayers + 1];
  int b_end[kLayers + 1];
};

__global__ void __launch_bounds__(256) k_init(int k, uint64_t seed, InitBounds ib, ObjDesc d,
                                              ObjDesc* __restrict__ desc, float* __restrict__ theta,
                                              float* __restrict__ mom, float* __restrict__ vel,
                                              float* __restrict__ grad, int p_stride, int P, int use_rng) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) desc[k] = d;
  if (p >= p_stride) return;
  const size_t i = (size_t)k * p_stride + p;
  if (use_rng) {
    float w = 0.f;
    if (p < P) {
      for (int l = 0; l <= kLayers; ++l) {
        if (p < ib.w_end[l]) {  // weight of layer l
          const uint64_t z = splitmix64_at(seed, (uint64_t)p);
          const double u = (double)(z >> 40) * 0x1p-24;
          w = (float)(ib.bound[l] * (2.0 * u - 1.0));
          break;
        }
        if (p < ib.b_end[l]) break;  // bias of layer l: zero
      }
    }
    theta[i] = w;
  } else if (p >= P) {
    theta[i] = 0.f;
  }
  mom[i] = 0.f;
  vel[i] = 0.f;
  grad[i] = 0.f;
}

// ---------------------------------------------------------------------------------------------
// Depth-guided sampling (Sec. 3.3, Eqs. 1 and 2). A group of P lanes (P = S rounded up to a power
// of two) holds one ray: lane i < S draws sample i — stratified in [t_n, t_s] for i < n_strat,
// N(t_s, sigma^2) otherwise — in FP64 from counter-based SplitMix64 uniforms, and the group sorts
// its S values with a bitonic network over lane shuffles (padding lanes carry +inf).

__global__ void __launch_bounds__(256) k_sample(int n_rays, int S, int P, int n_strat,
                                                const float* __restrict__ t_near,
                                                const float* __restrict__ t_far,
                                                const float* __restrict__ depth, float sigma,
                                                uint64_t seed, float* __restrict__ t_out) {
  const int lane = threadIdx.x & 63;
  const int groups_per_wave = kWave / P;
  const int wave_global = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int i = lane & (P - 1);
  const int r = wave_global * groups_per_wave + lane / P;
  float v = INFINITY;
  if (r < n_rays && i < S) {
    const double tn = t_near[r], tf = t_far[r], d = depth[r];
    const double ts = (d > 0.0) ? d : tf;
    const uint64_t idx = ((uint64_t)r * (uint64_t)S + (uint64_t)i) * 2ull;
    const double top0 = (double)(splitmix64_at(seed, idx) >> 40);
    double t;
    if (i < n_strat) {
      t = tn + ((double)i + top0 * 0x1p-24) / (double)n_strat * (ts - tn);
    } else {
      const double top1 = (double)(splitmix64_at(seed, idx + 1ull) >> 40);
      const double z = sqrt(-2.0 * log((top0 + 1.0) * 0x1p-24)) * cos(6.283185307179586477 * top1 * 0x1p-24);
      t = ts + (double)sigma * z;
    }
    v = (float)t;
  }
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const float other = __shfl_xor(v, j);
      const bool ascending = (i & k) == 0;
      const bool lower = (i & j) == 0;
      v = (lower == ascending) ? fminf(v, other) : fmaxf(v, other);
    }
  }
  if (r < n_rays && i < S) t_out[(size_t)r * S + i] = v;
}

hipError_t launch_sample(int n_rays, int S, int n_strat, const float* t_near, const float* t_far,
                         const float* depth, float sigma, uint64_t seed, float* t_out,
                         hipStream_t s) {
  if (n_rays <= 0) return hipSuccess;
  int P = 1;
  while (P < S) P <<= 1;
  const int rays_per_wave = kWave / P;
  const long long waves = (n_rays + rays_per_wave - 1) / rays_per_wave;
  const int blocks = (int)((waves + 3) / 4);
  hipLaunchKernelGGL(k_sample, dim3(blocks), dim3(256), 0, s, n_rays, S, P, n_strat, t_near,
                     t_far, depth, sigma, seed, t_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Scene rendering from object models (Sec. 3.4): ray-box intersection per (ray, object), the
// object renders of the rays that meet each bound, and a per-ray ranking by rendered depth.
// The pairs are laid out as a batch (object-major, rays in image order), which the forward-mode
// tile kernels render through a device batch descriptor; the host never reads the pair count.

// Entry of ray (o, d) into the box c +- s after t_min, and exit; the ray meets the box iff
// t1 > t0. Slab method in FP64 without contraction (the oracle's arithmetic).
__device__ __forceinline__ void scene_slab(const float* o, const float* d, const ObjDesc& od,
                                           double t_min, double& t0, double& t1) {
  const double s = 1.0 / od.inv_scale;
  t0 = -INFINITY;
  t1 = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double lo = __dsub_rn(od.centre[a], s), hi = __dadd_rn(od.centre[a], s);
    const double oa = (double)o[a], da = (double)d[a];
    double near, far;
    if (da == 0.0) {
      const bool inside = oa >= lo && oa <= hi;
      near = inside ? -INFINITY : INFINITY;
      far = inside ? INFINITY : -INFINITY;
    } else {
      const double ta = __ddiv_rn(__dsub_rn(lo, oa), da), tb = __ddiv_rn(__dsub_rn(hi, oa), da);
      near = fmin(ta, tb);
      far = fmax(ta, tb);
    }
    t0 = fmax(t0, near);
    t1 = fmin(t1, far);
  }
  t0 = fmax(t0, t_min);
}

__device__ __forceinline__ bool scene_pair_valid(const SceneArgs& a, int j, int& k) {
  k = a.object_ids[j];
  return k >= 0 && k < a.max_objects && a.desc[k].registered;
}

// Block (x, j): rays [256 x, 256 x + 256) against batch object j; writes the block's hit count.
__global__ void __launch_bounds__(256) k_scene_count(const SceneArgs a) {
  __shared__ int wsum[4];
  const int j = blockIdx.y, r = blockIdx.x * 256 + threadIdx.x;
  int k;
  bool hit = false;
  if (scene_pair_valid(a, j, k) && r < a.n_rays) {
    double t0, t1;
    scene_slab(a.rays_o + 3 * (size_t)r, a.rays_d + 3 * (size_t)r, a.desc[k], a.t_min, t0, t1);
    hit = t1 > t0;
  }
  const unsigned long long m = __ballot(hit);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0)
    a.counts[(size_t)j * gridDim.x + blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// One block: exclusive scan of the counts (object-major), the batch's CSR offsets (clamped to
// the pair capacity) and its device descriptor.
__global__ void __launch_bounds__(1024) k_scene_scan(const SceneArgs a, int nblk) {
  __shared__ int part[1024];
  const int n = a.n_objects * nblk;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int i0 = min(tid * per, n), i1 = min(i0 + per, n);
  int local = 0;
  for (int i = i0; i < i1; ++i) local += a.counts[i];
  part[tid] = local;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    const int v = (tid >= off) ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - local;
  for (int i = i0; i < i1; ++i) {
    const int c = a.counts[i];
    a.counts[i] = run;
    if (i % nblk == 0) a.ray_offsets[i / nblk] = min(run, a.max_pairs);
    run += c;
  }
  if (tid == nt - 1) {
    const int total = part[nt - 1];
    a.ray_offsets[a.n_objects] = min(total, a.max_pairs);
    if (a.n_pairs_out) *a.n_pairs_out = total;
    if (total > a.max_pairs) atomicOr(&a.scaler->device_error, 2);
    // one store of the whole descriptor: every field is written (the scratch holding it is not
    // cleared, and a field left out would be read as garbage); no targets or losses, point samples
    *a.bd = make_batch_dev(a.n_objects, a.S, min(total, a.max_pairs), a.object_ids, a.ray_offsets,
                           a.pair_o, a.pair_d, a.pair_t, nullptr, nullptr, nullptr, nullptr, nullptr);
  }
}

// Block (x, j): the pairs of its rays with batch object j, in ray order: ray, samples at the
// midpoints of S equal parts of [t0, t1] (FP64, rounded once), and the (object, ray) -> pair map.
__global__ void __launch_bounds__(256) k_scene_fill(const SceneArgs a) {
  __shared__ int wsum[4];
  const int j = blockIdx.y, r = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int k;
  bool hit = false;
  double t0 = 0.0, t1 = 0.0;
  if (scene_pair_valid(a, j, k) && r < a.n_rays) {
    scene_slab(a.rays_o + 3 * (size_t)r, a.rays_d + 3 * (size_t)r, a.desc[k], a.t_min, t0, t1);
    hit = t1 > t0;
  }
  const unsigned long long m = __ballot(hit);
  if (lane == 0) wsum[w] = __popcll(m);
  __syncthreads();
  int pos = a.counts[(size_t)j * gridDim.x + blockIdx.x];
  for (int i = 0; i < w; ++i) pos += wsum[i];
  pos += __popcll(m & ((1ull << lane) - 1ull));
  if (r >= a.n_rays) return;
  int p = -1;
  if (hit && pos < a.max_pairs) {
    p = pos;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.pair_o[3 * (size_t)p + c] = a.rays_o[3 * (size_t)r + c];
      a.pair_d[3 * (size_t)p + c] = a.rays_d[3 * (size_t)r + c];
    }
    const double span = __dsub_rn(t1, t0);
    for (int i = 0; i < a.S; ++i) {
      const double frac = __ddiv_rn((double)i + 0.5, (double)a.S);
      a.pair_t[(size_t)p * a.S + i] = (float)__dadd_rn(t0, __dmul_rn(frac, span));
    }
  }
  a.pair_map[(size_t)j * a.n_rays + r] = p;
}

// Per ray: the nearest object (rendered depth) whose rendered occupancy reaches the threshold;
// an equal depth keeps the earlier batch object.
__global__ void __launch_bounds__(256) k_scene_composite(const SceneArgs a) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= a.n_rays) return;
  float best = INFINITY, occ = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
  int id = -1;
  for (int j = 0; j < a.n_objects; ++j) {
    const int p = a.pair_map[(size_t)j * a.n_rays + r];
    if (p < 0) continue;
    const float O = a.pair_occ[p], D = a.pair_depth[p];
    if (O >= a.occ_threshold && D < best) {
      best = D;
      occ = O;
      c0 = a.pair_rgb[3 * (size_t)p];
      c1 = a.pair_rgb[3 * (size_t)p + 1];
      c2 = a.pair_rgb[3 * (size_t)p + 2];
      id = a.object_ids[j];
    }
  }
  a.depth_out[r] = id >= 0 ? best : 0.f;
  if (a.rgb_out) {
    a.rgb_out[3 * (size_t)r] = c0;
    a.rgb_out[3 * (size_t)r + 1] = c1;
    a.rgb_out[3 * (size_t)r + 2] = c2;
  }
  if (a.occ_out) a.occ_out[r] = occ;
  if (a.id_out) a.id_out[r] = id;
}

hipError_t launch_scene(int phase, const SceneArgs& a, hipStream_t s) {
  if (a.n_rays <= 0 || a.n_objects <= 0) return hipSuccess;
  const int nblk = (a.n_rays + 255) / 256;
  switch (phase) {
    case 0:
      hipLaunchKernelGGL(k_scene_count, dim3(nblk, a.n_objects), dim3(256), 0, s, a);
      hipLaunchKernelGGL(k_scene_scan, dim3(1), dim3(1024), 0, s, a, nblk);
      hipLaunchKernelGGL(k_scene_fill, dim3(nblk, a.n_objects), dim3(256), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL(k_scene_composite, dim3(nblk), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

// Debug validation of a batch (contexts created with VMAP_DEBUG=1), before its step: workgroup 0
// checks that no object id appears twice (an id's mark takes the batch index of each occurrence in
// turn; a mark that was not cleared names a repeat), the others that every ray's sample depths
// ascend. Findings go to the sticky device error bits; the step itself is not changed.
__global__ void __launch_bounds__(256) k_debug_batch(const StepArgs a_in, int32_t* __restrict__ mark) {
  StepArgs a = a_in;
  read_batch(a);
  if (blockIdx.x == 0) {
    for (int j = threadIdx.x; j < a.n_objects; j += blockDim.x) {
      const int k = a.object_ids[j];
      if (k >= 0 && k < a.max_objects) mark[k] = -1;
    }
    __syncthreads();
    int dup = 0;
    for (int j = threadIdx.x; j < a.n_objects; j += blockDim.x) {
      const int k = a.object_ids[j];
      if (k >= 0 && k < a.max_objects) dup |= atomicExch(&mark[k], j) != -1;
    }
    if (__syncthreads_or(dup) && threadIdx.x == 0) atomicOr(&a.scaler->device_error, DERR_DUP_ID);
    return;
  }
  const int S = a.S;
  int bad = 0;
  for (int r = (blockIdx.x - 1) * blockDim.x + threadIdx.x; r < a.n_rays; r += (gridDim.x - 1) * blockDim.x) {
    const float* tr = a.t + (size_t)r * S;
    for (int i = 0; i + 1 < S; ++i) bad |= !(tr[i] <= tr[i + 1]);
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&a.scaler->device_error, DERR_T_ORDER);
}

hipError_t launch_debug_batch(const StepArgs& a, int32_t* mark, hipStream_t s) {
  const int blocks = 1 + std::max(1, std::min(1024, (a.n_rays + 255) / 256));
  hipLaunchKernelGGL(k_debug_batch, dim3(blocks), dim3(256), 0, s, a, mark);
  return hipGetLastError();
}

__global__ void k_fill_zero(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void k_init_scaler(ScalerState* sc, float scale) {
  if (threadIdx.x == 0) {
    sc->scale = scale;
    sc->good_steps = 0;
    sc->skipped = 0;
    sc->device_error = 0;
  }
}

// ---------------------------------------------------------------------------------------------
// Launchers.

// Raise a kernel's dynamic-LDS limit to what a launch needs (once per size increase). Asking for
// the whole 160 KB fails when the kernel also holds static LDS.
static hipError_t allow_lds(const void* fn, int bytes, int* allowed) {
  if (bytes <= *allowed || bytes <= 64 * 1024) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) *allowed = bytes;
  return e;
}

template <int H, bool BF, int MODE>
static hipError_t launch_tiles_t(const StepArgs& a_in, int nwaves, int grid, hipStream_t s) {
  static int allowed = 0;
  StepArgs a = a_in;
  const void* fn;
  int bytes;
  if constexpr (H == 32) {
    fn = reinterpret_cast<const void*>(k_step_tiles<H, BF, MODE>);
    bytes = lds_layout(H, BF, nwaves).total;
    if constexpr (MODE == MODE_STEP) {  // the tile table follows the layout
      if (a.n_objects > kTableMaxObjects || !a.tile_bad) return hipErrorInvalidValue;
      a.lds_table = bytes;  // first tiles, ray offsets and object ids
      bytes += 3 * round_up(a.n_objects + 1, 4) * 4;
    }
  } else {
    static_assert(MODE != MODE_STEP, "the in-kernel tile table is built for width 32 only");
    fn = reinterpret_cast<const void*>(k_step_coop<H, BF, MODE>);
    bytes = coop_layout(H, BF).total;
    nwaves = 4;
  }
  hipError_t e = allow_lds(fn, bytes, &allowed);
  if (e != hipSuccess) return e;
  if constexpr (H == 32)
    hipLaunchKernelGGL((k_step_tiles<H, BF, MODE>), dim3(grid), dim3(nwaves * kWave), bytes, s, a);
  else
    hipLaunchKernelGGL((k_step_coop<H, BF, MODE>), dim3(grid), dim3(nwaves * kWave), bytes, s, a);
  return hipGetLastError();
}

int tiles_supported(int H, bool bf16) {
  return H == 16 || H == 32 || H == 64 || (H == 128 && bf16) || (generic_width(H) && bf16);
}

int tile_waves(int H, int requested) { return H == 32 ? requested : 4; }

int tile_lds_bytes(int H, bool bf16, int nwaves) {
  if (generic_width(H)) return kGenLdsBytes;
  return H == 32 ? lds_layout(H, bf16, nwaves).total : coop_layout(H, bf16).total;
}

hipError_t launch_tiles(int H, bool bf16, int mode, const StepArgs& a, int nwaves, int grid,
                        hipStream_t s) {
  if (grid <= 0) return hipSuccess;
#define VMAP_TILES(HH, BB)                                                                     \
  if (H == HH && bf16 == BB) {                                                                 \
    return mode == MODE_TRAIN ? launch_tiles_t<HH, BB, MODE_TRAIN>(a, nwaves, grid, s)        \
                              : launch_tiles_t<HH, BB, MODE_FWD>(a, nwaves, grid, s);         \
  }
  if (mode == MODE_STEP) {
    if (H != 32) return hipErrorInvalidValue;
    return bf16 ? launch_tiles_t<32, true, MODE_STEP>(a, nwaves, grid, s)
                : launch_tiles_t<32, false, MODE_STEP>(a, nwaves, grid, s);
  }
  VMAP_TILES(32, false)
  VMAP_TILES(32, true)
  VMAP_TILES(64, false)
  VMAP_TILES(64, true)
  VMAP_TILES(128, true)
#undef VMAP_TILES
  return hipErrorInvalidValue;
}

hipError_t launch_stage_images(int H, bool bf16, const StepArgs& a, int single, hipStream_t s) {
  if (!weights_global(H)) return hipSuccess;
  if (H != 128 || !bf16 || !a.wimage) return hipErrorInvalidValue;
  const int ny = single >= 0 ? 1 : a.n_objects;
  if (ny <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_stage_image<128, true>), dim3(16, ny), dim3(256), 0, s, a, single);
  return hipGetLastError();
}

hipError_t launch_stage_image32(bool bf16, const StepArgs& a, int k, hipStream_t s) {
  if (!a.img32 || k < 0) return hipErrorInvalidValue;
  if (bf16) hipLaunchKernelGGL((k_stage_image<32, true>), dim3(8), dim3(256), 0, s, a, k);
  else hipLaunchKernelGGL((k_stage_image<32, false>), dim3(8), dim3(256), 0, s, a, k);
  return hipGetLastError();
}

template <int H, bool BF>
static hipError_t launch_query_t(const QueryArgs& q, hipStream_t s) {
  static int allowed = 0;
  auto fn = k_query<H, BF>;
  const int bytes = weights_global(H) ? coop_layout(H, BF).B_off + 3 * kFeatures * 4
                                      : lds_layout(H, BF, 1).B_off + 3 * kFeatures * 4;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(fn), bytes, &allowed);
  if (e != hipSuccess) return e;
  const int nw = 4;
  int64_t chunks = (q.n + kSlots - 1) / kSlots;
  int grid = (int)std::min<int64_t>((chunks + nw - 1) / nw, 2048);
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(nw * kWave), bytes, s, q);
  return hipGetLastError();
}

hipError_t launch_query(int H, bool bf16, const QueryArgs& q, hipStream_t s) {
  if (H == 32 && !bf16) return launch_query_t<32, false>(q, s);
  if (H == 32 && bf16) return launch_query_t<32, true>(q, s);
  if (H == 64 && !bf16) return launch_query_t<64, false>(q, s);
  if (H == 64 && bf16) return launch_query_t<64, true>(q, s);
  if (H == 128 && bf16) return launch_query_t<128, true>(q, s);
  return hipErrorInvalidValue;
}

hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, s, reinterpret_cast<uint32_t*>(dst), n);
  return hipGetLastError();
}

hipError_t launch_worklist(int n_objects, int n_rays, const int32_t* object_ids,
                           const int32_t* ray_offsets, int rays_per_tile, int rays_per_tile_wide,
                           int rays_per_tile_gen,
                           int max_objects, const ObjDesc* desc, ScalerState* scaler,
                           int32_t* tile_start, int32_t* flags, int32_t* t_next,
                           const BatchDev* bd, hipStream_t s) {
  if (rays_per_tile_gen < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_worklist, dim3(1), dim3(1024), 0, s, n_objects, n_rays, object_ids,
                     ray_offsets, rays_per_tile, rays_per_tile_wide, rays_per_tile_gen, max_objects,
                     desc, scaler, tile_start, flags, t_next, bd);
  return hipGetLastError();
}

// Parameter slots per object from which the optimiser is k_reduce_adam_wide (objects of hidden 128
// and up: whole vectors of theta, m, v and the partials; four parameters per thread measured 5 %
// faster on a step with a hidden-128 object). Below, k_reduce_adam's one parameter per thread keeps
// more workgroups in flight for the few-thousand-parameter objects (four per thread measured 2 %
// slower at hidden 32).
constexpr int kReduceWide = 32768;

hipError_t launch_optimizer(int kind, const OptArgs& a, hipStream_t s) {
  if (a.n_objects <= 0) return hipSuccess;
  const dim3 grid((a.p_stride + 255) / 256, a.n_objects);
  if (kind == OPT_REDUCE) hipLaunchKernelGGL(k_reduce, grid, dim3(256), 0, s, a, 1);
  else if (kind == OPT_LOSS) hipLaunchKernelGGL(k_reduce, dim3(1, a.n_objects), dim3(256), 0, s, a, 0);
  else if (kind == OPT_ADAM) hipLaunchKernelGGL(k_adam, grid, dim3(256), 0, s, a);
  else if (a.p_stride >= kReduceWide && a.p_stride % 4 == 0) {
    // four parameters per thread, about 4096 workgroups over the batch
    const int per_object = std::max(1, std::min((a.p_stride / 4 + 255) / 256, (4096 + a.n_objects - 1) / a.n_objects));
    hipLaunchKernelGGL(k_reduce_adam_wide, dim3(per_object, a.n_objects + 1), dim3(256), 0, s, a);
  } else {
    if (a.wimage) return hipErrorInvalidValue;  // hidden-128 images are kept by the wide kernel
    hipLaunchKernelGGL(k_reduce_adam, dim3(grid.x, a.n_objects + 1), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_init_object(int k, int H, uint64_t seed, const double* bounds,
                              const ObjDesc& d, ObjDesc* desc, float* theta, float* m,
                              float* v, float* grad, int p_stride, int use_rng,
                              hipStream_t s) {
  InitBounds ib{};
  int off = 0;
  for (int l = 0; l <= kLayers; ++l) {
    const int K = (l == 0) ? kEnc : H;
    const int O = (l == kLayers) ? kOut : H;
    ib.bound[l] = bounds[l];
    off += O * K;
    ib.w_end[l] = off;
    off += O;
    ib.b_end[l] = off;
  }
  const int P = off;
  hipLaunchKernelGGL(k_init, dim3((p_stride + 255) / 256), dim3(256), 0, s, k, seed, ib, d, desc,
                     theta, m, v, grad, p_stride, P, use_rng);
  return hipGetLastError();
}

hipError_t launch_init_scaler(ScalerState* sc, float scale, hipStream_t s) {
  hipLaunchKernelGGL(k_init_scaler, dim3(1), dim3(64), 0, s, sc, scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Layered path (widths without a fused tile kernel: hidden 256, 512, 1024; BF16). The step
// of Sec. 3.2-3.3 as a chain of launches over activations kept in device memory: row tiles,
// encoding, one product launch per layer forward, rendering with its adjoint (the fused kernels'
// own render_subtile), then per layer one launch for the weight gradient and one for the input
// gradient. The arithmetic takes the BF16 tile kernels' rounding points: every operand of every
// product is rounded to BF16 (encoding, activations, weights, deltas, the output layer's seed),
// products accumulate in FP32 on v_mfma_f32_32x32x16_bf16; biases, sigmoids, rendering, losses
// and the output layer's bias gradient stay FP32. An object's weight gradient is summed per work
// tile (about kGenWorkRows of its rows) by one workgroup per block of each weight matrix, in an
// order fixed by the object's rows alone, into one partial per work tile that the optimiser adds
// in tile order: the result does not depend on the grid or on the other objects.
//
// Row-tile product kernel (k_gen_gemm): a workgroup (four waves) computes a 64 x 64 block of
// D = A B over one row tile, each wave a 32 x 32 quarter, over K in chunks of 64 staged in LDS as
// BF16. Accumulator element 4 jj + i of lane l holds D[8 jj + 4 (l / 32) + i][l mod 32].
//   forward  (GEN_FWD): rows = samples, n = outputs, k = inputs;   A = h_l,   B = W_l^T
//   input gradient (GEN_DX): rows = samples, n = inputs, k = outputs;  A = delta, B = W_l
// A is staged as its rows lie (k contiguous) and read as one 16-byte LDS read per lane; B is the
// rows of W from the BF16 parameter copy, staged as they lie, read directly (forward) or
// transposed (input gradient).
// Weight gradients (k_gen_dw, k_gen_dw_small): rows = outputs, n = inputs, k = samples;
// A = delta^T, B = h_l^T, both staged as the sample rows lie and read transposed.

// Batch object of element t (a row tile, row block or work tile) of a chain given by its exclusive
// scan: the largest j below n_objects with scan[j] <= t (objects without elements have an empty
// range and are passed over; scan[0] = 0 <= t). Searched by the whole wave, 64 ways at a time: the
// lanes read 64 evenly spaced entries of the remaining range together and a ballot keeps the last
// one at or below t, so a lookup waits on ceil(log64 n) loads rather than log2 n dependent ones.
// Every lane of the wave must be active and pass the same t.
__device__ __forceinline__ int gen_object(const int32_t* __restrict__ scan, int n_objects, int t) {
  const int lane = (int)(threadIdx.x & 63);
  int lo = 0, len = n_objects;  // the answer lies in [lo, lo + len), scan[lo] <= t
  while (len > 1) {
    const int step = (len + 63) >> 6;
    const int i = lane * step;
    const bool le = i < len && scan[lo + i] <= t;  // a prefix of the lanes (scan is nondecreasing)
    const int c = __popcll(__ballot(le)) - 1;      // lane 0 always counts
    lo += c * step;
    len = min(step, len - c * step);
  }
  return lo;
}

// Buffer of the deltas at layer m's outputs (m = 0..3): the two buffers alternately (layer m in
// buffer (3 - m) mod 2). A select: indexing the kernel argument's array by a run-time value would
// put the whole argument block in per-lane scratch memory.
__device__ __forceinline__ uint16_t* gen_delta_out(const GenArgs& g, int m) {
  return ((3 - m) & 1) ? g.delta[1] : g.delta[0];
}

struct GenTile {
  int j, k, lo, hi;  // batch object, object id, rays [lo, hi)
};

// Row tile t of the chain, if it exists (t below the clamped tile count).
__device__ __forceinline__ bool gen_tile(const GenArgs& g, const StepArgs& a, int t, GenTile& o) {
  const int total = clamp_tiles(g.gts[a.n_objects], g.max_gen_tiles);
  if (t >= total) return false;
  const int j = gen_object(g.gts, a.n_objects, t);
  const RayRange rr = tile_ray_range(a.ray_offsets[j], a.ray_offsets[j + 1], t - g.gts[j], g.rpw,
                                     a.n_rays);
  o = GenTile{j, a.object_ids[j], rr.lo, rr.hi};
  return true;
}

// Row tiles per batch object, ceil(rays / rpw), 128-row product blocks, ceil(rays S / 128), and
// work tiles, ceil(rays / work_rays) (as the work list counts them), for the objects of width H;
// none for the others or for a batch that failed the offsets check (ScalerState::batch_ok, from
// the work-list launch). gts, gbs and gws: their exclusive scans.
__global__ void __launch_bounds__(1024) k_gen_tiles(const GenArgs g_in) {
  GenArgs g = g_in;
  read_batch(g.a);
  const StepArgs& a = g.a;
  __shared__ int part[3][1024];
  const bool ok = a.scaler->batch_ok != 0;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (a.n_objects + nt - 1) / nt;
  const int j0 = min(tid * per, a.n_objects), j1 = min(j0 + per, a.n_objects);
  auto rays = [&](int j) {
    const int k = a.object_ids[j];
    if (!ok || k < 0 || k >= a.max_objects) return 0;
    if (!a.desc[k].registered || a.desc[k].hidden != g.H) return 0;
    const int nr = a.ray_offsets[j + 1] - a.ray_offsets[j];
    return nr > 0 ? nr : 0;
  };
  auto nblk = [&](int nr) { return (int)(((long long)nr * a.S + kGenBlockRows - 1) / kGenBlockRows); };
  int lt = 0, lb = 0, lw = 0;
  for (int j = j0; j < j1; ++j) {
    const int nr = rays(j);
    lt += tiles_of(nr, g.rpw);
    lb += nblk(nr);
    lw += tiles_of(nr, g.work_rays);
  }
  part[0][tid] = lt;
  part[1][tid] = lb;
  part[2][tid] = lw;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    const int vt = (tid >= off) ? part[0][tid - off] : 0;
    const int vb = (tid >= off) ? part[1][tid - off] : 0;
    const int vw = (tid >= off) ? part[2][tid - off] : 0;
    __syncthreads();
    part[0][tid] += vt;
    part[1][tid] += vb;
    part[2][tid] += vw;
    __syncthreads();
  }
  int rt = part[0][tid] - lt, rb = part[1][tid] - lb, rw = part[2][tid] - lw;
  for (int j = j0; j < j1; ++j) {
    const int nr = rays(j);
    g.gts[j] = rt;
    g.gbs[j] = rb;
    g.gws[j] = rw;
    rt += tiles_of(nr, g.rpw);
    rb += nblk(nr);
    rw += tiles_of(nr, g.work_rays);
  }
  if (tid == nt - 1) {
    g.gts[a.n_objects] = part[0][nt - 1];
    g.gbs[a.n_objects] = part[1][nt - 1];
    g.gws[a.n_objects] = part[2][nt - 1];
  }
}

// Encoding of sample `slot` of row tile tl: normalised point in FP64 rounded once, Gaussian Fourier
// features (and the integrated encoding's attenuation) as in forward_pass, rounded to BF16 in
// pairs: w[0..7] the sines of features (0, 1) .. (14, 15), w[8..15] the cosines.
__device__ __forceinline__ void gen_encode_row(const StepArgs& a, const GenTile& tl, int slot, unsigned int w[16]) {
  const ObjDesc& d = a.desc[tl.k];
  const int S = a.S;
  const int64_t row = (int64_t)tl.lo * S + slot;
  const int ray = tl.lo + slot / S;
  const double tt = (double)a.t[row];
  const float* o3 = a.rays_o + 3 * (size_t)ray;
  const float* d3 = a.rays_d + 3 * (size_t)ray;
  const double inv_s = d.inv_scale;
  float xt[4];
  xt[0] = (float)(((double)o3[0] + tt * (double)d3[0] - d.centre[0]) * inv_s);
  xt[1] = (float)(((double)o3[1] + tt * (double)d3[1] - d.centre[1]) * inv_s);
  xt[2] = (float)(((double)o3[2] + tt * (double)d3[2] - d.centre[2]) * inv_s);
  xt[3] = a.var ? (float)((double)a.var[row] * inv_s * inv_s) : 0.f;
  const float* Bm = a.B;
#pragma unroll
  for (int f = 0; f < kFeatures; f += 2) {
    float sv[2], cv[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int ff = f + u;
      const float phi = xt[0] * Bm[ff] + xt[1] * Bm[kFeatures + ff] + xt[2] * Bm[2 * kFeatures + ff];
      vmap_sincosf(phi, &sv[u], &cv[u]);
      if (a.var) {
        const float nb = Bm[ff] * Bm[ff] + Bm[kFeatures + ff] * Bm[kFeatures + ff] +
                         Bm[2 * kFeatures + ff] * Bm[2 * kFeatures + ff];
        const float att = expf(-0.5f * xt[3] * nb);
        sv[u] *= att;
        cv[u] *= att;
      }
    }
    w[f / 2] = pack2(sv[0], sv[1]);
    w[(kFeatures + f) / 2] = pack2(cv[0], cv[1]);
  }
}

// Encoding of every sample of a row tile (one wave per tile) into layer 0 of the activations.
__global__ void __launch_bounds__(256) k_gen_encode(const GenArgs g_in) {
  GenArgs g = g_in;
  read_batch(g.a);
  const StepArgs& a = g.a;
  const int lane = threadIdx.x & 63, t = blockIdx.x * 4 + (threadIdx.x >> 6);
  GenTile tl;
  if (!gen_tile(g, a, t, tl)) return;
  const int S = a.S, nslots = (tl.hi - tl.lo) * S;
  if (lane >= nslots) return;
  unsigned int w[16];
  gen_encode_row(a, tl, lane, w);
  unsigned int* out = reinterpret_cast<unsigned int*>(g.act + ((int64_t)tl.lo * S + lane) * g.ld);
#pragma unroll
  for (int i = 0; i < 16; ++i) out[i] = w[i];
}

// Lane `lane`'s MFMA operand from a row-major BF16 tile T (pitch P elements, a multiple of 4): the
// operand's K index runs down the rows kb + 8 (lane / 32) + 0..7 and its row or column index is
// column cb + (lane mod 32). Lanes x, x + 4, x + 8 and x + 12 of each 16-lane group address four
// consecutive rows at the same four-column run, so each ds_read_b64_tr_b16 hands every lane four
// consecutive rows of its own column (the lane mapping the fused kernels' weight gradients use);
// the second read, four rows further down, gives the other four of its eight.
template <int P>
__device__ __forceinline__ bf16x8 tr_operand(const uint16_t* T, int kb, int cb, int lane) {
  typedef __attribute__((address_space(3))) v4i16 lds_v4;
  const uint16_t* p = T + (kb + 8 * (lane >> 5) + ((lane & 15) >> 2)) * P + cb + 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
  const v4i16 x = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4*)(p));
  const v4i16 y = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4*)(p + 4 * P));
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(x, y, 0, 1, 2, 3, 4, 5, 6, 7));
}

// Sum of the eight BF16 of an MFMA operand, two at a time (v_dot2 against ones), added to s.
__device__ __forceinline__ float operand_sum(bf16x8 v, float s) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  const u4 w = __builtin_bit_cast(u4, v);
  const b2 ones = {(__bf16)1.0f, (__bf16)1.0f};
#pragma unroll
  for (int e = 0; e < 4; ++e) s = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(b2, (unsigned int)w[e]), ones, s, false);
  return s;
}

// Rows of product block b of the layered chain: T = 64, row tile b (at most 64 rows, whole rays);
// T = 128, the 128-row block b of the block table (an object's rows in order, cut every 128 rows).
// False if b is past the chain's blocks or holds no row.
template <int T>
__device__ __forceinline__ bool gen_rows(const GenArgs& g, const StepArgs& a, int b, int& k, int64_t& r0, int& nrows) {
  if constexpr (T == 64) {
    GenTile tl;
    if (!gen_tile(g, a, b, tl)) return false;
    k = tl.k;
    r0 = (int64_t)tl.lo * a.S;
    nrows = (tl.hi - tl.lo) * a.S;
  } else {
    static_assert(T == kGenBlockRows, "row blocks of 128");
    const int total = clamp_tiles(g.gbs[a.n_objects], g.max_gen_blocks);
    if (b >= total) return false;
    const int j = gen_object(g.gbs, a.n_objects, b);
    const RayRange rr = tile_ray_range(a.ray_offsets[j], a.ray_offsets[j + 1], 0, kWholeObject, a.n_rays);
    const int64_t first = (int64_t)(b - g.gbs[j]) * T;
    const int64_t rows = (int64_t)(rr.hi - rr.lo) * a.S;
    k = a.object_ids[j];
    r0 = (int64_t)rr.lo * a.S + first;
    nrows = (int)(rows - first < T ? rows - first : T);
  }
  return nrows > 0;  // (a validated batch has no empty block)
}

// Forward and input-gradient products of one row block: a workgroup (four waves, 2 x 2) computes
// a T x T block of D = A B (T = 64 or 128), each wave a T/2 x T/2 quarter as (T/64)^2 32 x 32
// MFMA tiles, over K in chunks of 64. A (h_l, or the deltas at layer l's outputs) is staged as its
// rows lie; B is rows of W from the object's BF16 parameter copy (the optimiser keeps it equal to
// the parameters rounded to nearest even), read directly (forward: W rows are
// the output columns, k contiguous) or transposed (input gradient: W rows are the k index). The
// next chunk's loads are in flight while the current chunk's products run. The 128-row input
// gradient is compiled for three waves per SIMD (164 registers, no spill; it had taken 182 and
// run two), as the forward product already runs.
template <int KIND, int T>
__global__ void __launch_bounds__(256, (KIND == GEN_DX && T == 128) ? 3 : 1) k_gen_gemm(const GenArgs g_in, int l, int ncol_blocks) {
  static_assert(KIND == GEN_FWD || KIND == GEN_DX, "products over one row block");
  static_assert(T == 64 || T == 128, "block sizes");
  GenArgs g = g_in;
  read_batch(g.a);
  const StepArgs& a = g.a;
  constexpr int KC = kGenKChunk, PA = KC + 8;  // K per chunk; pitch of k-contiguous tiles
  constexpr int PT = T + T / 8;                // pitch of the transposed W tile (rows = k)
  constexpr int WT = T / 2, NS = WT / 32;      // wave tile, 32 x 32 MFMA tiles per dimension
  constexpr int NA = T * KC / 8 / 256;         // A pieces (8 BF16) per thread and chunk
  constexpr int NB = T * KC / 8 / 256;         // W pieces (8 BF16) per thread and chunk
  constexpr int PC = T + 8;                    // pitch of the staged result block
  constexpr int kA = T * PA, kB = (KIND == GEN_FWD) ? T * PA : KC * PT;
  static_assert(T * PC <= kA + kB, "the result block fits the operand tiles");
  __shared__ __attribute__((aligned(16))) uint16_t lds[kA + kB];
  uint16_t* As = lds;
  uint16_t* Bs = lds + kA;
  const int H = g.H;
  const bool head = (l == kLayers);
  const int K = (l == 0) ? kEnc : H;  // inputs of layer l
  const int O = head ? kOut : H;      // outputs of layer l
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, m32 = lane & 31, kh = lane >> 5;
  const int64_t ld = g.ld;
  const uint16_t* act_l = g.act + (int64_t)l * g.layer_elems;  // h_l (l = 0: the encoding)
  const uint16_t* dout = head ? nullptr : gen_delta_out(g, l);  // delta at layer l's outputs
  // row block bx, column block by (of ncol_blocks), the row blocks dealt to the XCDs in turn
  int bx, by;
  xcd_unit_block(ncol_blocks, bx, by);
  int k, nrows;
  int64_t r0;
  if (!gen_rows<T>(g, a, bx, k, r0, nrows)) return;
  const int n0 = by * T;
  const float* W = a.theta + (size_t)k * a.p_stride + layer_param_off(H, l);  // [O][K], then b [O]
  const uint16_t* Wb = a.gimg + (size_t)k * a.p_stride + layer_param_off(H, l);  // W in BF16
  const int ktot = (KIND == GEN_FWD) ? K : O;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  // A piece p = tid + 256 q: row p / 8, k columns 8 (p mod 8); ktot is a multiple of 8, or the
  // output layer's 4 seeds (FP32 [rows][4], rounded here)
  u4 va[NA], vw[NB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int p = tid + 256 * q, m = p >> 3, c = (p & 7) * 8;
      va[q] = u4{0u, 0u, 0u, 0u};
      if (m < nrows && k0 + c < ktot) {
        const int64_t row = r0 + m;
        if (KIND == GEN_DX && head) {
          const float4 d4 = *reinterpret_cast<const float4*>(g.dz + row * kOut);
          va[q] = u4{pack2(d4.x, d4.y), pack2(d4.z, d4.w), 0u, 0u};
        } else {
          va[q] = *reinterpret_cast<const u4*>(((KIND == GEN_FWD) ? act_l : dout) + row * ld + k0 + c);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int p = tid + 256 * q;
      vw[q] = u4{0u, 0u, 0u, 0u};
      if constexpr (KIND == GEN_FWD) {  // W rows n0 + n, k0 + c .. + 7 (K is a multiple of 8)
        const int n = p >> 3, c = (p & 7) * 8;
        if (n0 + n < O && k0 + c < K) vw[q] = *reinterpret_cast<const u4*>(Wb + (size_t)(n0 + n) * K + k0 + c);
      } else {  // W rows k0 + o, columns n0 + c .. + 7
        const int o = p / (T / 8), c = (p % (T / 8)) * 8;
        if (k0 + o < O && n0 + c < K) vw[q] = *reinterpret_cast<const u4*>(Wb + (size_t)(k0 + o) * K + n0 + c);
      }
    }
  };
  f32x16 acc[NS][NS];
#pragma unroll
  for (int mi = 0; mi < NS; ++mi)
#pragma unroll
    for (int ni = 0; ni < NS; ++ni)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mi][ni][i] = 0.f;
  fetch(0);
  for (int k0 = 0; k0 < ktot; k0 += KC) {
    __syncthreads();  // the previous chunk's operands have been read
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int p = tid + 256 * q;
      *reinterpret_cast<u4*>(As + (p >> 3) * PA + (p & 7) * 8) = va[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int p = tid + 256 * q;
      if constexpr (KIND == GEN_FWD) *reinterpret_cast<u4*>(Bs + (p >> 3) * PA + (p & 7) * 8) = vw[q];
      else *reinterpret_cast<u4*>(Bs + (p / (T / 8)) * PT + (p % (T / 8)) * 8) = vw[q];
    }
    if (k0 + KC < ktot) fetch(k0 + KC);
    __syncthreads();
#pragma unroll
    for (int kc = 0; kc < KC / 16; ++kc) {
      bf16x8 av[NS], bv[NS];
#pragma unroll
      for (int mi = 0; mi < NS; ++mi)
        av[mi] = *reinterpret_cast<const bf16x8*>(As + (wm * WT + mi * 32 + m32) * PA + kc * 16 + kh * 8);
#pragma unroll
      for (int ni = 0; ni < NS; ++ni) {
        if constexpr (KIND == GEN_FWD)
          bv[ni] = *reinterpret_cast<const bf16x8*>(Bs + (wn * WT + ni * 32 + m32) * PA + kc * 16 + kh * 8);
        else
          bv[ni] = tr_operand<PT>(Bs, 16 * kc, wn * WT + ni * 32, lane);
      }
#pragma unroll
      for (int mi = 0; mi < NS; ++mi)
#pragma unroll
        for (int ni = 0; ni < NS; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[mi], bv[ni], acc[mi][ni], 0, 0, 0);
    }
  }

  // epilogue: element 4 jj + i of a tile is D[row 8 jj + 4 kh + i][column m32] of that tile
  if (KIND == GEN_FWD && head) {  // the output layer's pre-activations, FP32 [rows][4]
#pragma unroll
    for (int ni = 0; ni < NS; ++ni) {
      const int col = n0 + wn * WT + ni * 32 + m32;
      if (col >= O) continue;
      const float b = W[(size_t)O * K + col];
#pragma unroll
      for (int mi = 0; mi < NS; ++mi)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int r = wm * WT + mi * 32 + 8 * (i >> 2) + 4 * kh + (i & 3);
          if (r < nrows) g.z[(r0 + r) * kOut + col] = acc[mi][ni][i] + b;
        }
    }
    return;
  }
  // Hidden outputs (forward: ReLU(D + b); input gradient: D) rounded to BF16 into a T x T block in
  // LDS, then written as rows, 16 bytes at a time; the input gradient multiplies by ReLU' of layer
  // l - 1 (its BF16 output h_l is +0 exactly where the unit is inactive), read as rows too.
  __syncthreads();  // every wave is done with the operand tiles
  uint16_t* Cs = lds;
  const int ncols = (KIND == GEN_FWD) ? O : K;
#pragma unroll
  for (int ni = 0; ni < NS; ++ni) {
    const int cl = wn * WT + ni * 32 + m32;
    float b = 0.f;
    if constexpr (KIND == GEN_FWD) b = (n0 + cl < O) ? W[(size_t)O * K + n0 + cl] : 0.f;
#pragma unroll
    for (int mi = 0; mi < NS; ++mi)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int rl = wm * WT + mi * 32 + 8 * (i >> 2) + 4 * kh + (i & 3);
        float y = acc[mi][ni][i];
        if constexpr (KIND == GEN_FWD) {
          y += b;
          y = (y <= 0.f) ? 0.f : y;  // ReLU (a NaN stays NaN)
        }
        Cs[rl * PC + cl] = (uint16_t)(pack2(y, 0.f) & 0xffffu);
      }
  }
  __syncthreads();
  uint16_t* dst = (KIND == GEN_FWD) ? g.act + (int64_t)(l + 1) * g.layer_elems : gen_delta_out(g, l - 1);
  constexpr int CPR = T / 8;  // 16-byte pieces per row
#pragma unroll
  for (int q = 0; q < T * CPR / 256; ++q) {
    const int p = tid + 256 * q, r = p / CPR, c = (p % CPR) * 8;
    if (r >= nrows || n0 + c >= ncols) continue;  // ncols is a multiple of 8
    u4 v = *reinterpret_cast<const u4*>(Cs + r * PC + c);
    const int64_t off = (r0 + r) * ld + n0 + c;
    if constexpr (KIND == GEN_DX) {
      const u4 h = *reinterpret_cast<const u4*>(act_l + off);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const unsigned int lo = (h[e] & 0xffffu) ? 0xffffu : 0u, hi = (h[e] >> 16) ? 0xffff0000u : 0u;
        v[e] &= lo | hi;
      }
    }
    *reinterpret_cast<u4*>(dst + off) = v;
  }
}

// Work tile w of the layered chain (counted over the chain's objects alone, gws), whose
// weight-gradient partial a workgroup computes: its object's id, its index in the batch's work
// list (tile_start, shared with the other widths) and its rows (g.work_rays rays of one object),
// if w is a work tile of one of the chain's objects with rows (else false).
struct GenObj {
  int k, ts;
  int64_t r0;  // first row
  int nrows;
};
__device__ __forceinline__ bool gen_work_rows(const GenArgs& g, const StepArgs& a, int w, GenObj& o) {
  if (!a.scaler->batch_ok) return false;
  const int total = clamp_tiles(g.gws[a.n_objects], a.max_tiles);
  if (w >= total) return false;
  const int j = gen_object(g.gws, a.n_objects, w);
  const int k = a.object_ids[j];
  if (k < 0 || k >= a.max_objects || !a.desc[k].registered || a.desc[k].hidden != g.H) return false;
  const int i = w - g.gws[j];  // work tile i of object j
  const TileRange tr = clamp_tile_range(a.tile_start[j], a.tile_start[j + 1], a.max_tiles);
  if (i < 0 || tr.t0 + i >= tr.t1) return false;
  const RayRange rr = tile_ray_range(a.ray_offsets[j], a.ray_offsets[j + 1], i, g.work_rays, a.n_rays);
  o = GenObj{k, tr.t0 + i, (int64_t)rr.lo * a.S, (rr.hi - rr.lo) * a.S};
  return o.nrows > 0;
}

// Weight gradient of a hidden layer of more than 32 outputs: dW_l[o][i] = sum over the object's
// rows r of delta_l[r][o] h_l[r][i], and the bias gradient sum_r delta_l[r][o] (the deltas as the
// products see them, BF16). A workgroup computes the T x T block (outputs m0.., inputs n0..) of
// one object (T = 64 or 128), each wave a T/2 x T/2 quarter, over the object's rows in chunks of
// 64 taken in row order. A chunk's rows are staged as they lie in memory (16-byte loads; the next
// chunk's loads are in flight while the current chunk's products run) and the operands are read
// transposed; rows past the object's end are staged as zeros.
template <int T>
__global__ void __launch_bounds__(256) k_gen_dw(const GenArgs g_in, int l, int nblk) {
  static_assert(T == 64 || T == 128, "block sizes");
  GenArgs g = g_in;
  read_batch(g.a);
  const StepArgs& a = g.a;
  constexpr int R = 64, P = T + T / 8;      // rows per chunk; LDS pitch (elements)
  constexpr int WT = T / 2, NS = WT / 32;   // wave tile, 32 x 32 MFMA tiles per dimension
  constexpr int CPR = T / 8;                // 16-byte pieces per staged row
  constexpr int NP = R * CPR / 256;         // pieces per thread and operand
  __shared__ __attribute__((aligned(16))) uint16_t As[R * P];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[R * P];
  const int H = g.H;
  const int K = (l == 0) ? kEnc : H, O = H;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, m32 = lane & 31, kh = lane >> 5;
  // work tile bj, weight block by (of nblk), the work tiles dealt to the XCDs in turn
  int bj, by;
  xcd_unit_block(nblk, bj, by);
  GenObj ob;
  if (l >= kLayers || O <= 32 || !gen_work_rows(g, a, bj, ob)) return;
  const int64_t ld = g.ld;
  const int nrows = ob.nrows;
  const int nbi = (K + T - 1) / T;
  const int m0 = (by / nbi) * T, n0 = (by % nbi) * T;
  // this thread's pieces of a chunk: p = tid + 256 q, row p / CPR, columns 8 (p mod CPR) .. + 7,
  // the same columns in every chunk
  const int c8 = (tid % CPR) * 8;
  const uint16_t* dsrc = gen_delta_out(g, l) + ob.r0 * ld + m0 + c8;
  const uint16_t* hsrc = g.act + (int64_t)l * g.layer_elems + ob.r0 * ld + n0 + c8;
  const bool aok = m0 + c8 < O, bok = n0 + c8 < K;  // O and K are multiples of 8
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 va[NP], vb[NP];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int r = k0 + (tid + 256 * q) / CPR;
      va[q] = u4{0u, 0u, 0u, 0u};
      vb[q] = u4{0u, 0u, 0u, 0u};
      if (r < nrows) {
        if (aok) va[q] = *reinterpret_cast<const u4*>(dsrc + (int64_t)r * ld);
        if (bok) vb[q] = *reinterpret_cast<const u4*>(hsrc + (int64_t)r * ld);
      }
    }
  };
  f32x16 acc[NS][NS];
#pragma unroll
  for (int mi = 0; mi < NS; ++mi)
#pragma unroll
    for (int ni = 0; ni < NS; ++ni)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mi][ni][i] = 0.f;
  // bias gradient (first column block, the waves of its first half): this lane's rows of
  // outputs m0 + wm WT + 32 mi + m32
  const bool bias = (n0 == 0 && wn == 0);
  float db[NS];
#pragma unroll
  for (int mi = 0; mi < NS; ++mi) db[mi] = 0.f;
  fetch(0);
  for (int k0 = 0; k0 < nrows; k0 += R) {
    __syncthreads();  // the previous chunk's operands have been read
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int row = (tid + 256 * q) / CPR;
      *reinterpret_cast<u4*>(As + row * P + c8) = va[q];
      *reinterpret_cast<u4*>(Bs + row * P + c8) = vb[q];
    }
    if (k0 + R < nrows) fetch(k0 + R);
    __syncthreads();
#pragma unroll
    for (int kc = 0; kc < R / 16; ++kc) {
      bf16x8 av[NS], bv[NS];
#pragma unroll
      for (int mi = 0; mi < NS; ++mi) av[mi] = tr_operand<P>(As, 16 * kc, wm * WT + 32 * mi, lane);
#pragma unroll
      for (int ni = 0; ni < NS; ++ni) bv[ni] = tr_operand<P>(Bs, 16 * kc, wn * WT + 32 * ni, lane);
#pragma unroll
      for (int mi = 0; mi < NS; ++mi)
#pragma unroll
        for (int ni = 0; ni < NS; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[mi], bv[ni], acc[mi][ni], 0, 0, 0);
      if (bias) {
#pragma unroll
        for (int mi = 0; mi < NS; ++mi) db[mi] = operand_sum(av[mi], db[mi]);
      }
    }
  }
  const float inv = a.use_scale ? 1.0f / a.scaler->scale : 1.0f;
  float* dst = a.partial + (size_t)ob.ts * a.p_stride + layer_param_off(H, l);
  int bad = 0;
#pragma unroll
  for (int ni = 0; ni < NS; ++ni) {
    const int col = n0 + wn * WT + ni * 32 + m32;
    if (col >= K) continue;
#pragma unroll
    for (int mi = 0; mi < NS; ++mi)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int o = m0 + wm * WT + mi * 32 + 8 * (i >> 2) + 4 * kh + (i & 3);
        if (o >= O) continue;
        const float v = acc[mi][ni][i] * inv;
        bad |= partial_bad(v);
        dst[(size_t)o * K + col] = v;
      }
  }
  if (bias) {
#pragma unroll
    for (int mi = 0; mi < NS; ++mi) {
      const float other = __shfl(db[mi], lane + 32);  // the output's other eight rows of each step
      const int o = m0 + wm * WT + mi * 32 + m32;
      if (kh == 0 && o < O) {
        const float v = (db[mi] + other) * inv;
        bad |= partial_bad(v);
        dst[(size_t)O * K + o] = v;
      }
    }
  }
  if (__syncthreads_or(bad) && tid == 0) atomicOr(&a.flags[ob.k], 1);
}

// Weight gradient of the output layer (4 outputs) of the layered path: a workgroup computes
// outputs [0, 4) x inputs [n0, n0 + 32) over one work tile of an object, and its NW waves take the
// tile's rows in 32-row chunks in turn (chunk c to wave c mod NW), each in its own LDS tiles,
// staged as the rows lie in memory (16-byte loads, the wave's next chunk in flight during the
// current chunk's products) and read transposed: A = the FP32 seeds dz rounded to BF16 (the MFMA
// operand; rows 4..31 of the tile stay zero), B = h_4. The waves' sums are added in wave order,
// so the result does not depend on the grid. Bias gradient: the FP32 seeds unrounded, summed per
// lane over its staged rows and then over lanes and waves in a fixed order. The wave count is
// fixed (kGenDwWaves, not chosen by the size of the launch), so an object's sums do not depend on
// the rest of the batch; eight waves leave a wave an eighth of the work tile's rows and fit two
// workgroups on a CU (registers).
__global__ void __launch_bounds__(kGenDwWaves * 64) k_gen_dw_small(const GenArgs g_in) {
  constexpr int NW = kGenDwWaves;
  GenArgs g = g_in;
  read_batch(g.a);
  constexpr int l = kLayers;
  const StepArgs& a = g.a;
  constexpr int P = kGenPitch;                   // 32 columns + 4 (elements)
  constexpr int kWaveTile = 2 * 32 * P;          // one wave's A and B tiles (uint16 elements)
  constexpr int kRed = NW * 16 * 64 + NW * 32;  // floats of the final sums: accumulators, bias sums
  __shared__ __attribute__((aligned(16))) uint16_t lds[(NW * kWaveTile > 2 * kRed) ? NW * kWaveTile : 2 * kRed];
  const int H = g.H;
  const int K = H;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  GenObj ob;
  if (!gen_work_rows(g, a, blockIdx.x, ob)) return;
  const int64_t ld = g.ld;
  const int nrows = ob.nrows;
  const int n0 = blockIdx.y * 32;
  const bool bias = (n0 == 0);
  uint16_t* As = lds + wave * kWaveTile;
  uint16_t* Bs = As + 32 * P;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  typedef unsigned int u2w __attribute__((ext_vector_type(2)));
  // columns that no piece covers (A's past the 4 outputs) stay zero
  for (int i = lane; i < kWaveTile / 8; i += 64) *reinterpret_cast<u4*>(As + 8 * i) = u4{0u, 0u, 0u, 0u};
  // pieces of a 32-row chunk: B (h_4, columns n0..n0+31): p = lane + 64 q, row p / 4, columns
  // 8 (p mod 4); A (the FP32 seed [rows][4]): lane < 32, row lane. A lane's columns are the same
  // in every chunk.
  const uint16_t* hsrc = g.act + (int64_t)l * g.layer_elems + ob.r0 * ld + n0;
  const float* zsrc = g.dz + ob.r0 * kOut;
  u4 vb[2];
  float4 vz;
  auto fetch = [&](int c) {
    const int rb = c * 32;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = lane + 64 * q, r = rb + (p >> 2), cc = 8 * (p & 3);
      vb[q] = u4{0u, 0u, 0u, 0u};
      if (r < nrows && n0 + cc < K) vb[q] = *reinterpret_cast<const u4*>(hsrc + (int64_t)r * ld + cc);
    }
    vz = make_float4(0.f, 0.f, 0.f, 0.f);
    if (lane < 32 && rb + lane < nrows) vz = *reinterpret_cast<const float4*>(zsrc + (int64_t)(rb + lane) * kOut);
  };
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  float dbv[kOut] = {0.f, 0.f, 0.f, 0.f};  // this lane's bias parts
  if (wave * 32 < nrows) fetch(wave);
  for (int c = wave; c * 32 < nrows; c += NW) {
    wave_lds_sync();  // this wave's previous chunk has been read
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = lane + 64 * q;
      *reinterpret_cast<u4*>(Bs + (p >> 2) * P + 8 * (p & 3)) = vb[q];
    }
    if (lane < 32) {
      *reinterpret_cast<u2w*>(As + lane * P) = u2w{pack2(vz.x, vz.y), pack2(vz.z, vz.w)};
      if (bias) {
        dbv[0] += vz.x;
        dbv[1] += vz.y;
        dbv[2] += vz.z;
        dbv[3] += vz.w;
      }
    }
    if ((c + NW) * 32 < nrows) fetch(c + NW);
    wave_lds_sync();
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const bf16x8 av = tr_operand<P>(As, 16 * kc, 0, lane);
      const bf16x8 bv = tr_operand<P>(Bs, 16 * kc, 0, lane);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
  }
  // bias parts: a butterfly over the wave's lanes (the seeds sit on lanes 0..31, the others hold
  // zeros), leaving the wave's sums on every lane, in a fixed order
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int e = 0; e < kOut; ++e) dbv[e] += __shfl_xor(dbv[e], off);
  }
  __syncthreads();  // every wave is done with its tiles
  float* red = reinterpret_cast<float*>(lds);  // [NW waves][16][64], then [NW waves][32] bias sums
  float* redb = red + NW * 16 * 64;
#pragma unroll
  for (int i = 0; i < 16; ++i) red[(wave * 16 + i) * 64 + lane] = acc[i];
  if (lane == 0) {
#pragma unroll
    for (int e = 0; e < kOut; ++e) redb[wave * 32 + e] = dbv[e];
  }
  __syncthreads();
  // element i of the accumulators (output 8 (i / 4) + 4 (lane / 32) + i mod 4, input n0 + lane mod
  // 32) is summed over the waves in wave order by wave i mod NW; outputs 0..3 are elements 0..3
  // of lanes 0..31
  int bad = 0;
  const float inv = a.use_scale ? 1.0f / a.scaler->scale : 1.0f;
  float* dst = a.partial + (size_t)ob.ts * a.p_stride + layer_param_off(H, l);
  const int col = n0 + (lane & 31);
  for (int i = wave; i < kOut; i += NW) {
    if (lane >= 32 || col >= K) continue;
    float v = red[i * 64 + lane];
    for (int w = 1; w < NW; ++w) v += red[(w * 16 + i) * 64 + lane];
    v *= inv;
    bad |= partial_bad(v);
    dst[(size_t)i * K + col] = v;
  }
  if (bias && wave == 0 && lane < kOut) {
    float v = 0.f;
    for (int w = 0; w < NW; ++w) v += redb[w * 32 + lane];
    v *= inv;
    bad |= partial_bad(v);
    dst[(size_t)kOut * K + lane] = v;
  }
  if (__syncthreads_or(bad) && tid == 0) atomicOr(&a.flags[ob.k], 1);
}

// Rendering, loss and (training) the adjoint of one row tile per wave, by the fused kernels'
// render_subtile; the tile's loss (a fixed-order wave sum) goes to gen_loss, dL/dz to dz.
template <bool TRAIN>
__global__ void __launch_bounds__(256) k_gen_render(const GenArgs g_in) {
  GenArgs g = g_in;
  read_batch(g.a);
  const StepArgs& a = g.a;
  const int lane = threadIdx.x & 63, t = blockIdx.x * 4 + (threadIdx.x >> 6);
  GenTile tl;
  if (!gen_tile(g, a, t, tl)) return;  // uniform over the wave
  const int S = a.S, nslots = (tl.hi - tl.lo) * S;
  const int64_t row0 = (int64_t)tl.lo * S;
  float zs[kOut] = {0.f, 0.f, 0.f, 0.f};
  if (lane < nslots) {
#pragma unroll
    for (int c = 0; c < kOut; ++c) zs[c] = g.z[(row0 + lane) * kOut + c];
  }
  float wseed = 1.0f;
  if constexpr (TRAIN) {
    if (a.dloss) wseed = a.dloss[tl.j];
    if (a.use_scale) wseed *= a.scaler->scale;
  }
  const RenderIn rin = render_inputs<TRAIN>(a, tl.lo, nslots);
  float dzs[kOut] = {0.f, 0.f, 0.f, 0.f};
  float loss = 0.f;
  render_subtile<TRAIN>(a, tl.lo, nslots, wseed, rin, zs, dzs, loss);
  if constexpr (TRAIN) {
    if (lane < nslots) {
#pragma unroll
      for (int c = 0; c < kOut; ++c) g.dz[(row0 + lane) * kOut + c] = dzs[c];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off);
  if (lane == 0) g.gen_loss[t] = loss;
}

// Loss of each object of the chain: its row tiles' losses in order, into its first work tile (its
// other work tiles hold zero, so the optimiser's sum over them is the object's loss).
__global__ void __launch_bounds__(256) k_gen_loss(const GenArgs g_in) {
  GenArgs g = g_in;
  read_batch(g.a);
  const StepArgs& a = g.a;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);  // a wave per batch object
  if (j >= a.n_objects) return;
  const int total = clamp_tiles(g.gts[a.n_objects], g.max_gen_tiles);
  const TileRange tr = clamp_tile_range(g.gts[j], g.gts[j + 1], total);
  const TileRange wr = clamp_tile_range(a.tile_start[j], a.tile_start[j + 1], a.max_tiles);
  if (tr.t1 <= tr.t0 || wr.t1 <= wr.t0) return;
  // the row tiles' losses are read 64 at a time (one per lane) and added one after another in
  // tile order from lane registers: the same sum as a serial loop, without a load per addition
  float s = 0.f;
  for (int t0 = tr.t0; t0 < tr.t1; t0 += 64) {
    const float v = (t0 + lane < tr.t1) ? g.gen_loss[t0 + lane] : 0.f;
    const int n = min(64, tr.t1 - t0);
    for (int i = 0; i < n; ++i) s += __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), i));
  }
  if (lane == 0) a.tile_loss[wr.t0] = s;
  for (int t = wr.t0 + 1 + lane; t < wr.t1; t += 64) a.tile_loss[t] = 0.f;
}

// BF16 copy of object k's parameter slots (round to nearest even), eight per thread.
__global__ void __launch_bounds__(256) k_gen_stage_gimg(const float* __restrict__ theta, uint16_t* __restrict__ gimg,
                                                       int k, int p_stride) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const int p = (blockIdx.x * blockDim.x + threadIdx.x) * 8;  // p_stride is a multiple of 8
  if (p >= p_stride) return;
  const size_t i = (size_t)k * p_stride + p;
  const float4 x0 = *reinterpret_cast<const float4*>(theta + i);
  const float4 x1 = *reinterpret_cast<const float4*>(theta + i + 4);
  *reinterpret_cast<u4*>(gimg + i) = u4{pack2(x0.x, x0.y), pack2(x0.z, x0.w), pack2(x1.x, x1.y), pack2(x1.z, x1.w)};
}

hipError_t launch_stage_gimg(const float* theta, uint16_t* gimg, int k, int p_stride, hipStream_t s) {
  if (!theta || !gimg || k < 0 || p_stride <= 0 || p_stride % 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gen_stage_gimg, dim3((p_stride / 8 + 255) / 256), dim3(256), 0, s, theta, gimg, k, p_stride);
  return hipGetLastError();
}

hipError_t launch_generic(int mode, const GenArgs& g, int tiles_bound, int blocks_bound, int work_bound,
                          hipStream_t s) {
  if (tiles_bound <= 0 || g.a.n_objects <= 0) return hipSuccess;
  if (!generic_width(g.H) || g.a.S < 1 || g.a.S > kSlots || blocks_bound <= 0 || work_bound <= 0 ||
      g.work_rays < 1)
    return hipErrorInvalidValue;
  // the wide products read W from the BF16 parameter copy
  if (keeps_gimg(g.H) && !g.a.gimg) return hipErrorInvalidValue;
  const bool train = (mode == MODE_TRAIN);
  const int H = g.H;
  const int wave_blocks = (tiles_bound + 3) / 4;
  auto blocks = [](int n, int t) { return (n + t - 1) / t; };
  // a product whose output columns number at least 128 takes 128 x 128 blocks over 128-row blocks;
  // narrower ones 64 x 64 blocks over the row tiles
  // one-dimensional grids of 8 ceil(units / 8) x blocks-per-unit workgroups (xcd_unit_block)
  auto grid1 = [&](int units, int nblk) { return dim3((unsigned)(8 * blocks(units, 8) * nblk)); };
  auto fwd_dx = [&](int kind, int ncols, int l) {
    if (ncols >= 128) {
      const int nb = blocks(ncols, 128);
      if (kind == GEN_FWD) hipLaunchKernelGGL((k_gen_gemm<GEN_FWD, 128>), grid1(blocks_bound, nb), dim3(256), 0, s, g, l, nb);
      else hipLaunchKernelGGL((k_gen_gemm<GEN_DX, 128>), grid1(blocks_bound, nb), dim3(256), 0, s, g, l, nb);
    } else {
      const int nb = blocks(ncols, 64);
      if (kind == GEN_FWD) hipLaunchKernelGGL((k_gen_gemm<GEN_FWD, 64>), grid1(tiles_bound, nb), dim3(256), 0, s, g, l, nb);
      else hipLaunchKernelGGL((k_gen_gemm<GEN_DX, 64>), grid1(tiles_bound, nb), dim3(256), 0, s, g, l, nb);
    }
  };
  hipLaunchKernelGGL(k_gen_tiles, dim3(1), dim3(1024), 0, s, g);
  hipLaunchKernelGGL(k_gen_encode, dim3(wave_blocks), dim3(256), 0, s, g);
  for (int l = 0; l <= kLayers; ++l) fwd_dx(GEN_FWD, (l == kLayers) ? kOut : H, l);
  if (train) hipLaunchKernelGGL(k_gen_render<true>, dim3(wave_blocks), dim3(256), 0, s, g);
  else hipLaunchKernelGGL(k_gen_render<false>, dim3(wave_blocks), dim3(256), 0, s, g);
  hipLaunchKernelGGL(k_gen_loss, dim3((g.a.n_objects + 3) / 4), dim3(256), 0, s, g);
  if (train) {
    for (int l = kLayers; l >= 0; --l) {
      const int K = (l == 0) ? kEnc : H, O = (l == kLayers) ? kOut : H;
      if (l == kLayers)
        hipLaunchKernelGGL(k_gen_dw_small, dim3(work_bound, blocks(K, 32)), dim3(kGenDwWaves * 64), 0, s, g);
      else if (O >= 128 && K >= 128) {
        const int nb = blocks(O, 128) * blocks(K, 128);
        hipLaunchKernelGGL(k_gen_dw<128>, grid1(work_bound, nb), dim3(256), 0, s, g, l, nb);
      } else {
        const int nb = blocks(O, 64) * blocks(K, 64);
        hipLaunchKernelGGL(k_gen_dw<64>, grid1(work_bound, nb), dim3(256), 0, s, g, l, nb);
      }
      if (l > 0) fwd_dx(GEN_DX, K, l);
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Scratch of the allocation-free scene render: one array per GPU, held until the process ends,
// shared by every call on that GPU. Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returned for the GPU, looked up once per GPU with that GPU current.
static __device__ __align__(256) unsigned char scratch[kStaticSceneScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device]) return hipSuccess;
  int current = -1;
  hipError_t e = hipGetDevice(&current);
  if (e != hipSuccess) return e;
  if (current != device) return hipErrorInvalidDevice;  // the caller makes `device` current
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  return g_scratch_ptr[device];
}

}  // namespace vmapi
