// Internal types shared by the host library (vmap_api.cpp) and the HIP kernels (vmap_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vmapi {

constexpr int kFeatures = 16;        // Fourier features per sine/cosine half
constexpr int kEnc = 2 * kFeatures;  // encoding width E
constexpr int kOut = 4;              // (r, g, b, occupancy)
constexpr int kLayers = 4;           // hidden ReLU layers
constexpr int kWave = 64;
constexpr int kSlots = 64;           // sample slots per wave sub-tile (two MFMA column blocks)
constexpr int kTableMaxObjects = 2048;  // batch objects MODE_STEP keeps in its LDS tile table

// MODE_STEP: training whose tile kernel builds the tile table itself (no work-list launch).
enum Mode { MODE_FWD = 0, MODE_TRAIN = 1, MODE_STEP = 2 };

// Per-object descriptor in device memory (one slot per possible object id).
struct ObjDesc {
  double centre[3];    // normalisation centre c_k
  double inv_scale;    // 1 / s_k
  int32_t hidden;      // MLP width
  int32_t registered;  // 1 once vmap_add_object ran
  int32_t step;        // Adam step count t_k
  int32_t n_params;    // parameters of this object
};

// Bits of ScalerState::device_error (sticky).
enum DeviceError {
  DERR_OBJECT = 1,    // a batch named an unregistered or out-of-range object id
  DERR_PAIRS = 2,     // a scene render found more (ray, object) pairs than its capacity
  DERR_OFFSETS = 4,   // ray offsets not a CSR over the batch's rays; the batch was not run
  DERR_T_ORDER = 8,   // debug validation: sample depths not ascending within a ray
  DERR_DUP_ID = 16,   // debug validation: an object id appears twice in a batch
};

// Loss scaler and step bookkeeping in device memory.
struct ScalerState {
  float scale;          // dynamic loss scale (1 in FP32 mode)
  int32_t good_steps;   // consecutive steps without a skipped object
  int32_t skipped;      // objects skipped by the last Adam launch
  int32_t device_error; // DeviceError bits
  int32_t batch_ok;     // the last work list's batch passed the offsets check (read by Adam)
  int32_t pad[11];
};

// Device-side checks of a batch's ray offsets. The tile count and every ray index come from
// offsets in device memory, which the host does not read; a batch is run only if every object's
// segment satisfies 0 <= o0 <= o1 <= n_rays and the last offset equals the host's ray count. Then
// the segments tile [0, n_rays) in order and the tile count is at most the workspace's (the host
// checked ceil(n_rays / rays_per_tile) + n_objects against it); the clamps below keep every index
// in bounds regardless.
__host__ __device__ constexpr bool segment_ok(int o0, int o1, int n_rays) {
  return 0 <= o0 && o0 <= o1 && o1 <= n_rays;
}
// Segment [o0, o1) of batch object j of n: inside [0, n_rays], in order, starting the batch at 0
// (j = 0) and ending it at n_rays (j = n - 1). Every object passing means a CSR over n_rays rays.
__host__ __device__ constexpr bool batch_segment_ok(int j, int n_objects, int o0, int o1, int n_rays) {
  return segment_ok(o0, o1, n_rays) && (j != 0 || o0 == 0) && (j != n_objects - 1 || o1 == n_rays);
}
__host__ __device__ constexpr int clamp_tiles(int n_tiles, int max_tiles) {
  return n_tiles < 0 ? 0 : (n_tiles > max_tiles ? max_tiles : n_tiles);
}
// Tile range [t0, t1) of one object, both in [0, n_tiles].
struct TileRange {
  int t0, t1;
};
__host__ __device__ constexpr TileRange clamp_tile_range(int t0, int t1, int n_tiles) {
  const int a = t0 < 0 ? 0 : (t0 > n_tiles ? n_tiles : t0);
  const int b = t1 < a ? a : (t1 > n_tiles ? n_tiles : t1);
  return TileRange{a, b};
}
// Rays [lo, hi) of the tile that is number `tile_in_object` of an object whose segment is
// [o0, o1): both in [0, n_rays] with lo <= hi whatever the inputs (64-bit intermediates).
struct RayRange {
  int lo, hi;
};
__host__ __device__ constexpr RayRange tile_ray_range(int o0, int o1, int tile_in_object, int rpt,
                                                      int n_rays) {
  const long long lo0 = (long long)o0 + (long long)tile_in_object * rpt;
  const long long hi0 = lo0 + rpt < (long long)o1 ? lo0 + rpt : (long long)o1;
  const long long lo = lo0 < 0 ? 0 : (lo0 > n_rays ? n_rays : lo0);
  const long long hi = hi0 < lo ? lo : (hi0 > n_rays ? n_rays : hi0);
  return RayRange{(int)lo, (int)hi};
}
// Tiles of an object of nr rays (0 for an empty or invalid segment).
__host__ __device__ constexpr int tiles_of(int nr, int rpt) { return nr > 0 ? (nr + rpt - 1) / rpt : 0; }

// A tile partial is reported non-finite also when an element's magnitude reaches this bound. An
// object has T < 2^27 tiles and each rounded addition grows a running sum by at most a factor
// (1 + 2^-24), so a sum of partials below 2^64 in magnitude stays below 2^27 * 2^64 * e^8 < 2^103
// and cannot overflow FP32: the skip of an object is decided from its tiles' reports alone,
// before any store.
constexpr float kPartialLimit = 18446744073709551616.0f;  // 2^64
__host__ __device__ inline bool partial_bad(float g) { return !(g > -kPartialLimit && g < kPartialLimit); }

// Byte offsets of the LDS regions of the tile kernel (computed identically on host and device).
struct LdsLayout {
  int w_off[kLayers];   // W_l, rows = H, padded row stride, permuted columns
  int w_stride[kLayers];
  int wt_off[kLayers];  // BF16 only: W_l^T for l >= 1 (rows = inputs), stride H + 8
  int b_off;            // kLayers x H biases (FP32)
  int wh_off;           // head weights [4][H + 4] FP32, permuted columns (FP32 mode)
  int whb_off;          // BF16: head weights [4][H + 8] BF16, permuted columns
  int whtb_off;         // BF16: head weights transposed [H][4] BF16
  int bh_off;           // head biases [4]
  int bA_off;           // BF16: bias operand table [kLayers][H][16] (hi, mid, lo split)
  int B_off;            // encoding matrix [3][16] FP32
  int scratch_off;      // per-wave staging, then the tile's gradient sum
  int scratch_wave;     // bytes per wave
  int loss_off;         // one float
  int total;
};

__host__ __device__ constexpr int round_up(int x, int a) { return (x + a - 1) / a * a; }

__host__ __device__ constexpr int n_params_of(int H) {
  return (H * kEnc + H) + (kLayers - 1) * (H * H + H) + (kOut * H + kOut);
}

// Per-wave staging: the output-layer seeds dz (FP32 [32][4], or BF16 [4][40]) and two transposed
// tiles (delta and activations): FP32 [32 samples][H + 4], BF16 [H features][40].
// dL/dz of a 32-sample pass: BF16 as four output rows of 40 (the output layer's weight-gradient
// operand), then sample-major, four per sample (the output layer's delta operand); FP32
// sample-major.
constexpr int kDzRowsBytes = 4 * 40 * 2;
__host__ __device__ constexpr int dz_tile_bytes(bool bf16) { return bf16 ? kDzRowsBytes + 32 * kOut * 2 : 32 * kOut * 4; }
__host__ __device__ constexpr int tr_tile_bytes(int H, bool bf16) {
  return bf16 ? H * 40 * 2 : 32 * (H + 4) * 4;
}

// BF16 training keeps the encodings of a sub-tile's two 32-sample passes in LDS (BF16, 32 features
// per sample) for the backward's recomputation, which then starts at the first layer.
__host__ __device__ constexpr int enc_cache_bytes(bool bf16) { return bf16 ? 2 * 32 * kEnc * 2 : 0; }

// Every offset except `total` is independent of the wave count, so kernels evaluate the layout at
// compile time (immediate LDS offsets) and only the host needs `total`.
// Copies of the tile's gradient in the width-32 tile kernel's end-of-tile reduction: wave w adds
// into copy w mod copies, and the partial is the copies' sum in order.
__host__ __device__ constexpr int red_copies(int nwaves) { return nwaves >= 8 ? 4 : (nwaves >= 2 ? 2 : 1); }

__host__ __device__ constexpr LdsLayout lds_layout(int H, bool bf16, int nwaves) {
  LdsLayout L{};
  const int es = bf16 ? 2 : 4;
  const int pad = bf16 ? 8 : 4;
  int off = 0;
  for (int l = 0; l < kLayers; ++l) {
    const int K = (l == 0) ? kEnc : H;
    L.w_stride[l] = K + pad;
    L.w_off[l] = off;
    off = round_up(off + H * (K + pad) * es, 16);
  }
  for (int l = 0; l < kLayers; ++l) {
    L.wt_off[l] = off;
    if (bf16 && l > 0) off = round_up(off + H * (H + 8) * 2, 16);
  }
  L.b_off = off;
  off = round_up(off + kLayers * H * 4, 16);
  L.wh_off = off;
  if (!bf16) off = round_up(off + kOut * (H + 4) * 4, 16);
  L.whb_off = off;
  if (bf16) off = round_up(off + kOut * (H + 8) * 2, 16);
  L.whtb_off = off;
  if (bf16) off = round_up(off + H * kOut * 2, 16);
  L.bh_off = off;
  off = round_up(off + kOut * 4, 16);
  L.bA_off = off;
  if (bf16) off = round_up(off + kLayers * H * 32, 16);
  L.B_off = off;
  off = round_up(off + 3 * kFeatures * 4, 16);
  L.loss_off = off;  // the tile's loss per gradient copy (up to 4), then its non-finite flag
  off = round_up(off + 32, 16);
  L.scratch_wave = round_up(dz_tile_bytes(bf16) + 2 * tr_tile_bytes(H, bf16) + enc_cache_bytes(bf16), 16);
  L.scratch_off = off;
  int scratch = nwaves * L.scratch_wave;
  // the tile's gradient at the end: red_copies(nwaves) copies, each summing a fixed set of waves
  const int red = red_copies(nwaves) * round_up(n_params_of(H), 4) * 4;
  if (red > scratch) scratch = red;
  off = round_up(off + scratch, 16);
  L.total = off;
  return L;
}

// Wide models (H >= 128) keep their weights in a per-object image in device memory with the byte
// layout of the LDS staging above (offsets below B_off), since weights and BF16 transposes do not
// fit in LDS next to the cooperative kernel's staging tiles.
__host__ __device__ constexpr bool weights_global(int H) { return H >= 128; }
__host__ __device__ constexpr int image_bytes(int H, bool bf16) {
  return round_up(lds_layout(H, bf16, 1).B_off, 256);
}

// LDS of the cooperative tile kernel (H >= 64): the weights as in lds_layout unless they live in
// the device image, then the encoding matrix, the tile's loss / output-bias sums and a flag, and
// four waves' staging tiles, which the waves read from each other.
struct CoopLayout {
  int B_off;
  int loss_off;     // float loss, float head-bias gradient [4], int non-finite flag
  int scratch_off;
  int scratch_wave;
  int total;
};
__host__ __device__ constexpr CoopLayout coop_layout(int H, bool bf16) {
  CoopLayout C{};
  int off = weights_global(H) ? 0 : lds_layout(H, bf16, 1).B_off;
  C.B_off = off;
  off = round_up(off + 3 * kFeatures * 4, 16);
  C.loss_off = off;
  off = round_up(off + 32, 16);
  C.scratch_wave = round_up(dz_tile_bytes(bf16) + 2 * tr_tile_bytes(H, bf16), 16);
  C.scratch_off = off;
  off += 4 * C.scratch_wave;
  C.total = off;
  return C;
}

// Weight image of a width-32 object: the bytes its LDS staging holds before the encoding matrix
// (lds_layout(32, bf16, 1) up to B_off), kept in device memory so that a tile kernel stages it with
// a plain copy. Written whole when the object's parameters are set, then per parameter by the
// optimiser kernels after each update.
__host__ __device__ constexpr int img32_bytes(bool bf16) { return round_up(lds_layout(32, bf16, 1).B_off, 256); }

// Widths without a fused tile kernel, trained (BF16) by the layered path: a chain of launches
// over activations kept in device memory (encoding, one product launch per layer forward and per
// layer and direction backward, rendering). Its work tiles (one weight-gradient partial each) are
// runs of about kGenWorkRows rows of an object: an object of fewer rows is one work tile.
__host__ __device__ constexpr bool generic_width(int H) {
  return H == 256 || H == 512 || H == 1024;
}

// Width of the fused kernels that run an object of width H: hidden 16 runs in the width-32
// kernels with its weights zero-padded to 32 units (the padded units' pre-activations are exactly
// zero, so they stay inactive, add exact zeros to every sum and get zero gradients), sharing their
// tiles, weight images and partials with the width-32 objects of the stack.
__host__ __device__ constexpr int kernel_width(int H) { return H == 16 ? 32 : H; }

// Slot of parameter p of a width-H object in the parameter layout of its kernel width (the
// layout of the weight images and the tile partials): p itself, except at hidden 16, where
// layer l's weight (o, i) and bias o keep their indices in the width-32 layout. Closed form
// (no loop: the optimiser evaluates it for every parameter): at hidden 16 the first layer's
// weights (32 inputs) keep their index, its 16 biases follow at 1024, each hidden layer's 272
// parameters (16 x 16 weights, 16 biases) land in a 1056-slot block, and the output layer's
// 4 x 16 weights and 4 biases at 4224.
__host__ __device__ constexpr int padded_index(int H, int p) {
  if (H != 16) return p;
  if (p < 16 * kEnc) return p;                           // W_1 [16][32]: rows of 32 either way
  if (p < 16 * kEnc + 16) return 32 * kEnc + (p - 16 * kEnc);  // b_1
  const int h0 = 16 * kEnc + 16, h0_32 = 32 * kEnc + 32;  // first hidden-to-hidden layer
  if (p < h0 + (kLayers - 1) * 272) {
    const int l = (p - h0) / 272, e = (p - h0) - l * 272;
    const int base = h0_32 + l * 1056;
    return e < 256 ? base + (e >> 4) * 32 + (e & 15) : base + 1024 + (e - 256);
  }
  const int o0 = h0 + (kLayers - 1) * 272, o0_32 = h0_32 + (kLayers - 1) * 1056;  // output layer
  if (p < o0 + kOut * 16) return o0_32 + ((p - o0) >> 4) * 32 + ((p - o0) & 15);
  if (p < o0 + kOut * 16 + kOut) return o0_32 + kOut * 32 + (p - o0 - kOut * 16);
  return -1;  // p beyond the object's parameters
}

// Inverse of padded_index at hidden 16: the parameter of a width-16 object held in slot q of the
// width-32 layout, or -1 for a padding slot (zero weight or bias).
__host__ __device__ constexpr int unpadded_index16(int q) {
  constexpr int H2 = 32;
  int off = 0, off2 = 0;
  for (int l = 0; l <= kLayers; ++l) {
    const int K = (l == 0) ? kEnc : 16, O = (l == kLayers) ? kOut : 16;
    const int K2 = (l == 0) ? kEnc : H2, O2 = (l == kLayers) ? kOut : H2;
    if (q < off2 + O2 * K2) {
      const int e = q - off2, o = e / K2, i = e - o * K2;
      return (o < O && i < K) ? off + o * K + i : -1;
    }
    if (q < off2 + O2 * K2 + O2) {
      const int o = q - off2 - O2 * K2;
      return o < O ? off + O * K + o : -1;
    }
    off += O * K + O;
    off2 += O2 * K2 + O2;
  }
  return -1;
}
constexpr int kWholeObject = 1 << 26;  // rays per tile of a layered-path object (max_rays bound)
constexpr int kGenWorkRows = 4096;     // rows (samples) per work tile of a layered-path object

// Rays per work tile of an object of width H.
__host__ __device__ constexpr int tile_rays(int H, int rpt, int rpt_wide) {
  return generic_width(H) ? kWholeObject : (H > 32 ? rpt_wide : rpt);
}

// Offset of layer l's weights in an object's parameter vector (l = kLayers: the output layer).
__host__ __device__ constexpr int layer_param_off(int H, int l) {
  return l == 0 ? 0 : (H * kEnc + H) + (l - 1) * (H * H + H);
}

// A batch's shape and buffers in device memory. Graph replays of the training step read the batch
// from here (refreshed by one small copy per call) instead of from their captured arguments.
struct BatchDev {
  int32_t n_objects;
  int32_t S;
  int32_t n_rays;
  int32_t pad;
  const int32_t* object_ids;
  const int32_t* ray_offsets;
  const float* rays_o;
  const float* rays_d;
  const float* t;
  const float* depth;
  const float* rgb;
  const float* mask;
  float* loss_out;
  const float* var;
};
static_assert(sizeof(BatchDev) == 4 * 4 + 10 * 8, "make_batch_dev must set every field");

// The whole descriptor from its fields, zero-initialised first: every writer (host ring, device
// scene scan) stores it as one value, so no field is left holding a previous batch's bytes.
__host__ __device__ inline BatchDev make_batch_dev(int n_objects, int S, int n_rays,
                                                   const int32_t* object_ids,
                                                   const int32_t* ray_offsets, const float* rays_o,
                                                   const float* rays_d, const float* t,
                                                   const float* depth, const float* rgb,
                                                   const float* mask, float* loss_out,
                                                   const float* var) {
  BatchDev b{};
  b.n_objects = n_objects;
  b.S = S;
  b.n_rays = n_rays;
  b.object_ids = object_ids;
  b.ray_offsets = ray_offsets;
  b.rays_o = rays_o;
  b.rays_d = rays_d;
  b.t = t;
  b.depth = depth;
  b.rgb = rgb;
  b.mask = mask;
  b.loss_out = loss_out;
  b.var = var;
  return b;
}

// Arguments of the gradient / optimiser kernels.
struct OptArgs {
  int n_objects;
  const int32_t* ids;
  const int32_t* offs;        // ray offsets of the batch
  const int32_t* tile_start;
  const float* partial;
  const float* tile_loss;
  const int32_t* t_next;      // per batch object, from k_worklist
  const int32_t* tile_bad;    // [tiles] non-finite partial per tile (MODE_STEP), or NULL: flags
  unsigned char* img32;       // weight images of width-32 objects [max_objects][img32_bytes]
  unsigned char* wimage;      // BF16 weight images of hidden-128 objects [max_objects][stride], or NULL
  int64_t wimage_stride;
  uint16_t* gimg;             // BF16 copies of the parameters of layered-path objects of hidden
                              // 128 or more [max_objects][p_stride], or NULL
  int p_stride;
  int max_objects;
  ObjDesc* desc;
  ScalerState* scaler;
  int32_t* flags;
  float* theta;
  float* m;
  float* v;
  float* grad;
  float* grad_out;
  float* loss_out;
  double lr, beta1, beta2, eps;
  int bf16;
  int growth;
  int max_tiles;              // tiles the workspace holds (bounds every tile range)
  const BatchDev* bd;         // if not NULL, n_objects, ids, offs and loss_out come from here
};

struct StepArgs {
  // batch
  int n_objects;
  int n_rays;            // rays in the batch's arrays (the host's ray count)
  int max_tiles;         // tiles the workspace holds
  int S;
  int rays_per_tile;
  int rays_per_tile_wide;     // tiles of objects wider than 32
  int max_objects;
  const int32_t* object_ids;
  const int32_t* ray_offsets;
  const float* rays_o;
  const float* rays_d;
  const float* t;
  const float* depth;
  const float* rgb;
  const float* mask;
  const float* var;      // [R][S] integrated-encoding variances or NULL
  // model state
  const float* theta;
  int p_stride;
  int hidden;            // width handled by this launch
  const ObjDesc* desc;
  ScalerState* scaler;
  const float* B;        // [3][16]
  // work buffers
  const int32_t* tile_start;  // [n_objects + 1]
  float* partial;             // [tiles][p_stride]
  float* tile_loss;           // [tiles]
  const float* dloss;         // [n_objects] upstream weights (backward) or NULL
  int32_t* flags;             // [max_objects] non-finite partial flags
  float* out_depth;
  float* out_rgb;
  float* out_occ;
  float lambda_c;
  float lambda_o;
  int use_scale;              // multiply seeds by the loss scale (BF16 training)
  const BatchDev* bd;         // if not NULL, the batch fields above are read from here
  unsigned char* wimage;      // weight images of wide objects, [max_objects][wimage_stride]
  int64_t wimage_stride;
  unsigned char* img32;       // weight images of width-32 objects [max_objects][img32_bytes]
  const uint16_t* gimg;       // BF16 copies of layered-path parameters (hidden >= 128), or NULL
  // MODE_STEP only: the tile table (in LDS at byte offset lds_table) is also written to
  // tile_start_out, with the next Adam step counts (t_next) and cleared flags, for the optimiser;
  // tiles report a non-finite partial in tile_bad [tiles].
  int32_t* tile_start_out;
  int32_t* t_next;
  int32_t* tile_bad;
  int lds_table;
};

// The layered path (generic_width objects of one width H per launch chain). Row = sample:
// row r * S + i is sample i of batch ray r. Row tiles are whole rays, floor(64 / S) of them (one
// rendering sub-tile, at most 64 rows), listed per batch object in gts (exclusive scan).
struct GenArgs {
  StepArgs a;            // batch, model state and the fused path's work buffers
  int H;                 // width of this chain's objects
  int rpw;               // rays per row tile
  int max_gen_tiles;     // row tiles the workspace holds
  int32_t* gts;          // [n_objects + 1] first row tile of each batch object
  float* gen_loss;       // [max_gen_tiles] loss per row tile
  uint16_t* act;         // BF16 [kLayers + 1][rows][ld]: encoding (32 wide), then h_1 .. h_4
  uint16_t* delta[2];    // BF16 [rows][ld] each: back-propagated deltas, alternately
  float* z;              // [rows][4] output pre-activations
  float* dz;             // [rows][4] their adjoints (times the seed's scale)
  int64_t ld;            // elements per row of act and delta
  int64_t layer_elems;   // elements per layer of act
  int max_gen_blocks;    // 128-row blocks the block table holds
  int32_t* gbs;          // [n_objects + 1] first 128-row block of each batch object
  int work_rays;         // rays per work tile of this chain's objects (the work list's)
  int32_t* gws;          // [n_objects + 1] first work tile of each batch object among this chain's
                         // work tiles (the chain's objects' tiles, counted alone)
};
// Kinds of the layered path's row-block product kernel (the weight gradients have their own).
enum GenKind { GEN_FWD = 0, GEN_DX = 1 };
// Rows of a block of the wide products (128 x 128 output blocks): an object's rows in order, cut
// every kGenBlockRows rows regardless of ray boundaries (rows are independent in those products).
constexpr int kGenBlockRows = 128;
// LDS of the product kernels: k_gen_gemm and k_gen_dw stage two BF16 operand tiles of up to
// 128 x (kGenKChunk + 8) or kGenKChunk x (128 + 16) elements; k_gen_dw_small (the output layer)
// its kGenDwWaves waves' pairs of 32-row tiles (rows of kGenPitch elements), then the waves' FP32 sums (16
// accumulators per lane and 32 bias sums per wave).
constexpr int kGenKChunk = 64;
constexpr int kGenPitch = 36;
constexpr int kGenDwWaves = 8;
constexpr int kGenTileLds = 2 * 128 * (kGenKChunk + 8) * 2;
constexpr int kGenSmallLds = (kGenDwWaves * 2 * 32 * kGenPitch * 2 > 4 * kGenDwWaves * (16 * 64 + 32))
                                 ? kGenDwWaves * 2 * 32 * kGenPitch * 2
                                 : 4 * kGenDwWaves * (16 * 64 + 32);
constexpr int kGenLdsBytes = kGenTileLds > kGenSmallLds ? kGenTileLds : kGenSmallLds;

struct QueryArgs {
  const float* pts;
  int64_t n;
  int k;
  const float* theta;
  int p_stride;
  const ObjDesc* desc;
  const float* B;
  float* occ;
  float* rgb;
  unsigned char* wimage;      // as in StepArgs (wide objects)
  int64_t wimage_stride;
  int max_objects;
};


// Scene rendering (Sec. 3.4): rays against the bounds of a list of objects.
struct SceneArgs {
  int n_rays;
  int n_objects;
  int S;
  int max_objects;
  int max_pairs;
  float occ_threshold;
  double t_min;
  const float* rays_o;       // [n_rays][3]
  const float* rays_d;
  const int32_t* object_ids; // [n_objects] (device)
  const ObjDesc* desc;
  ScalerState* scaler;
  // scratch
  int32_t* counts;           // [n_objects][blocks] hit counts, then their exclusive scan
  int32_t* ray_offsets;      // [n_objects + 1] pairs per object (CSR)
  int32_t* pair_map;         // [n_objects][n_rays] pair index or -1
  float* pair_o;             // [max_pairs][3]
  float* pair_d;
  float* pair_t;             // [max_pairs][S]
  float* pair_depth;         // [max_pairs] object renders of the pairs
  float* pair_rgb;           // [max_pairs][3]
  float* pair_occ;           // [max_pairs]
  BatchDev* bd;              // the pairs as a batch
  int32_t* n_pairs_out;      // optional: pairs found (device)
  // outputs
  float* depth_out;
  float* rgb_out;
  float* occ_out;
  int32_t* id_out;
};

// Kernel launchers (vmap_kernels.hip). Return hipSuccess or the launch error.
hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t s);
hipError_t launch_worklist(int n_objects, int n_rays, const int32_t* object_ids,
                           const int32_t* ray_offsets, int rays_per_tile, int rays_per_tile_wide,
                           int rays_per_tile_gen,
                           int max_objects, const ObjDesc* desc, ScalerState* scaler,
                           int32_t* tile_start, int32_t* flags, int32_t* t_next,
                           const BatchDev* bd, hipStream_t s);
hipError_t launch_tiles(int H, bool bf16, int mode, const StepArgs& a, int nwaves, int grid,
                        hipStream_t s);
// Debug validation of a batch (distinct ids, ascending sample depths); mark: [max_objects] int32.
hipError_t launch_debug_batch(const StepArgs& a, int32_t* mark, hipStream_t s);
// The layered path's chain for the objects of width g.H of a batch: row tiles, encoding, forward
// products, rendering (and loss), then in training the backward products, writing each object's
// unscaled gradient into its one tile partial and its loss into that tile's loss. tiles_bound:
// host bound on the row tiles (ceil(n_rays / rpw) + n_objects).
hipError_t launch_generic(int mode, const GenArgs& g, int tiles_bound, int blocks_bound, int work_bound,
                          hipStream_t s);
// The BF16 parameter copy of layered-path object k (hidden >= 128) from its parameters.
hipError_t launch_stage_gimg(const float* theta, uint16_t* gimg, int k, int p_stride, hipStream_t s);
// Whether objects of width H keep a BF16 parameter copy (layered path, wide products).
__host__ __device__ constexpr bool keeps_gimg(int H) { return generic_width(H) && H >= 128; }
enum OptKind { OPT_LOSS = 0, OPT_REDUCE = 1, OPT_ADAM = 2, OPT_REDUCE_ADAM = 3 };
hipError_t launch_optimizer(int kind, const OptArgs& a, hipStream_t s);
hipError_t launch_init_object(int k, int H, uint64_t seed, const double* bounds,
                              const ObjDesc& d, ObjDesc* desc, float* theta, float* m,
                              float* v, float* grad, int p_stride, int use_rng,
                              hipStream_t s);
hipError_t launch_query(int H, bool bf16, const QueryArgs& q, hipStream_t s);
hipError_t launch_init_scaler(ScalerState* sc, float scale, hipStream_t s);
hipError_t launch_sample(int n_rays, int S, int n_strat, const float* t_near, const float* t_far,
                         const float* depth, float sigma, uint64_t seed, float* t_out,
                         hipStream_t s);
int tiles_supported(int H, bool bf16);
// The allocation-free scene render's scratch: a static device array per GPU of this many bytes.
constexpr size_t kStaticSceneScratchBytes = (size_t)16 << 20;
// Looks up the array's device address on `device`, which must be current (once per GPU).
hipError_t static_scratch_init(int device);
// The address found by static_scratch_init for `device`, or NULL before it ran.
void* static_scratch(int device);
// phase 0: pairs (count, scan, fill); phase 1: per-ray composite
hipError_t launch_scene(int phase, const SceneArgs& a, hipStream_t s);
int tile_lds_bytes(int H, bool bf16, int nwaves);
int tile_waves(int H, int requested);
// Weight images of wide objects: those of the batch (single < 0) or of object `single`.
hipError_t launch_stage_images(int H, bool bf16, const StepArgs& a, int single, hipStream_t s);
// The weight image of width-32 object k, whole, from its parameters.
hipError_t launch_stage_image32(bool bf16, const StepArgs& a, int k, hipStream_t s);

}  // namespace vmapi
