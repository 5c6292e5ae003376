/*
 * vmap.h - C ABI of the MI355X (gfx950) library for vectorised per-object neural-field training.
 *
 * The library trains K independent tiny MLP occupancy fields ("objects") in one batched step, as
 * in vMAP (Kong, Liu, Taher, Davison; CVPR 2023, arXiv 2302.01838):
 *
 *   - objects appear on the fly and are appended to a stack of models of one design
 *     (Sec. 3.2, "Object Initialisation and Association");
 *   - every object trains only from its own rays and can be stopped or resumed without
 *     interfering with the others (Sec. 3.2, "Object Supervision");
 *   - all objects train together in one vectorised pass (Sec. 3.2, "Vectorised Training");
 *   - a step maps the samples of each ray through the object-level encoding (supplement Sec. B)
 *     and the object's MLP to colour and occupancy, renders occupancy, depth and colour (Eq. 3),
 *     takes the masked L1 losses (Eqs. 4-7), backpropagates and applies Adam per object;
 *   - objects are rendered along rays and queried inside their bounds (Sec. 3.4).
 *
 * Conventions shared by every call:
 *   - Return value: a vmap_status; 0 (VMAP_OK) on success. On any error nothing is enqueued and
 *     no state changes; vmap_last_error() returns a message.
 *   - "Device pointer" means memory of the GPU the context was created on (for example a torch
 *     tensor's data_ptr()). The library never allocates or frees device memory: the caller
 *     provides the state and workspace buffers and every input and output buffer.
 *   - `stream` is a hipStream_t (NULL is the default stream). All work of a call is enqueued on
 *     it and runs asynchronously unless a call says it synchronises. A context is not thread
 *     safe; use one stream per context.
 *   - Floating-point inputs are FP32; integer inputs are int32 unless stated.
 *   - Device-side preconditions are checked by the kernels where cheap: an object id that is
 *     out of range or unregistered is skipped, and a batch whose ray offsets are not a CSR over
 *     its n_rays_total rays is not run; both raise a device error bit reported by
 *     vmap_step_info(). Sorted samples and distinct ids are checked when the context was created
 *     with the environment variable VMAP_DEBUG=1 (report only). No kernel reads or writes past a
 *     buffer whatever the device-side inputs hold.
 */
#ifndef VMAP_H
#define VMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VMAP_OK = 0,
  VMAP_EINVAL = 1,     /* bad argument: NULL pointer, size or value out of range */
  VMAP_ECAPACITY = 2,  /* more objects, rays or bytes than the context was sized for */
  VMAP_EHIP = 3,       /* a HIP runtime call failed (message names it) */
  VMAP_ESTATE = 4,     /* call not valid in the current state (e.g. unregistered object) */
  VMAP_ENOTSUP = 5     /* configuration the library does not support */
} vmap_status;

enum { VMAP_FP32 = 0, VMAP_BF16 = 1 };

/* Which per-object array vmap_get_state / vmap_set_state move. */
enum { VMAP_STATE_PARAMS = 0, VMAP_STATE_ADAM_M = 1, VMAP_STATE_ADAM_V = 2,
       VMAP_STATE_GRAD = 3, VMAP_STATE_STEP = 4, VMAP_STATE_SCALER = 5 };

typedef struct vmap_ctx vmap_ctx; /* opaque; created by vmap_init_objects, freed by vmap_destroy */

/*
 * Model, optimiser and capacity settings (copied by vmap_init_objects).
 *
 * The MLP of an object maps the 2*n_features encoding through n_hidden_layers ReLU layers of
 * width `hidden` to four outputs (r, g, b, occupancy), each through a sigmoid (Sec. 3.3,
 * "Surface and Volume Rendering"). Parameters of one object are stored, in this order,
 * W_1 [H x E], b_1 [H], W_2 [H x H], b_2, ..., W_L, b_L, W_out [4 x H], b_out [4], every W
 * row-major as [out][in]; E = 2 * n_features. Supported: n_features = 16, n_hidden_layers = 4,
 * hidden in {16, 32, 64} in both precisions and 128 in VMAP_BF16 (the background
 * model's width, Sec. 4, Implementation Details), 1 <= max_samples_per_ray <= 64. Objects of
 * different widths may share a stack and a batch (max_hidden bounds them). Width 16 runs in the
 * width-32 kernels with its weights zero-padded to 32 units (exact: the extra units never
 * activate), so its objects share the width-32 objects' launches, and a stack whose max_hidden
 * is 16 is sized as for 32. In VMAP_BF16 the widths 256, 512 and 1024 (with 16, the hidden-size
 * range of Sec. 4.3's vectorised-vs-sequential study) are trained by a layered path (launches
 * per layer and direction, activations in the workspace) with the same rounding points; a stack
 * holds objects of at most one of them, and vmap_query_occupancy does not take them.
 */
typedef struct {
  int32_t max_objects;          /* capacity of the model stack, 1..65536 */
  int32_t n_features;           /* Fourier features per sine/cosine half (16) */
  int32_t hidden;               /* default width H of an object model */
  int32_t n_hidden_layers;      /* L, ReLU layers before the output layer (4) */
  int32_t max_hidden;           /* largest width any object may use; sizes parameter slots */
  int32_t max_samples_per_ray;  /* S bound for batches */
  int32_t max_rays;             /* rays per batch the workspace is sized for */
  int32_t precision;            /* VMAP_FP32, or VMAP_BF16: MLP products on BF16 MFMA */
  int32_t rays_per_tile;        /* rays per work tile; 0 = library default for (H, S) */
  int32_t scale_growth_interval;/* BF16: good steps before the loss scale doubles (2000) */
  int32_t rays_per_tile_wide;   /* rays per work tile of objects wider than 32; 0 = one round
                                 * of the cooperative kernel (4 waves x floor(64 / S) rays) */
  int32_t split_step;           /* 0: when every object has width 32 and a batch has at most
                                 * 2048 objects, the training step's tile kernel builds its work
                                 * list itself (two launches per step: tiles, then gradient sums
                                 * and Adam); 1: always a separate work-list launch first (three).
                                 * Results are bitwise the same either way. */
  double lr;                    /* Adam learning rate (1e-3) */
  double beta1, beta2, eps;     /* Adam moments (0.9, 0.999) and epsilon (1e-8) */
  double lambda_colour;         /* lambda_1 of Eq. 7 (5) */
  double lambda_occ;            /* lambda_2 of Eq. 7 (10) */
  double loss_scale_init;       /* BF16: initial dynamic loss scale (4096), a power of two in
                                 * [2^-125, 2^126]; FP32 ignores it */
} vmap_config;

/* One object to append to the stack (Sec. 3.2). */
typedef struct {
  float centre[3];   /* centre of the object's bound, world frame (metres) */
  float scale;       /* half the largest extent of the bound; points map to (x - centre)/scale */
  int32_t hidden;    /* width of this object's MLP; 0 = config.hidden */
  int32_t reserved;
  uint64_t seed;     /* initialisation seed (Xavier-uniform from SplitMix64) */
} vmap_object_desc;

/*
 * A training / rendering batch: the rays of n_objects objects, segmented CSR-style.
 * Every pointer is a DEVICE pointer owned by the caller and must stay valid until the work
 * enqueued on the stream has finished. Rays are world-frame with unit directions; t holds the
 * S sample depths of each ray in non-decreasing order (depth-guided samples, Sec. 3.3, Eqs. 1-2).
 */
typedef struct {
  int32_t n_objects;          /* objects in this batch (>= 0); zero-ray objects are allowed */
  int32_t n_rays_total;       /* equals ray_offsets[n_objects]; host copy for capacity checks */
  int32_t samples_per_ray;    /* S, 1..config.max_samples_per_ray */
  int32_t reserved;
  const int32_t* object_ids;  /* [n_objects] distinct registered object ids */
  const int32_t* ray_offsets; /* [n_objects + 1], ray_offsets[0] = 0, non-decreasing */
  const float* rays_o;        /* [R, 3] origins */
  const float* rays_d;        /* [R, 3] unit directions */
  const float* t;             /* [R, S] sample depths along each ray, ascending per ray */
  const float* depth;         /* [R] observed depth D (used where mask = 1) */
  const float* rgb;           /* [R, 3] observed colour C (used where mask = 1) */
  const float* mask;          /* [R] instance mask M in {0, 1} (Sec. 3.3, Training Objective) */
  const float* var;           /* [R, S] or NULL: per-sample variance (world units squared) of an
                               * isotropic Gaussian the sample stands for; each Fourier feature is
                               * then its expectation under it, the integrated positional
                               * encoding (supplementary Sec. B, object-level positional
                               * encoding): [sin, cos](x B) * exp(-var |b_f|^2 / (2 s^2)) in the
                               * object frame. NULL: point samples. */
} vmap_batch;

/* Bytes of the caller-owned device state buffer (parameters, Adam moments, gradients,
 * per-object descriptors, loss scaler). Returns 0 for an invalid config. Host only. */
size_t vmap_state_bytes(const vmap_config* cfg);

/* Bytes of the caller-owned device workspace for batches of up to config.max_rays rays and
 * config.max_objects objects: tile partial gradients, work lists, weight images (hidden 16 and
 * 32, one per object slot in either precision; hidden 128 in VMAP_BF16: the training kernels read
 * them) and, when max_hidden is a layered-path width, every sample's activations and deltas for
 * max_rays rays of max_samples_per_ray samples, and a BF16 copy of each object slot's parameters.
 * Returns 0 for an invalid config. Host only. */
size_t vmap_workspace_bytes(const vmap_config* cfg);

/* Number of parameters of one object of width `hidden` under cfg (no padding). Host only. */
int32_t vmap_object_params(const vmap_config* cfg, int32_t hidden);

/*
 * Create a context over caller-owned device buffers (256-byte aligned, at least the sizes
 * above). B_host is the [3 x n_features] FP32 encoding matrix (row-major), copied. The state is
 * cleared on `stream`. On success *out receives the context.
 */
int vmap_init_objects(const vmap_config* cfg, const float* B_host, void* state_dev,
                      size_t state_bytes, void* workspace_dev, size_t workspace_bytes,
                      void* stream, vmap_ctx** out);

/*
 * Append an object to the stack (Sec. 3.2). Its parameters are Xavier-uniform from
 * desc->seed (bound sqrt(6/(fan_in+fan_out)), uniforms from SplitMix64 in counter mode over the
 * flat parameter index, biases zero) unless init_params_host (FP32, vmap_object_params values)
 * is given. Adam moments and the step count start at zero. *object_id_out gets the new id.
 */
int vmap_add_object(vmap_ctx* ctx, const vmap_object_desc* desc, const float* init_params_host,
                    void* stream, int32_t* object_id_out);

/*
 * One optimisation step of every object in the batch (the vectorised step, Sec. 3.2-3.3):
 * encode, MLP, render (Eq. 3), losses (Eqs. 4-7), backward, Adam. Objects with zero rays
 * keep parameters, moments and step count unchanged. In BF16 mode the loss is scaled before
 * the backward, gradients are unscaled, and an object whose gradient is not finite skips its
 * update (parameters, moments and step count unchanged) while the scale halves; after
 * config.scale_growth_interval consecutive steps without a skipped object the scale doubles.
 * An object counts as not finite when a tile's partial gradient holds a non-finite element or
 * one of magnitude 2^64 or more (the sum over its tiles can then not overflow unnoticed); the
 * decision is taken for the whole object before any of its parameters is stored. The scale is a
 * power of two and stays in [2^-125, 2^126]. loss_out_dev (device, [n_objects], may be NULL)
 * receives each object's loss L^k of Eq. 7 (unscaled).
 */
int vmap_train_step(vmap_ctx* ctx, const vmap_batch* batch, float* loss_out_dev, void* stream);

/* Forward rendering of each ray with its object's model (Eq. 3): occupancy [R], depth [R],
 * colour [R, 3] (device pointers; any may be NULL). */
int vmap_render(vmap_ctx* ctx, const vmap_batch* batch, float* depth_out, float* rgb_out,
                float* occ_out, void* stream);

/*
 * Scene rendering from the object models (Sec. 3.4, "Compositional Scene Rendering"): each of
 * n_rays world-frame rays (device rays_o, rays_d [n_rays, 3], unit directions) is intersected
 * with the bound [c - s, c + s]^3 of every listed object (object_ids, device [n_objects],
 * registered ids) by the slab method; a ray that meets a bound after t_min is sampled at the
 * midpoints of S equal parts of its [entry, exit] interval and rendered with that object's
 * model (Eq. 3). Each ray then takes, among the objects it met, the one with the nearest
 * rendered depth whose rendered occupancy is >= occ_threshold (equal depths keep the earlier
 * listed object). Outputs (device): depth_out [n_rays] (0 where no object qualifies), and if not
 * NULL rgb_out [n_rays, 3], occ_out [n_rays], id_out [n_rays] (object id or -1), n_pairs_out [1]
 * (the number of (ray, object) pairs found). At most max_pairs pairs are rendered (0 <= max_pairs
 * <= config.max_rays); pairs beyond it are dropped and bit 1 of the device error reported by
 * vmap_step_info is set. scratch (device, 256-byte aligned, vmap_scene_scratch_bytes bytes,
 * caller-owned) holds the pairs. Returns VMAP_EINVAL / VMAP_ECAPACITY for bad arguments.
 */
size_t vmap_scene_scratch_bytes(int32_t n_rays, int32_t n_objects, int32_t max_pairs, int32_t S);
int vmap_render_scene(vmap_ctx* ctx, int32_t n_rays, const float* rays_o, const float* rays_d,
                      int32_t n_objects, const int32_t* object_ids, int32_t S, float t_min,
                      float occ_threshold, int32_t max_pairs, void* scratch, size_t scratch_bytes,
                      float* depth_out, float* rgb_out, float* occ_out, int32_t* id_out,
                      int32_t* n_pairs_out, void* stream);

/*
 * vmap_render_scene without the scratch arguments, for callers that cannot allocate device
 * memory per call: code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation. The pairs go to a static array of VMAP_SCENE_STATIC_SCRATCH_BYTES bytes that the
 * library holds on each GPU it runs on until the process ends (looked up once per GPU by
 * vmap_init_objects); the call allocates nothing and frees nothing. Arguments, outputs and
 * results are those of vmap_render_scene (bitwise: the same kernels run). A scene whose
 * vmap_scene_scratch_bytes(n_rays, n_objects, max_pairs, S) exceeds the array returns
 * VMAP_ECAPACITY with a message, before anything is enqueued. Every call on a GPU, from any
 * context, uses that GPU's one array: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller; a call needs nothing left in the array by
 * an earlier one (every byte it reads it first writes).
 */
#define VMAP_SCENE_STATIC_SCRATCH_BYTES ((size_t)16 << 20)
int vmap_render_scene_static(vmap_ctx* ctx, int32_t n_rays, const float* rays_o,
                             const float* rays_d, int32_t n_objects, const int32_t* object_ids,
                             int32_t S, float t_min, float occ_threshold, int32_t max_pairs,
                             float* depth_out, float* rgb_out, float* occ_out, int32_t* id_out,
                             int32_t* n_pairs_out, void* stream);

/* Occupancy [n] and, if rgb_out is not NULL, colour [n, 3] of n world-frame points (device
 * [n, 3]) under object `object_id`'s model (shape query inside its bound, Sec. 3.4). */
int vmap_query_occupancy(vmap_ctx* ctx, int32_t object_id, const float* pts_world_dev,
                         int64_t n, float* occ_out, float* rgb_out, void* stream);

/*
 * Depth-guided samples along rays (Sec. 3.3, Eqs. 1 and 2): for ray r, n_strat stratified
 * samples t_n + (i + u) / n_strat * (t_s - t_n), i < n_strat, and S - n_strat samples
 * t_s + sigma * z with z standard normal, where t_s = depth[r] if depth[r] > 0 and t_far[r]
 * otherwise (invalid depth). The S values are sorted ascending into t_out [n_rays, S].
 * Randomness: uniform j of sample i of ray r is output 2 (r S + i) + j of the SplitMix64 stream
 * started at `seed` (top 24 bits * 2^-24; the Box-Muller u1 is (top 24 bits + 1) * 2^-24).
 * Arithmetic in FP64, rounded once to FP32. All arrays are device pointers: t_near, t_far,
 * depth [n_rays] FP32 in, t_out [n_rays, S] FP32 out. 1 <= S <= 64, 0 <= n_strat <= S.
 */
int vmap_sample_rays(vmap_ctx* ctx, int32_t n_rays, int32_t S, int32_t n_strat,
                     const float* t_near, const float* t_far, const float* depth, float sigma,
                     uint64_t seed, float* t_out, void* stream);

/* Autograd split of the step. vmap_forward: per-object losses and renders (outputs may be
 * NULL). vmap_backward: gradient of sum_j dloss[j] * L^{object_ids[j]} with respect to the
 * parameters of each batch object (recomputing the forward), written to the internal gradient
 * slots and, if grad_out is not NULL, to grad_out (device, [n_objects, P_stride] FP32 where
 * P_stride is vmap_param_layout's stride). vmap_adam_step: Adam with the internal gradients for
 * the batch's objects that have rays. */
int vmap_forward(vmap_ctx* ctx, const vmap_batch* batch, float* loss_out, float* depth_out,
                 float* rgb_out, float* occ_out, void* stream);
int vmap_backward(vmap_ctx* ctx, const vmap_batch* batch, const float* dloss_dev,
                  float* grad_out, void* stream);
int vmap_adam_step(vmap_ctx* ctx, const vmap_batch* batch, void* stream);

/* Copy one object's parameters / Adam m / Adam v / gradient (FP32, `bytes` = 4 * n_params) or
 * step count (int32, bytes = 4) to or from host memory, or (VMAP_STATE_SCALER, object_id
 * ignored, bytes = 8) the context's loss scaler: FP32 scale, int32 consecutive good steps. With
 * these a training run stops and resumes where it was (Sec. 3.2: objects stop and resume without
 * interference): saving every object's four entries and the scaler after N steps and restoring
 * them into a fresh context gives, after M more steps, bitwise the state of N + M straight steps.
 * A scaler written must hold a power-of-two scale in [2^-125, 2^126] (VMAP_EINVAL otherwise).
 * Synchronises `stream`. */
int vmap_get_state(vmap_ctx* ctx, int32_t object_id, int32_t which, void* host_dst,
                   size_t bytes, void* stream);
int vmap_set_state(vmap_ctx* ctx, int32_t object_id, int32_t which, const void* host_src,
                   size_t bytes, void* stream);

/* Loss scale, objects skipped by the last step (non-finite gradients) and the device error
 * flags, sticky until the context is destroyed:
 *   bit 0 (1)  a batch named an unregistered or out-of-range object id (that object is skipped);
 *   bit 1 (2)  a scene render found more pairs than its max_pairs;
 *   bit 2 (4)  a batch's ray offsets were not a CSR over its rays: ray_offsets[0] != 0, a
 *              decreasing pair, or ray_offsets[n_objects] != n_rays_total. Checked on the device
 *              before any tile runs; such a batch is not run at all: no object, Adam moment, step
 *              count or loss scale changes, its losses are 0 and its renders are not written;
 *   bit 3 (8)  (contexts created with environment VMAP_DEBUG=1) a ray's sample depths were not
 *              ascending;
 *   bit 4 (16) (VMAP_DEBUG=1) an object id appeared twice in a batch.
 * The VMAP_DEBUG checks run one more kernel per call and only report: the step runs as usual.
 * Synchronises `stream`. */
int vmap_step_info(vmap_ctx* ctx, float* loss_scale, int32_t* skipped, int32_t* device_error,
                   void* stream);

/* Parameter count and slot stride (floats) of a registered object. Host only. */
int vmap_param_layout(const vmap_ctx* ctx, int32_t object_id, int32_t* n_params,
                      int32_t* stride);

/* Use hipGraph replay for vmap_train_step (1) or plain launches (0, default). */
int vmap_set_graph_mode(vmap_ctx* ctx, int32_t enabled);

/* Launch shape of the step's tile kernel: rays per tile is fixed at init; waves per block (1 to 4
 * in FP32, 1 to 8 in BF16; objects wider than 32 always take 4) and grid size (0 = one block per
 * tile) may change between steps. VMAP_EINVAL for a wave count out of range. */
int vmap_set_launch(vmap_ctx* ctx, int32_t waves_per_block, int32_t grid_blocks);

/* Average duration (ms) and count of the tile kernel launches timed with HIP events since the
 * last reset, when timing is enabled (enable = 1 starts and resets, 0 stops). The events are
 * recorded on the launch stream around the tile kernel (plain launches only). */
int vmap_kernel_timing(vmap_ctx* ctx, int32_t enable, double* avg_ms, int32_t* count);

/* Last error message of the context (or of the last failed vmap_init_objects if ctx is NULL). */
const char* vmap_last_error(const vmap_ctx* ctx);

/* Free the context (not the caller's buffers). Safe on NULL. */
void vmap_destroy(vmap_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* VMAP_H */
