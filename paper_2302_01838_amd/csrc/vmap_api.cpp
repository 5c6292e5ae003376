// Host side of the C ABI declared in include/vmap.h: context, object registry, validation,
// buffer layout, launch sequencing and optional hipGraph replay of the training step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "vmap.h"
#include "vmap_internal.h"

using namespace vmapi;

namespace {

thread_local std::string g_init_error;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int pad_params(int P) { return (P + 63) / 64 * 64; }

struct StateLayout {
  size_t desc, scaler, B, theta, m, v, grad, total;
};

struct WorkLayout {
  size_t tile_start, flags, t_next, mark, batch, tile_bad, tile_loss, partial, wimage, img32, gimg, total;
  size_t wimage_stride;
  int max_tiles;
  // layered path (generic widths): row tiles, their losses, activations, deltas, z and dz
  size_t gts, gbs, gws, gen_loss, gact, gdelta, gz, gdz;
  int max_gen_tiles, max_gen_blocks;
  int64_t gen_ld, gen_rows;
};

bool hidden_ok(int H, int precision) { return tiles_supported(H, precision == VMAP_BF16) != 0; }

const char* check_config(const vmap_config* c) {
  if (!c) return "config is NULL";
  if (c->max_objects < 1 || c->max_objects > 65536) return "max_objects must be in [1, 65536]";
  if (c->n_features != kFeatures) return "n_features must be 16";
  if (c->n_hidden_layers != kLayers) return "n_hidden_layers must be 4";
  if (c->precision != VMAP_FP32 && c->precision != VMAP_BF16) return "precision must be VMAP_FP32 or VMAP_BF16";
  if (!hidden_ok(c->hidden, c->precision))
    return "hidden width not supported (16, 32 or 64; 128, and 256, 512, 1024 by the layered path, in BF16)";
  if (c->max_hidden < c->hidden || !hidden_ok(c->max_hidden, c->precision))
    return "max_hidden must be a supported width >= hidden";
  if (c->max_samples_per_ray < 1 || c->max_samples_per_ray > kSlots) return "max_samples_per_ray must be in [1, 64]";
  if (c->max_rays < 0 || c->max_rays > (1 << 26)) return "max_rays must be in [0, 2^26]";
  if (c->rays_per_tile < 0 || c->rays_per_tile > (1 << 16)) return "rays_per_tile must be in [0, 65536]";
  if (c->rays_per_tile_wide < 0 || c->rays_per_tile_wide > (1 << 16))
    return "rays_per_tile_wide must be in [0, 65536]";
  if (c->split_step != 0 && c->split_step != 1) return "split_step must be 0 or 1";
  if (!(c->lr > 0.0) || !(c->beta1 >= 0.0 && c->beta1 < 1.0) || !(c->beta2 >= 0.0 && c->beta2 < 1.0) ||
      !(c->eps > 0.0))
    return "Adam settings out of range (lr > 0, 0 <= beta < 1, eps > 0)";
  if (!(c->lambda_colour >= 0.0) || !(c->lambda_occ >= 0.0)) return "loss weights must be >= 0";
  if (c->precision == VMAP_BF16) {
    int e2 = 0;
    if (!(c->loss_scale_init > 0.0) || !std::isfinite(c->loss_scale_init) ||
        std::frexp(c->loss_scale_init, &e2) != 0.5 || e2 - 1 < -125 || e2 - 1 > 126)
      return "loss_scale_init must be a power of two in [2^-125, 2^126] (the unscale is then exact)";
    if (c->scale_growth_interval < 1) return "scale_growth_interval must be >= 1";
  }
  return nullptr;
}

int default_rays_per_tile(const vmap_config* c) {
  if (c->rays_per_tile > 0) return c->rays_per_tile;
  const int rpw = std::max(1, kSlots / c->max_samples_per_ray);
  return rpw * 4 * 2;  // two sub-tiles per wave of a four-wave block
}

// Objects wider than 32 run in the cooperative kernel, whose tiles hold whole rounds (a sub-tile
// for each of its four waves). Few rays per object (a room's background: 1,200 rays) want one
// round per tile, to spread the object over many workgroups; many rays per object want longer
// tiles, to write fewer partial gradients (each is a whole object's parameter vector). Default:
// about max_rays / max_objects / 32 rays, in whole rounds, between one and eight rounds.
int default_rays_per_tile_wide(const vmap_config* c) {
  if (c->rays_per_tile_wide > 0) return c->rays_per_tile_wide;
  const int rpw = std::max(1, kSlots / c->max_samples_per_ray);
  const int round = rpw * 4;
  const double per_object = (double)c->max_rays / std::max(1, c->max_objects);
  const int rounds = (int)std::lround(per_object / 32.0 / round);
  return round * std::min(8, std::max(1, rounds));
}

// Smallest tile any object of the config may use (capacity bound).
int min_rays_per_tile(const vmap_config* c) {
  const int rpt = default_rays_per_tile(c);
  return c->max_hidden > 32 ? std::min(rpt, default_rays_per_tile_wide(c)) : rpt;
}

// Floats per object in the parameter, moment and gradient arrays and per tile partial: the
// parameters of the widest kernel width the stack may run (hidden 16 runs at width 32, and its
// tiles write width-32 partials).
int param_stride(const vmap_config* c) { return pad_params(n_params_of(kernel_width(c->max_hidden))); }

StateLayout state_layout(const vmap_config* c) {
  StateLayout s{};
  const size_t K = (size_t)c->max_objects;
  const size_t ps = (size_t)param_stride(c);
  size_t off = 0;
  s.desc = off; off = align256(off + K * sizeof(ObjDesc));
  s.scaler = off; off = align256(off + sizeof(ScalerState));
  s.B = off; off = align256(off + 3 * kFeatures * sizeof(float));
  s.theta = off; off = align256(off + K * ps * 4);
  s.m = off; off = align256(off + K * ps * 4);
  s.v = off; off = align256(off + K * ps * 4);
  s.grad = off; off = align256(off + K * ps * 4);
  s.total = off;
  return s;
}

WorkLayout work_layout(const vmap_config* c) {
  WorkLayout w{};
  const int rpt = min_rays_per_tile(c);
  const size_t ps = (size_t)param_stride(c);
  w.max_tiles = (c->max_rays + rpt - 1) / rpt + c->max_objects;
  size_t off = 0;
  w.tile_start = off; off = align256(off + ((size_t)c->max_objects + 1) * 4);
  w.flags = off; off = align256(off + (size_t)c->max_objects * 4);
  w.t_next = off; off = align256(off + (size_t)c->max_objects * 4);
  w.mark = off; off = align256(off + (size_t)c->max_objects * 4);  // debug validation of ids
  w.batch = off; off = align256(off + sizeof(BatchDev));
  w.tile_loss = off; off = align256(off + (size_t)w.max_tiles * 4);
  w.tile_bad = off; off = align256(off + (size_t)w.max_tiles * 4);
  w.partial = off; off = align256(off + (size_t)w.max_tiles * ps * 4);
  // weight images of hidden-128 objects (weights read from device memory by the tile kernel)
  const bool bf = c->precision == VMAP_BF16;
  w.wimage_stride = (bf && c->max_hidden >= 128) ? (size_t)image_bytes(128, true) : 0;
  w.wimage = off; off = align256(off + (size_t)c->max_objects * w.wimage_stride);
  // weight images of width-32 objects (staged by a plain copy)
  w.img32 = off; off = align256(off + (size_t)c->max_objects * img32_bytes(bf));
  // BF16 parameter copies of layered-path objects of hidden 128 and up (the wide products' W)
  w.gimg = off;
  if (bf && keeps_gimg(c->max_hidden)) off = align256(off + (size_t)c->max_objects * ps * 2);
  // layered path: when max_hidden is one of its widths, activations and deltas of every sample
  // (rows = max_rays * max_samples_per_ray, ld = max(32, max_hidden) BF16 per row)
  if (bf && generic_width(c->max_hidden)) {
    const int rpw = std::max(1, kSlots / c->max_samples_per_ray);
    w.max_gen_tiles = (c->max_rays + rpw - 1) / rpw + c->max_objects;
    w.gen_ld = std::max(kEnc, c->max_hidden);
    w.gen_rows = (int64_t)c->max_rays * c->max_samples_per_ray;
    const size_t layer = (size_t)w.gen_rows * (size_t)w.gen_ld * 2;
    w.max_gen_blocks = (int)((w.gen_rows + kGenBlockRows - 1) / kGenBlockRows) + c->max_objects;
    w.gts = off; off = align256(off + ((size_t)c->max_objects + 1) * 4);
    w.gbs = off; off = align256(off + ((size_t)c->max_objects + 1) * 4);
    w.gws = off; off = align256(off + ((size_t)c->max_objects + 1) * 4);
    w.gen_loss = off; off = align256(off + (size_t)w.max_gen_tiles * 4);
    w.gact = off; off = align256(off + (size_t)(kLayers + 1) * layer);
    // deltas: two buffers taken alternately
    w.gdelta = off; off = align256(off + 2 * layer);
    w.gz = off; off = align256(off + (size_t)w.gen_rows * kOut * 4);
    w.gdz = off; off = align256(off + (size_t)w.gen_rows * kOut * 4);
  }
  w.total = off;
  return w;
}

struct HostObj {
  int registered = 0;
  int hidden = 0;
  int n_params = 0;
};

struct TimedLaunch {
  hipEvent_t a, b;
};

}  // namespace

struct vmap_ctx {
  vmap_config cfg{};
  StateLayout sl{};
  WorkLayout wl{};
  unsigned char* state = nullptr;
  unsigned char* work = nullptr;
  int p_stride = 0;
  int rays_per_tile = 0;
  int rays_per_tile_wide = 0;
  int min_rays_per_tile = 0;
  // second stream for the width groups after the first (overlapped), with fork/join events
  hipStream_t side_stream = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int waves = 4;
  int grid_blocks = 0;
  int device = 0;
  int gen_width = 0;  // the one layered-path width of the stack's objects (0: none yet)
  bool debug = false;  // VMAP_DEBUG=1 at creation: device validation of every batch
  std::vector<HostObj> objs;
  int n_registered = 0;
  std::string err;
  // timing of the tile kernel
  bool timing = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  // graph replay of the training step
  bool graph_mode = false;
  struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::map<std::vector<int64_t>, GraphEntry> graphs;
  hipStream_t capture_stream = nullptr;
  // pinned host ring of batch descriptors copied to the workspace before each graph replay
  static constexpr int kRing = 64;
  BatchDev* ring = nullptr;
  hipEvent_t ring_ev[kRing] = {};
  bool ring_used[kRing] = {};
  int ring_next = 0;

  ObjDesc* desc() { return reinterpret_cast<ObjDesc*>(state + sl.desc); }
  ScalerState* scaler() { return reinterpret_cast<ScalerState*>(state + sl.scaler); }
  float* B() { return reinterpret_cast<float*>(state + sl.B); }
  float* theta() { return reinterpret_cast<float*>(state + sl.theta); }
  float* m() { return reinterpret_cast<float*>(state + sl.m); }
  float* v() { return reinterpret_cast<float*>(state + sl.v); }
  float* grad() { return reinterpret_cast<float*>(state + sl.grad); }
  int32_t* tile_start() { return reinterpret_cast<int32_t*>(work + wl.tile_start); }
  int32_t* flags() { return reinterpret_cast<int32_t*>(work + wl.flags); }
  int32_t* t_next() { return reinterpret_cast<int32_t*>(work + wl.t_next); }
  int32_t* mark() { return reinterpret_cast<int32_t*>(work + wl.mark); }
  BatchDev* batch_dev() { return reinterpret_cast<BatchDev*>(work + wl.batch); }
  int32_t* tile_bad() { return reinterpret_cast<int32_t*>(work + wl.tile_bad); }
  unsigned char* img32() { return work + wl.img32; }
  // BF16 parameter copies (layered path, hidden >= 128), or NULL when the stack keeps none
  uint16_t* gimg() {
    return (cfg.precision == VMAP_BF16 && keeps_gimg(cfg.max_hidden)) ? reinterpret_cast<uint16_t*>(work + wl.gimg) : nullptr;
  }
  float* tile_loss() { return reinterpret_cast<float*>(work + wl.tile_loss); }
  float* partial() { return reinterpret_cast<float*>(work + wl.partial); }
  unsigned char* wimage() { return wl.wimage_stride ? work + wl.wimage : nullptr; }

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int hip_fail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return VMAP_EHIP;
  }
};

namespace {

int validate_batch(vmap_ctx* c, const vmap_batch* b, bool need_targets) {
  if (!b) return c->fail(VMAP_EINVAL, "batch is NULL");
  if (b->n_objects < 0) return c->fail(VMAP_EINVAL, "batch.n_objects must be >= 0");
  if (b->n_objects > c->cfg.max_objects)
    return c->fail(VMAP_ECAPACITY, "batch.n_objects exceeds max_objects");
  if (b->n_rays_total < 0) return c->fail(VMAP_EINVAL, "batch.n_rays_total must be >= 0");
  if (b->n_rays_total > c->cfg.max_rays) return c->fail(VMAP_ECAPACITY, "batch.n_rays_total exceeds max_rays");
  if (b->samples_per_ray < 1 || b->samples_per_ray > c->cfg.max_samples_per_ray)
    return c->fail(VMAP_EINVAL, "batch.samples_per_ray out of [1, max_samples_per_ray]");
  if (b->n_objects > 0 && (!b->object_ids || !b->ray_offsets))
    return c->fail(VMAP_EINVAL, "batch.object_ids and batch.ray_offsets must not be NULL");
  if (b->n_rays_total > 0) {
    if (!b->rays_o || !b->rays_d || !b->t) return c->fail(VMAP_EINVAL, "batch ray arrays must not be NULL");
    if (need_targets && (!b->depth || !b->rgb || !b->mask))
      return c->fail(VMAP_EINVAL, "batch targets (depth, rgb, mask) must not be NULL");
  }
  const int rpt = c->min_rays_per_tile;
  const long long tiles = ((long long)b->n_rays_total + rpt - 1) / rpt + b->n_objects;
  if (tiles > c->wl.max_tiles) return c->fail(VMAP_ECAPACITY, "batch needs more tiles than the workspace holds");
  return VMAP_OK;
}

// Kernel widths of the registered objects (hidden 16 shares the width-32 kernels), ascending:
// one width group, and one tile launch or layered chain, per entry.
std::vector<int> widths_present(vmap_ctx* c) {
  std::vector<int> w;
  for (const auto& o : c->objs) {
    const int kw = kernel_width(o.hidden);
    if (o.registered && std::find(w.begin(), w.end(), kw) == w.end()) w.push_back(kw);
  }
  std::sort(w.begin(), w.end());
  return w;
}

StepArgs make_step_args(vmap_ctx* c, const vmap_batch* b) {
  StepArgs a{};
  a.n_objects = b->n_objects;
  a.n_rays = b->n_rays_total;
  a.max_tiles = c->wl.max_tiles;
  a.S = b->samples_per_ray;
  a.rays_per_tile = c->rays_per_tile;
  a.rays_per_tile_wide = c->rays_per_tile_wide;
  a.max_objects = c->cfg.max_objects;
  a.object_ids = b->object_ids;
  a.ray_offsets = b->ray_offsets;
  a.rays_o = b->rays_o;
  a.rays_d = b->rays_d;
  a.t = b->t;
  a.depth = b->depth;
  a.rgb = b->rgb;
  a.mask = b->mask;
  a.var = b->var;
  a.theta = c->theta();
  a.p_stride = c->p_stride;
  a.desc = c->desc();
  a.scaler = c->scaler();
  a.B = c->B();
  a.tile_start = c->tile_start();
  a.partial = c->partial();
  a.tile_loss = c->tile_loss();
  a.flags = c->flags();
  a.lambda_c = (float)c->cfg.lambda_colour;
  a.lambda_o = (float)c->cfg.lambda_occ;
  a.wimage = c->wimage();
  a.wimage_stride = (int64_t)c->wl.wimage_stride;
  a.img32 = c->img32();
  a.gimg = c->gimg();
  return a;
}

// Debug validation of the batch before its first kernel (contexts created with VMAP_DEBUG=1).
int enqueue_debug(vmap_ctx* c, const vmap_batch* b, hipStream_t s, const BatchDev* bd = nullptr) {
  if (!c->debug || b->n_objects == 0) return VMAP_OK;
  StepArgs a = make_step_args(c, b);
  a.bd = bd;
  const hipError_t e = launch_debug_batch(a, c->mark(), s);
  return e == hipSuccess ? VMAP_OK : c->hip_fail(e, "debug validation launch");
}

hipEvent_t pooled_event(vmap_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Rays per work tile of a layered-path object in a batch of S samples per ray: about
// kGenWorkRows rows, never fewer rays than the narrow tiles the workspace's tile count allows for.
int gen_work_rays(const vmap_ctx* c, int S) {
  return std::max(c->min_rays_per_tile, (kGenWorkRows + S - 1) / std::max(S, 1));
}

hipError_t enqueue_worklist(vmap_ctx* c, const vmap_batch* b, hipStream_t s,
                            const BatchDev* bd = nullptr) {
  return launch_worklist(b->n_objects, b->n_rays_total, b->object_ids, b->ray_offsets,
                         c->rays_per_tile, c->rays_per_tile_wide, gen_work_rays(c, b->samples_per_ray),
                         c->cfg.max_objects, c->desc(), c->scaler(), c->tile_start(), c->flags(),
                         c->t_next(), bd, s);
}

OptArgs make_opt_args(vmap_ctx* c, const vmap_batch* b, float* loss_out, float* grad_out,
                      const BatchDev* bd = nullptr) {
  OptArgs a{};
  a.bd = bd;
  a.n_objects = b->n_objects;
  a.ids = b->object_ids;
  a.offs = b->ray_offsets;
  a.tile_start = c->tile_start();
  a.partial = c->partial();
  a.tile_loss = c->tile_loss();
  a.t_next = c->t_next();
  a.p_stride = c->p_stride;
  a.max_objects = c->cfg.max_objects;
  a.desc = c->desc();
  a.scaler = c->scaler();
  a.flags = c->flags();
  a.theta = c->theta();
  a.m = c->m();
  a.v = c->v();
  a.grad = c->grad();
  a.grad_out = grad_out;
  a.loss_out = loss_out;
  a.lr = c->cfg.lr;
  a.beta1 = c->cfg.beta1;
  a.beta2 = c->cfg.beta2;
  a.eps = c->cfg.eps;
  a.bf16 = c->cfg.precision == VMAP_BF16;
  a.growth = c->cfg.scale_growth_interval;
  a.max_tiles = c->wl.max_tiles;
  a.img32 = c->img32();
  a.wimage = c->wimage();
  a.wimage_stride = (int64_t)c->wl.wimage_stride;
  a.gimg = c->gimg();
  return a;
}

// Enqueue the tile kernel for every width group.
int enqueue_tiles(vmap_ctx* c, const vmap_batch* b, int mode, const float* dloss, float* d_out,
                  float* rgb_out, float* occ_out, hipStream_t s, bool allow_timing,
                  const BatchDev* bd = nullptr) {
  StepArgs a = make_step_args(c, b);
  a.bd = bd;
  a.dloss = dloss;
  a.out_depth = d_out;
  a.out_rgb = rgb_out;
  a.out_occ = occ_out;
  a.use_scale = (mode == MODE_TRAIN && c->cfg.precision == VMAP_BF16) ? 1 : 0;
  const bool bf = c->cfg.precision == VMAP_BF16;
  const int bound = (b->n_rays_total + c->min_rays_per_tile - 1) / c->min_rays_per_tile + b->n_objects;
  int grid = bound;
  if (c->grid_blocks > 0) grid = std::min(grid, c->grid_blocks);
  TimedLaunch tl{};
  const bool timed = allow_timing && c->timing;
  if (timed) {
    tl.a = pooled_event(c);
    tl.b = pooled_event(c);
    if (!tl.a || !tl.b) return c->fail(VMAP_EHIP, "hipEventCreate failed");
    hipError_t e = hipEventRecord(tl.a, s);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventRecord");
  }
  // Width groups run as separate kernels; with more than one, every group after the first goes
  // to a side stream (forked from and joined back into `s` by events, which graph capture
  // follows), so that the groups overlap on the GPU.
  const std::vector<int> widths = widths_present(c);
  const bool fork = widths.size() > 1;
  if (fork) {
    if (!c->side_stream) {
      hipError_t e = hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming);
      if (e != hipSuccess) return c->hip_fail(e, "side stream");
    }
    hipError_t e = hipEventRecord(c->fork_ev, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->side_stream, c->fork_ev, 0);
    if (e != hipSuccess) return c->hip_fail(e, "stream fork");
  }
  for (size_t i = 0; i < widths.size(); ++i) {
    const int H = widths[i];
    hipStream_t si = (i == 0) ? s : c->side_stream;
    a.hidden = H;
    if (generic_width(H)) {  // the layered path's chain of launches
      GenArgs g{};
      g.a = a;
      g.H = H;
      g.rpw = std::max(1, kSlots / b->samples_per_ray);
      g.max_gen_tiles = c->wl.max_gen_tiles;
      g.gts = reinterpret_cast<int32_t*>(c->work + c->wl.gts);
      g.gbs = reinterpret_cast<int32_t*>(c->work + c->wl.gbs);
      g.gws = reinterpret_cast<int32_t*>(c->work + c->wl.gws);
      g.max_gen_blocks = c->wl.max_gen_blocks;
      g.gen_loss = reinterpret_cast<float*>(c->work + c->wl.gen_loss);
      g.act = reinterpret_cast<uint16_t*>(c->work + c->wl.gact);
      const size_t layer = (size_t)c->wl.gen_rows * (size_t)c->wl.gen_ld;
      g.delta[0] = reinterpret_cast<uint16_t*>(c->work + c->wl.gdelta);
      g.delta[1] = g.delta[0] + layer;
      g.z = reinterpret_cast<float*>(c->work + c->wl.gz);
      g.dz = reinterpret_cast<float*>(c->work + c->wl.gdz);
      g.ld = c->wl.gen_ld;
      g.layer_elems = (int64_t)layer;
      const int tiles_bound = (b->n_rays_total + g.rpw - 1) / g.rpw + b->n_objects;
      if (tiles_bound > g.max_gen_tiles) return c->fail(VMAP_ECAPACITY, "batch needs more row tiles than the workspace holds");
      const long long rows = (long long)b->n_rays_total * b->samples_per_ray;
      const long long blocks_bound = (rows + kGenBlockRows - 1) / kGenBlockRows + b->n_objects;
      if (blocks_bound > g.max_gen_blocks) return c->fail(VMAP_ECAPACITY, "batch needs more row blocks than the workspace holds");
      g.work_rays = gen_work_rays(c, b->samples_per_ray);
      const int work_bound = (b->n_rays_total + g.work_rays - 1) / g.work_rays + b->n_objects;
      hipError_t e = launch_generic(mode, g, tiles_bound, (int)blocks_bound, work_bound, si);
      if (e != hipSuccess) return c->hip_fail(e, "layered-path launch");
      continue;
    }
    // The weight images are current (staged when parameters are set, then kept by the optimiser).
    // This width's tiles are at most ceil(rays / its rays per tile) + objects: wider tiles need
    // fewer workgroups than the stack's smallest tile size gives (the kernels stride over tiles).
    const int rpt_h = tile_rays(H, c->rays_per_tile, c->rays_per_tile_wide);
    const int grid_h = std::min(grid, (b->n_rays_total + rpt_h - 1) / rpt_h + b->n_objects);
    hipError_t e = launch_tiles(H, bf, mode, a, c->waves, grid_h, si);
    if (e != hipSuccess) return c->hip_fail(e, "tile kernel launch");
  }
  if (fork) {
    hipError_t e = hipEventRecord(c->join_ev, c->side_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->join_ev, 0);
    if (e != hipSuccess) return c->hip_fail(e, "stream join");
  }
  if (timed) {
    hipError_t e = hipEventRecord(tl.b, s);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventRecord");
    c->timed.push_back(tl);
  }
  return VMAP_OK;
}

// Training step whose tile kernel builds the tile table itself (no work-list launch), used when
// every registered object has width 32, the batch fits the kernel's LDS table and the
// configuration does not ask for the separate work-list launch.
bool table_in_tiles(vmap_ctx* c, const vmap_batch* b) {
  if (c->cfg.split_step || b->n_objects > kTableMaxObjects) return false;
  const std::vector<int> w = widths_present(c);
  return w.size() == 1 && w[0] == 32;
}

int enqueue_step(vmap_ctx* c, const vmap_batch* b, float* loss_out, hipStream_t s, bool allow_timing,
                 const BatchDev* bd) {
  StepArgs a = make_step_args(c, b);
  a.bd = bd;
  a.use_scale = c->cfg.precision == VMAP_BF16 ? 1 : 0;
  a.hidden = 32;
  a.tile_start_out = c->tile_start();
  a.t_next = c->t_next();
  a.tile_bad = c->tile_bad();
  int grid = (b->n_rays_total + c->rays_per_tile - 1) / c->rays_per_tile + b->n_objects;
  if (c->grid_blocks > 0) grid = std::min(grid, c->grid_blocks);
  TimedLaunch tl{};
  const bool timed = allow_timing && c->timing;
  if (timed) {
    tl.a = pooled_event(c);
    tl.b = pooled_event(c);
    if (!tl.a || !tl.b) return c->fail(VMAP_EHIP, "hipEventCreate failed");
    hipError_t e = hipEventRecord(tl.a, s);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventRecord");
  }
  hipError_t e = launch_tiles(32, c->cfg.precision == VMAP_BF16, MODE_STEP, a, c->waves, grid, s);
  if (e != hipSuccess) return c->hip_fail(e, "tile kernel launch");
  if (timed) {
    e = hipEventRecord(tl.b, s);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventRecord");
    c->timed.push_back(tl);
  }
  OptArgs o = make_opt_args(c, b, loss_out, nullptr, bd);
  o.tile_bad = c->tile_bad();
  e = launch_optimizer(OPT_REDUCE_ADAM, o, s);
  if (e != hipSuccess) return c->hip_fail(e, "gradient/Adam launch");
  return VMAP_OK;
}

int enqueue_train(vmap_ctx* c, const vmap_batch* b, float* loss_out, hipStream_t s, bool allow_timing,
                  const BatchDev* bd = nullptr) {
  if (int rc = enqueue_debug(c, b, s, bd)) return rc;
  if (table_in_tiles(c, b)) return enqueue_step(c, b, loss_out, s, allow_timing, bd);
  hipError_t e = enqueue_worklist(c, b, s, bd);
  if (e != hipSuccess) return c->hip_fail(e, "worklist launch");
  int rc = enqueue_tiles(c, b, MODE_TRAIN, nullptr, nullptr, nullptr, nullptr, s, allow_timing, bd);
  if (rc) return rc;
  e = launch_optimizer(OPT_REDUCE_ADAM, make_opt_args(c, b, loss_out, nullptr, bd), s);
  if (e != hipSuccess) return c->hip_fail(e, "gradient/Adam launch");
  return VMAP_OK;
}

struct SceneLayout {
  size_t counts, offsets, map, pair_o, pair_d, pair_t, pair_depth, pair_rgb, pair_occ, bd, total;
};

SceneLayout scene_layout(int64_t n_rays, int64_t n_objects, int64_t max_pairs, int64_t S) {
  SceneLayout L{};
  const int64_t nblk = (n_rays + 255) / 256;
  size_t off = 0;
  L.counts = off; off = align256(off + (size_t)(n_objects * nblk) * 4);
  L.offsets = off; off = align256(off + (size_t)(n_objects + 1) * 4);
  L.map = off; off = align256(off + (size_t)(n_objects * n_rays) * 4);
  L.pair_o = off; off = align256(off + (size_t)max_pairs * 12);
  L.pair_d = off; off = align256(off + (size_t)max_pairs * 12);
  L.pair_t = off; off = align256(off + (size_t)(max_pairs * S) * 4);
  L.pair_depth = off; off = align256(off + (size_t)max_pairs * 4);
  L.pair_rgb = off; off = align256(off + (size_t)max_pairs * 12);
  L.pair_occ = off; off = align256(off + (size_t)max_pairs * 4);
  L.bd = off; off = align256(off + sizeof(BatchDev));
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

size_t vmap_state_bytes(const vmap_config* cfg) {
  if (check_config(cfg)) return 0;
  return state_layout(cfg).total;
}

size_t vmap_workspace_bytes(const vmap_config* cfg) {
  if (check_config(cfg)) return 0;
  return work_layout(cfg).total;
}

int32_t vmap_object_params(const vmap_config* cfg, int32_t hidden) {
  if (check_config(cfg) || !hidden_ok(hidden, cfg->precision) || hidden > cfg->max_hidden) return 0;
  return n_params_of(hidden);
}

int vmap_init_objects(const vmap_config* cfg, const float* B_host, void* state_dev,
                      size_t state_bytes, void* workspace_dev, size_t workspace_bytes,
                      void* stream, vmap_ctx** out) {
  if (!out) {
    g_init_error = "out is NULL";
    return VMAP_EINVAL;
  }
  *out = nullptr;
  if (const char* m = check_config(cfg)) {
    g_init_error = m;
    return (cfg && (cfg->n_hidden_layers != kLayers || cfg->n_features != kFeatures)) ? VMAP_ENOTSUP : VMAP_EINVAL;
  }
  if (!B_host || !state_dev || !workspace_dev) {
    g_init_error = "B_host, state_dev and workspace_dev must not be NULL";
    return VMAP_EINVAL;
  }
  if (((uintptr_t)state_dev & 255) || ((uintptr_t)workspace_dev & 255)) {
    g_init_error = "state and workspace buffers must be 256-byte aligned";
    return VMAP_EINVAL;
  }
  const StateLayout sl = state_layout(cfg);
  const WorkLayout wl = work_layout(cfg);
  if (state_bytes < sl.total || workspace_bytes < wl.total) {
    g_init_error = "state or workspace buffer smaller than vmap_state_bytes / vmap_workspace_bytes";
    return VMAP_ECAPACITY;
  }
  for (int i = 0; i < 3 * kFeatures; ++i) {
    if (!std::isfinite(B_host[i])) {
      g_init_error = "B contains a non-finite value";
      return VMAP_EINVAL;
    }
  }
  const bool bf = cfg->precision == VMAP_BF16;
  for (int H = 32; H <= kernel_width(cfg->max_hidden); H *= 2) {
    if (tiles_supported(H, bf) && tile_lds_bytes(H, bf, 4) > 160 * 1024) {
      g_init_error = "model too large for the 160 KB LDS of a workgroup";
      return VMAP_ENOTSUP;
    }
  }
  vmap_ctx* c = new vmap_ctx();
  c->cfg = *cfg;
  c->sl = sl;
  c->wl = wl;
  c->state = reinterpret_cast<unsigned char*>(state_dev);
  c->work = reinterpret_cast<unsigned char*>(workspace_dev);
  c->p_stride = param_stride(cfg);
  c->rays_per_tile = default_rays_per_tile(cfg);
  c->rays_per_tile_wide = default_rays_per_tile_wide(cfg);
  c->min_rays_per_tile = min_rays_per_tile(cfg);
  c->objs.resize(cfg->max_objects);
  const char* dbg = std::getenv("VMAP_DEBUG");
  c->debug = dbg && dbg[0] && std::strcmp(dbg, "0") != 0;
  (void)hipGetDevice(&c->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the allocation-free scene render's static scratch on this GPU (looked up once per GPU)
  hipError_t e = static_scratch_init(c->device);
  if (e != hipSuccess) {
    g_init_error = std::string("looking up the static scene scratch: ") + hipGetErrorString(e);
    delete c;
    return VMAP_EHIP;
  }
  e = launch_fill_zero(state_dev, sl.total, s);
  if (e == hipSuccess) e = launch_fill_zero(workspace_dev, wl.total, s);
  if (e == hipSuccess) e = launch_init_scaler(c->scaler(), bf ? (float)cfg->loss_scale_init : 1.0f, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->B(), B_host, 3 * kFeatures * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    g_init_error = std::string("initialising state: ") + hipGetErrorString(e);
    delete c;
    return VMAP_EHIP;
  }
  *out = c;
  return VMAP_OK;
}

// The weight image of object k (width 32, or the BF16 image of hidden 128), or its BF16 parameter
// copy (layered path, hidden 256 and up), from its current parameters. The optimiser kernels keep
// them current after each update.
hipError_t restage_image(vmap_ctx* c, int k, hipStream_t s) {
  if (keeps_gimg(c->objs[k].hidden)) {
    uint16_t* gimg = c->gimg();
    return gimg ? launch_stage_gimg(c->theta(), gimg, k, c->p_stride, s) : hipSuccess;
  }
  const int kw = kernel_width(c->objs[k].hidden);
  if (kw != 32 && !weights_global(kw)) return hipSuccess;
  StepArgs a{};
  a.max_objects = c->cfg.max_objects;
  a.theta = c->theta();
  a.p_stride = c->p_stride;
  a.desc = c->desc();
  a.img32 = c->img32();
  a.wimage = c->wimage();
  a.wimage_stride = (int64_t)c->wl.wimage_stride;
  a.gimg = c->gimg();
  if (weights_global(kw)) return launch_stage_images(kw, c->cfg.precision == VMAP_BF16, a, k, s);
  return launch_stage_image32(c->cfg.precision == VMAP_BF16, a, k, s);
}

int vmap_add_object(vmap_ctx* c, const vmap_object_desc* d, const float* init_params_host,
                    void* stream, int32_t* object_id_out) {
  if (!c) return VMAP_EINVAL;
  if (!d || !object_id_out) return c->fail(VMAP_EINVAL, "desc and object_id_out must not be NULL");
  const int H = d->hidden ? d->hidden : c->cfg.hidden;
  if (!hidden_ok(H, c->cfg.precision) || H > c->cfg.max_hidden)
    return c->fail(VMAP_ENOTSUP, "object hidden width not supported or above max_hidden");
  if (generic_width(H) && c->gen_width != 0 && c->gen_width != H)
    return c->fail(VMAP_ENOTSUP, "a stack holds objects of at most one layered-path width");
  if (!(d->scale > 0.f) || !std::isfinite(d->scale)) return c->fail(VMAP_EINVAL, "desc.scale must be > 0");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(d->centre[i])) return c->fail(VMAP_EINVAL, "desc.centre must be finite");
  if (c->n_registered >= c->cfg.max_objects) return c->fail(VMAP_ECAPACITY, "model stack is full (max_objects)");
  const int k = c->n_registered;
  const int P = n_params_of(H);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ObjDesc od{};
  for (int i = 0; i < 3; ++i) od.centre[i] = (double)d->centre[i];
  od.inv_scale = 1.0 / (double)d->scale;
  od.hidden = H;
  od.registered = 1;
  od.step = 0;
  od.n_params = P;
  double bounds[kLayers + 1];
  for (int l = 0; l <= kLayers; ++l) {
    const int fi = (l == 0) ? kEnc : H;
    const int fo = (l == kLayers) ? kOut : H;
    bounds[l] = std::sqrt(6.0 / (double)(fi + fo));
  }
  hipError_t e = launch_init_object(k, H, d->seed, bounds, od, c->desc(), c->theta(), c->m(), c->v(),
                                    c->grad(), c->p_stride, init_params_host ? 0 : 1, s);
  if (e != hipSuccess) return c->hip_fail(e, "init kernel launch");
  if (init_params_host) {
    e = hipMemcpyAsync(c->theta() + (size_t)k * c->p_stride, init_params_host, (size_t)P * 4,
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return c->hip_fail(e, "copying initial parameters");
  }
  c->objs[k].registered = 1;
  c->objs[k].hidden = H;
  c->objs[k].n_params = P;
  c->n_registered++;
  if (generic_width(H)) c->gen_width = H;
  e = restage_image(c, k, s);
  if (e != hipSuccess) return c->hip_fail(e, "weight image launch");
  *object_id_out = k;
  return VMAP_OK;
}

int vmap_train_step(vmap_ctx* c, const vmap_batch* b, float* loss_out, void* stream) {
  if (!c) return VMAP_EINVAL;
  int rc = validate_batch(c, b, true);
  if (rc) return rc;
  if (b->n_objects == 0) return VMAP_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!c->graph_mode) return enqueue_train(c, b, loss_out, s, true);
  // Graph replay. The graph is captured once per batch shape; the batch's buffers reach its
  // kernels through a device descriptor refreshed by one copy from a pinned host ring per call.
  if (!c->ring) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->ring), sizeof(BatchDev) * vmap_ctx::kRing, 0);
    if (e != hipSuccess) return c->hip_fail(e, "hipHostMalloc");
  }
  const int slot = c->ring_next;
  c->ring_next = (c->ring_next + 1) % vmap_ctx::kRing;
  if (c->ring_used[slot]) {  // the copy that last read this slot must have run
    hipError_t e = hipEventSynchronize(c->ring_ev[slot]);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventSynchronize");
  } else {
    hipError_t e = hipEventCreateWithFlags(&c->ring_ev[slot], hipEventDisableTiming);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventCreate");
    c->ring_used[slot] = true;
  }
  BatchDev& hb = c->ring[slot];
  hb = make_batch_dev(b->n_objects, b->samples_per_ray, b->n_rays_total, b->object_ids,
                      b->ray_offsets, b->rays_o, b->rays_d, b->t, b->depth, b->rgb, b->mask,
                      loss_out, b->var);
  std::vector<int64_t> key = {b->n_objects, b->n_rays_total, b->samples_per_ray, c->waves,
                              c->grid_blocks, (int64_t)widths_present(c).size(),
                              loss_out ? 1 : 0};
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    if (!c->capture_stream) {
      hipError_t e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return c->hip_fail(e, "hipStreamCreate");
    }
    hipError_t e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return c->hip_fail(e, "hipStreamBeginCapture");
    rc = enqueue_train(c, b, loss_out, c->capture_stream, false, c->batch_dev());
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->capture_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return c->hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return c->hip_fail(e, "hipGraphInstantiate");
    }
    it = c->graphs.emplace(key, vmap_ctx::GraphEntry{g, x}).first;
  }
  hipError_t e = hipMemcpyAsync(c->batch_dev(), &hb, sizeof(BatchDev), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return c->hip_fail(e, "copying the batch descriptor");
  e = hipEventRecord(c->ring_ev[slot], s);
  if (e != hipSuccess) return c->hip_fail(e, "hipEventRecord");
  e = hipGraphLaunch(it->second.exec, s);
  if (e != hipSuccess) return c->hip_fail(e, "hipGraphLaunch");
  return VMAP_OK;
}

int vmap_forward(vmap_ctx* c, const vmap_batch* b, float* loss_out, float* depth_out, float* rgb_out,
                 float* occ_out, void* stream) {
  if (!c) return VMAP_EINVAL;
  int rc = validate_batch(c, b, loss_out != nullptr);
  if (rc) return rc;
  if (b->n_objects == 0) return VMAP_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((rc = enqueue_debug(c, b, s))) return rc;
  hipError_t e = enqueue_worklist(c, b, s);
  if (e != hipSuccess) return c->hip_fail(e, "worklist launch");
  rc = enqueue_tiles(c, b, MODE_FWD, nullptr, depth_out, rgb_out, occ_out, s, true);
  if (rc) return rc;
  if (loss_out) {
    e = launch_optimizer(OPT_LOSS, make_opt_args(c, b, loss_out, nullptr), s);
    if (e != hipSuccess) return c->hip_fail(e, "loss launch");
  }
  return VMAP_OK;
}

int vmap_render(vmap_ctx* c, const vmap_batch* b, float* depth_out, float* rgb_out, float* occ_out,
                void* stream) {
  if (!c) return VMAP_EINVAL;
  if (!b) return c->fail(VMAP_EINVAL, "batch is NULL");
  if (b->n_rays_total > 0 && !depth_out && !rgb_out && !occ_out)
    return c->fail(VMAP_EINVAL, "vmap_render needs at least one output");
  // rendering reads no targets: the batch's depth, rgb and mask may be NULL
  vmap_batch rb = *b;
  rb.depth = nullptr;
  rb.rgb = nullptr;
  rb.mask = nullptr;
  b = &rb;
  return vmap_forward(c, b, nullptr, depth_out, rgb_out, occ_out, stream);
}

size_t vmap_scene_scratch_bytes(int32_t n_rays, int32_t n_objects, int32_t max_pairs, int32_t S) {
  if (n_rays < 0 || n_objects < 0 || max_pairs < 0 || S < 1 || S > kSlots) return 0;
  return scene_layout(n_rays, n_objects, max_pairs, S).total;
}

// The scene render over a given scratch (caller-owned, or the library's static array).
static int render_scene(vmap_ctx* c, int32_t n_rays, const float* rays_o, const float* rays_d,
                        int32_t n_objects, const int32_t* object_ids, int32_t S, float t_min,
                        float occ_threshold, int32_t max_pairs, void* scratch, size_t scratch_bytes,
                        float* depth_out, float* rgb_out, float* occ_out, int32_t* id_out,
                        int32_t* n_pairs_out, void* stream) {
  if (n_rays < 0) return c->fail(VMAP_EINVAL, "n_rays must be >= 0");
  if (n_objects < 0 || n_objects > c->cfg.max_objects)
    return c->fail(VMAP_EINVAL, "n_objects must be in [0, max_objects]");
  if (S < 1 || S > c->cfg.max_samples_per_ray)
    return c->fail(VMAP_EINVAL, "S must be in [1, max_samples_per_ray]");
  if (max_pairs < 0 || max_pairs > c->cfg.max_rays)
    return c->fail(VMAP_ECAPACITY, "max_pairs must be in [0, max_rays]");
  if (!std::isfinite(t_min) || !std::isfinite(occ_threshold))
    return c->fail(VMAP_EINVAL, "t_min and occ_threshold must be finite");
  if (n_rays == 0 || n_objects == 0) return VMAP_OK;
  if (!rays_o || !rays_d || !object_ids || !scratch || !depth_out)
    return c->fail(VMAP_EINVAL, "rays_o, rays_d, object_ids, scratch and depth_out must not be NULL");
  if ((uintptr_t)scratch & 255) return c->fail(VMAP_EINVAL, "scratch must be 256-byte aligned");
  if ((int64_t)n_rays * n_objects > ((int64_t)1 << 31) - 1)
    return c->fail(VMAP_ECAPACITY, "n_rays * n_objects must stay below 2^31");
  const SceneLayout L = scene_layout(n_rays, n_objects, max_pairs, S);
  if (scratch_bytes < L.total) return c->fail(VMAP_ECAPACITY, "scratch smaller than vmap_scene_scratch_bytes");
  unsigned char* sc = reinterpret_cast<unsigned char*>(scratch);
  SceneArgs a{};
  a.n_rays = n_rays;
  a.n_objects = n_objects;
  a.S = S;
  a.max_objects = c->cfg.max_objects;
  a.max_pairs = max_pairs;
  a.occ_threshold = occ_threshold;
  a.t_min = (double)t_min;
  a.rays_o = rays_o;
  a.rays_d = rays_d;
  a.object_ids = object_ids;
  a.desc = c->desc();
  a.scaler = c->scaler();
  a.counts = reinterpret_cast<int32_t*>(sc + L.counts);
  a.ray_offsets = reinterpret_cast<int32_t*>(sc + L.offsets);
  a.pair_map = reinterpret_cast<int32_t*>(sc + L.map);
  a.pair_o = reinterpret_cast<float*>(sc + L.pair_o);
  a.pair_d = reinterpret_cast<float*>(sc + L.pair_d);
  a.pair_t = reinterpret_cast<float*>(sc + L.pair_t);
  a.pair_depth = reinterpret_cast<float*>(sc + L.pair_depth);
  a.pair_rgb = reinterpret_cast<float*>(sc + L.pair_rgb);
  a.pair_occ = reinterpret_cast<float*>(sc + L.pair_occ);
  a.bd = reinterpret_cast<BatchDev*>(sc + L.bd);
  a.n_pairs_out = n_pairs_out;
  a.depth_out = depth_out;
  a.rgb_out = rgb_out;
  a.occ_out = occ_out;
  a.id_out = id_out;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_scene(0, a, s);
  if (e != hipSuccess) return c->hip_fail(e, "scene pair launch");
  if (max_pairs > 0) {
    // the pairs as a batch: shape bounds on the host, contents from the device descriptor
    vmap_batch hb{};
    hb.n_objects = n_objects;
    hb.n_rays_total = max_pairs;
    hb.samples_per_ray = S;
    hb.object_ids = object_ids;
    hb.ray_offsets = a.ray_offsets;
    e = enqueue_worklist(c, &hb, s, a.bd);
    if (e != hipSuccess) return c->hip_fail(e, "worklist launch");
    int rc = enqueue_tiles(c, &hb, MODE_FWD, nullptr, a.pair_depth, a.pair_rgb, a.pair_occ, s, false, a.bd);
    if (rc) return rc;
  }
  e = launch_scene(1, a, s);
  if (e != hipSuccess) return c->hip_fail(e, "scene composite launch");
  return VMAP_OK;
}

int vmap_render_scene(vmap_ctx* c, int32_t n_rays, const float* rays_o, const float* rays_d,
                      int32_t n_objects, const int32_t* object_ids, int32_t S, float t_min,
                      float occ_threshold, int32_t max_pairs, void* scratch, size_t scratch_bytes,
                      float* depth_out, float* rgb_out, float* occ_out, int32_t* id_out,
                      int32_t* n_pairs_out, void* stream) {
  if (!c) return VMAP_EINVAL;
  return render_scene(c, n_rays, rays_o, rays_d, n_objects, object_ids, S, t_min, occ_threshold,
                      max_pairs, scratch, scratch_bytes, depth_out, rgb_out, occ_out, id_out,
                      n_pairs_out, stream);
}

int vmap_render_scene_static(vmap_ctx* c, int32_t n_rays, const float* rays_o,
                             const float* rays_d, int32_t n_objects, const int32_t* object_ids,
                             int32_t S, float t_min, float occ_threshold, int32_t max_pairs,
                             float* depth_out, float* rgb_out, float* occ_out, int32_t* id_out,
                             int32_t* n_pairs_out, void* stream) {
  static_assert(VMAP_SCENE_STATIC_SCRATCH_BYTES == kStaticSceneScratchBytes,
                "the header states the static scratch's size");
  if (!c) return VMAP_EINVAL;
  if (n_rays > 0 && n_objects > 0 && S >= 1 && S <= kSlots && max_pairs >= 0 &&
      (int64_t)n_rays * n_objects <= ((int64_t)1 << 31) - 1) {
    const size_t need = scene_layout(n_rays, n_objects, max_pairs, S).total;
    if (need > kStaticSceneScratchBytes)
      return c->fail(VMAP_ECAPACITY,
                     "scene needs " + std::to_string(need) + " bytes of scratch, more than the " +
                         std::to_string(kStaticSceneScratchBytes) +
                         " of the static array (fewer rays, objects or max_pairs, or "
                         "vmap_render_scene with a caller scratch)");
  }
  void* ptr = static_scratch(c->device);
  if (!ptr) return c->fail(VMAP_ESTATE, "static scene scratch not set up on this context's GPU");
  return render_scene(c, n_rays, rays_o, rays_d, n_objects, object_ids, S, t_min, occ_threshold,
                      max_pairs, ptr, kStaticSceneScratchBytes, depth_out, rgb_out, occ_out,
                      id_out, n_pairs_out, stream);
}

int vmap_backward(vmap_ctx* c, const vmap_batch* b, const float* dloss, float* grad_out, void* stream) {
  if (!c) return VMAP_EINVAL;
  int rc = validate_batch(c, b, true);
  if (rc) return rc;
  if (!dloss && b->n_objects > 0) return c->fail(VMAP_EINVAL, "dloss must not be NULL");
  if (b->n_objects == 0) return VMAP_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((rc = enqueue_debug(c, b, s))) return rc;
  hipError_t e = enqueue_worklist(c, b, s);
  if (e != hipSuccess) return c->hip_fail(e, "worklist launch");
  rc = enqueue_tiles(c, b, MODE_TRAIN, dloss, nullptr, nullptr, nullptr, s, true);
  if (rc) return rc;
  e = launch_optimizer(OPT_REDUCE, make_opt_args(c, b, nullptr, grad_out), s);
  if (e != hipSuccess) return c->hip_fail(e, "gradient launch");
  return VMAP_OK;
}

int vmap_adam_step(vmap_ctx* c, const vmap_batch* b, void* stream) {
  if (!c) return VMAP_EINVAL;
  int rc = validate_batch(c, b, false);
  if (rc) return rc;
  if (b->n_objects == 0) return VMAP_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_optimizer(OPT_ADAM, make_opt_args(c, b, nullptr, nullptr), s);
  if (e != hipSuccess) return c->hip_fail(e, "adam launch");
  return VMAP_OK;
}

int vmap_query_occupancy(vmap_ctx* c, int32_t k, const float* pts, int64_t n, float* occ_out,
                         float* rgb_out, void* stream) {
  if (!c) return VMAP_EINVAL;
  if (k < 0 || k >= c->cfg.max_objects || !c->objs[k].registered)
    return c->fail(VMAP_ESTATE, "object id is not registered");
  if (n < 0) return c->fail(VMAP_EINVAL, "n must be >= 0");
  if (n == 0) return VMAP_OK;
  if (!pts || !occ_out) return c->fail(VMAP_EINVAL, "pts and occ_out must not be NULL");
  if (n > ((int64_t)1 << 40)) return c->fail(VMAP_EINVAL, "n too large");
  QueryArgs q{};
  q.pts = pts;
  q.n = n;
  q.k = k;
  q.theta = c->theta();
  q.p_stride = c->p_stride;
  q.desc = c->desc();
  q.B = c->B();
  q.occ = occ_out;
  q.rgb = rgb_out;
  const bool bf = c->cfg.precision == VMAP_BF16;
  const int H = kernel_width(c->objs[k].hidden);  // hidden 16: the width-32 kernel, zero-padded
  if (generic_width(H)) return c->fail(VMAP_ENOTSUP, "point queries of layered-path widths are not built");
  q.wimage = c->wimage();
  q.wimage_stride = (int64_t)c->wl.wimage_stride;
  q.max_objects = c->cfg.max_objects;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_query(H, bf, q, s);  // a hidden-128 object's image is current
  if (e != hipSuccess) return c->hip_fail(e, "query launch");
  return VMAP_OK;
}

int vmap_sample_rays(vmap_ctx* c, int32_t n_rays, int32_t S, int32_t n_strat, const float* t_near,
                     const float* t_far, const float* depth, float sigma, uint64_t seed,
                     float* t_out, void* stream) {
  if (!c) return VMAP_EINVAL;
  if (n_rays < 0) return c->fail(VMAP_EINVAL, "n_rays must be >= 0");
  if (S < 1 || S > kSlots) return c->fail(VMAP_EINVAL, "S must be in [1, 64]");
  if (n_strat < 0 || n_strat > S) return c->fail(VMAP_EINVAL, "n_strat must be in [0, S]");
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return c->fail(VMAP_EINVAL, "sigma must be finite and >= 0");
  if (n_rays == 0) return VMAP_OK;
  if (!t_near || !t_far || !depth || !t_out)
    return c->fail(VMAP_EINVAL, "t_near, t_far, depth and t_out must not be NULL");
  hipError_t e = launch_sample(n_rays, S, n_strat, t_near, t_far, depth, sigma, seed, t_out,
                               reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return c->hip_fail(e, "sampling launch");
  return VMAP_OK;
}

static int state_ptr(vmap_ctx* c, int32_t k, int32_t which, size_t bytes, void** dev) {
  if (which == VMAP_STATE_SCALER) {  // the context's loss scaler: scale (FP32), good steps (int32)
    static_assert(offsetof(ScalerState, good_steps) == 4, "scale and good_steps are adjacent");
    if (bytes != 8) return c->fail(VMAP_EINVAL, "scaler state is 8 bytes (float scale, int32 good steps)");
    *dev = c->scaler();
    return VMAP_OK;
  }
  if (k < 0 || k >= c->cfg.max_objects || !c->objs[k].registered)
    return c->fail(VMAP_ESTATE, "object id is not registered");
  const size_t P = (size_t)c->objs[k].n_params;
  float* base = nullptr;
  switch (which) {
    case VMAP_STATE_PARAMS: base = c->theta(); break;
    case VMAP_STATE_ADAM_M: base = c->m(); break;
    case VMAP_STATE_ADAM_V: base = c->v(); break;
    case VMAP_STATE_GRAD: base = c->grad(); break;
    case VMAP_STATE_STEP:
      if (bytes != 4) return c->fail(VMAP_EINVAL, "step count is 4 bytes (int32)");
      *dev = &c->desc()[k].step;
      return VMAP_OK;
    default: return c->fail(VMAP_EINVAL, "unknown state selector");
  }
  if (bytes != P * 4) return c->fail(VMAP_EINVAL, "bytes must equal 4 * n_params of the object");
  *dev = base + (size_t)k * c->p_stride;
  return VMAP_OK;
}

int vmap_get_state(vmap_ctx* c, int32_t k, int32_t which, void* host_dst, size_t bytes, void* stream) {
  if (!c) return VMAP_EINVAL;
  if (!host_dst) return c->fail(VMAP_EINVAL, "host_dst must not be NULL");
  void* dev = nullptr;
  int rc = state_ptr(c, k, which, bytes, &dev);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(host_dst, dev, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return c->hip_fail(e, "reading state");
  return VMAP_OK;
}

int vmap_set_state(vmap_ctx* c, int32_t k, int32_t which, const void* host_src, size_t bytes, void* stream) {
  if (!c) return VMAP_EINVAL;
  if (!host_src) return c->fail(VMAP_EINVAL, "host_src must not be NULL");
  void* dev = nullptr;
  int rc = state_ptr(c, k, which, bytes, &dev);
  if (rc) return rc;
  if (which == VMAP_STATE_SCALER) {
    float sc;
    int32_t good;
    std::memcpy(&sc, host_src, 4);
    std::memcpy(&good, static_cast<const char*>(host_src) + 4, 4);
    int e2 = 0;
    if (!(sc > 0.f) || !std::isfinite(sc) || std::frexp(sc, &e2) != 0.5f || e2 - 1 < -125 || e2 - 1 > 126 ||
        good < 0)
      return c->fail(VMAP_EINVAL, "scaler state: scale must be a power of two in [2^-125, 2^126], good steps >= 0");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(dev, host_src, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && which == VMAP_STATE_PARAMS) e = restage_image(c, k, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return c->hip_fail(e, "writing state");
  return VMAP_OK;
}

int vmap_step_info(vmap_ctx* c, float* loss_scale, int32_t* skipped, int32_t* device_error, void* stream) {
  if (!c) return VMAP_EINVAL;
  ScalerState h{};
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&h, c->scaler(), sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return c->hip_fail(e, "reading step info");
  if (loss_scale) *loss_scale = h.scale;
  if (skipped) *skipped = h.skipped;
  if (device_error) *device_error = h.device_error;
  return VMAP_OK;
}

int vmap_param_layout(const vmap_ctx* c, int32_t k, int32_t* n_params, int32_t* stride) {
  if (!c) return VMAP_EINVAL;
  if (k < 0 || k >= c->cfg.max_objects || !c->objs[k].registered) return VMAP_ESTATE;
  if (n_params) *n_params = c->objs[k].n_params;
  if (stride) *stride = c->p_stride;
  return VMAP_OK;
}

int vmap_set_graph_mode(vmap_ctx* c, int32_t enabled) {
  if (!c) return VMAP_EINVAL;
  c->graph_mode = enabled != 0;
  return VMAP_OK;
}

int vmap_set_launch(vmap_ctx* c, int32_t waves, int32_t grid_blocks) {
  if (!c) return VMAP_EINVAL;
  const int max_waves = c->cfg.precision == VMAP_BF16 ? 8 : 4;  // FP32 needs > 256 registers
  if (waves < 1 || waves > max_waves)
    return c->fail(VMAP_EINVAL, "waves_per_block must be in [1, 4] (FP32) or [1, 8] (BF16)");
  if (grid_blocks < 0) return c->fail(VMAP_EINVAL, "grid_blocks must be >= 0");
  c->waves = waves;
  c->grid_blocks = grid_blocks;
  return VMAP_OK;
}

int vmap_kernel_timing(vmap_ctx* c, int32_t enable, double* avg_ms, int32_t* count) {
  if (!c) return VMAP_EINVAL;
  double total = 0.0;
  int n = 0;
  for (auto& t : c->timed) {
    hipError_t e = hipEventSynchronize(t.b);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, t.a, t.b);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventElapsedTime");
    total += ms;
    ++n;
  }
  if (avg_ms) *avg_ms = n ? total / n : 0.0;
  if (count) *count = n;
  if (enable >= 0) {
    for (auto& t : c->timed) {
      c->event_pool.push_back(t.a);
      c->event_pool.push_back(t.b);
    }
    c->timed.clear();
    c->timing = enable != 0;
  }
  return VMAP_OK;
}

const char* vmap_last_error(const vmap_ctx* c) {
  if (!c) return g_init_error.c_str();
  return c->err.c_str();
}

void vmap_destroy(vmap_ctx* c) {
  if (!c) return;
  for (auto& kv : c->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  for (auto& t : c->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->join_ev) (void)hipEventDestroy(c->join_ev);
  for (int i = 0; i < vmap_ctx::kRing; ++i)
    if (c->ring_used[i]) (void)hipEventDestroy(c->ring_ev[i]);
  if (c->ring) (void)hipHostFree(c->ring);
  delete c;
}

}  // extern "C"
