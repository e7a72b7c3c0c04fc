// C ABI entry points: argument validation, workspace planning and kernel launches.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "common.h"

namespace gs {

// the last HIP error code seen by this thread's calls (gs_last_hip_error)
static thread_local int g_last_hip = 0;

int hip_status(hipError_t e) {
  if (e == hipSuccess) return GS_OK;
  g_last_hip = (int)e;
  return GS_ERR_HIP;
}
int launch_status() { return hip_status(hipGetLastError()); }

// kernels (other translation units)
int launch_preprocess(const gs_config&, const gs_gaussians&, const gs_view*, int, const gs_item*, const gs_projected&,
                      hipStream_t);
int launch_preprocess_bwd(const gs_config&, const gs_gaussians&, const gs_view*, int, const gs_item*, const float*,
                          const int32_t*, const gs_grads&, hipStream_t);
size_t bin_sort_workspace(int64_t E, int64_t cap, int64_t n_tiles);
int launch_bin_sort(const gs_config&, const gs_projected&, const gs_item*, int, int64_t, int, int64_t, void*, uint64_t*,
                    uint32_t*, uint32_t*, int64_t*, int32_t*, hipStream_t);
#define GS_RENDER_FWD_ARGS                                                                                 \
  const gs_config&, const gs_gaussians&, const gs_projected&, const gs_item*, int, int, const uint32_t*, \
      const uint32_t*, const gs_images&, hipStream_t
#define GS_RENDER_BWD_ARGS                                                                                 \
  const gs_config&, const gs_gaussians&, const gs_projected&, const gs_item*, int, int, const uint32_t*, \
      const uint32_t*, const gs_images&, const gs_images&, float*, const gs_grads&, hipStream_t
int launch_render_fwd_valu(GS_RENDER_FWD_ARGS);
int launch_render_bwd_valu(GS_RENDER_BWD_ARGS);
int launch_render_fwd_mfma(GS_RENDER_FWD_ARGS);
int launch_render_bwd_mfma(GS_RENDER_BWD_ARGS);
int launch_render_fwd_split(GS_RENDER_FWD_ARGS);
int launch_render_bwd_split(const gs_config&, const gs_gaussians&, const gs_projected&, const gs_item*, int, int,
                            const uint32_t*, const uint32_t*, const gs_images&, const gs_images&, float*,
                            const gs_grads&, void*, int64_t, hipStream_t);
size_t render_seg_workspace(int n_tiles, int64_t dup_capacity, int seg);
int64_t render_seg_capacity(int n_tiles, int seg, size_t bytes);
int render_seg_len(const gs_config& cfg);
size_t render_state_bytes(int n_tiles, int64_t dup_capacity, int K, int seg);
int64_t render_state_capacity(int n_tiles, int K, int seg, size_t bytes);

// Render kernel variants: 1 = per-lane FMA accumulation (VALU), 2 = single-precision
// matrix-core channel contraction, 3 = every contraction on the bfloat16 matrix cores with
// hi/lo split operands. 0 picks 3.
int launch_render_fwd(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items,
                      int n_items, int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& out,
                      hipStream_t s) {
  if (n_tiles == 0) return GS_OK;
  if (cfg.variant == 1) return launch_render_fwd_valu(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (cfg.variant == 2) return launch_render_fwd_mfma(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  return launch_render_fwd_split(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
}
int launch_render_bwd(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items,
                      int n_items, int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& fwd,
                      const gs_images& gin, float* g2d, const gs_grads& gr, void* seg_ws, int64_t cap,
                      hipStream_t s) {
  if (n_tiles == 0) return GS_OK;
  if (cfg.variant == 1)
    return launch_render_bwd_valu(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (cfg.variant == 2)
    return launch_render_bwd_mfma(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  return launch_render_bwd_split(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, seg_ws, cap, s);
}
int launch_loss(const gs_item*, int, int64_t, int, int, const float*, const float*, const gs_targets&, const gs_head*,
                const float*, float, float, float*, float*, float*, const gs_grads*, float*, hipStream_t);
int launch_downsample(const gs_item*, int, int64_t, int, int, float*, int32_t*, hipStream_t);
size_t loss_workspace(int n_items);
size_t head_bwd_workspace();
int head_shape_ok(const gs_head&);
int launch_head_fwd(const gs_item*, int, int64_t, int, const gs_head&, const float*, float*, hipStream_t);
int launch_head_bwd(const gs_item*, int, int64_t, int, const gs_head&, const float*, const float*, float*, float*,
                    float*, float*, float*, float*, hipStream_t);
int launch_adam(float*, const float*, float*, float*, int64_t, float, float, float, float, int, uint16_t*, hipStream_t);
int launch_gaussians_adam(int64_t, int, const gs_param_arrays&, const gs_grads&, const gs_param_arrays&,
                          const gs_param_arrays&, const gs_adam_config&, int, hipStream_t);
int launch_pose_adam(gs_view*, int, const float*, float*, float*, const gs_adam_config&, int, hipStream_t);
int launch_pose_perturb(const gs_view*, int, const float*, gs_view*, hipStream_t);
int launch_pose_perturb_bwd(const float*, int, const float*, float*, hipStream_t);
int launch_sh_fwd(const gs_gaussians&, const gs_sh&, int, const gs_view*, int, float*, float*, hipStream_t);
int launch_sh_bwd(const gs_gaussians&, const gs_sh&, int, const gs_view*, int, const float*, const float*, float*,
                  float*, float*, float*, float*, float*, hipStream_t);
int launch_distill(const gs_item*, int, int64_t, int, const float*, const float*, float, float*, float*, float*,
                   hipStream_t);
int launch_agree(const gs_item*, int, int64_t, int, const float*, const float*, unsigned long long*, hipStream_t);
int launch_fill_f32(float*, int64_t, float, hipStream_t);
int launch_zero_f32(float* const* p, const int64_t* n, int count, hipStream_t s);

namespace {

bool cfg_ok(const gs_config* c) {
  if (!c) return false;
  // 256-pixel tiles: 8x32, 16x16, 32x8 or 64x4
  if (!((c->tile_w == 8 || c->tile_w == 16 || c->tile_w == 32 || c->tile_w == 64) && c->tile_w * c->tile_h == kTilePx))
    return false;
  if (!(c->z_near > 0.0f) || !(c->eps_dilate >= 0.0f) || !(c->alpha_min >= 0.0f)) return false;
  if (!(c->alpha_max > c->alpha_min) || !(c->alpha_max < 1.0f) || !(c->t_min >= 0.0f) || !(c->guard > 0.0f)) return false;
  if (c->n_sem < 0 || c->n_sem > 60) return false;
  if (c->variant < 0 || c->variant > 3) return false;
  if (c->tile_order < 0 || c->tile_order > 1) return false;
  if (c->fwd_chunk < 0 || c->fwd_chunk > 65535) return false;
  if (!(c->ssim_lambda >= 0.0f && c->ssim_lambda <= 1.0f)) return false;
  if (!(c->sem_ssim_lambda >= 0.0f && c->sem_ssim_lambda <= 1.0f)) return false;
  if (c->isotropic < 0 || c->isotropic > 1) return false;
  if (c->view_features < 0 || c->view_features > 1) return false;
  // segments of split lists: the forward's state is sized for 256-entry ones
  if (c->seg_len != 0 && (c->seg_len < 256 || c->seg_len > (1 << 20) || c->seg_len % 32 != 0)) return false;
  if (c->sort_mode < 0 || c->sort_mode > 2) return false;
  return true;
}

bool gauss_ok(const gs_gaussians* g, bool need_features) {
  if (!g || g->n < 0 || g->n >= (int64_t)1 << 31) return false;
  if (g->n == 0) return true;
  if (!g->mean || !g->log_scale || !g->quat || !g->opacity) return false;
  if (need_features && !g->rgb) return false;
  return true;
}

constexpr int64_t kSortBwdRecord = 8;  // floats per (item, Gaussian) of 2D gradients

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

void gs_config_default(gs_config* c) {
  if (!c) return;
  c->tile_w = kTile;
  c->tile_h = kTile;
  c->z_near = 0.2f;
  c->eps_dilate = 0.3f;
  c->alpha_min = 1.0f / 255.0f;
  c->alpha_max = 0.99f;
  c->t_min = 1e-4f;
  c->guard = 1.3f;
  c->full_rect = 0;
  c->n_sem = 0;
  c->variant = 0;
  c->tile_order = 0;
  c->fwd_chunk = 0;
  c->ssim_lambda = 0.0f;
  c->isotropic = 0;
  c->view_features = 0;
  c->sem_ssim_lambda = 0.0f;
  c->seg_len = 0;
  c->sort_mode = 0;
}

const char* gs_status_string(int s) {
  switch (s) {
    case GS_OK: return "ok";
    case GS_ERR_INVALID_ARG: return "invalid argument";
    case GS_ERR_WORKSPACE: return "workspace too small";
    case GS_ERR_CAPACITY: return "duplicate capacity exceeded";
    case GS_ERR_HIP: return "HIP error";
    case GS_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

int gs_last_hip_error(void) { return g_last_hip; }
int gs_version(void) { return 100; }

int gs_make_items(const gs_config* cfg, int32_t n_views, gs_view* views, const int32_t* W, const int32_t* H,
                  const float* K, const int32_t* levels, gs_item* items, int64_t* n_pixels, int32_t* n_tiles) {
  if (!cfg_ok(cfg) || n_views < 0 || !views || !W || !H || !K || !levels || !items) return GS_ERR_INVALID_ARG;
  int n = 0;
  int64_t pix = 0;
  int64_t tiles = 0;
  for (int v = 0; v < n_views; ++v) {
    const int L = levels[v];
    if (L < 1 || L > 16 || W[v] <= 0 || H[v] <= 0) return GS_ERR_INVALID_ARG;
    const int div = 1 << (L - 1);
    if (W[v] % div || H[v] % div) return GS_ERR_INVALID_ARG;
    views[v].item_first = n;
    views[v].item_count = L;
    for (int l = 0; l < L; ++l) {
      gs_item& it = items[n++];
      const float s = std::ldexp(1.0f, -l);
      it.fx = K[4 * v + 0] * s;
      it.fy = K[4 * v + 1] * s;
      it.cx = K[4 * v + 2] * s;
      it.cy = K[4 * v + 3] * s;
      it.W = W[v] >> l;
      it.H = H[v] >> l;
      it.view = v;
      it.level = l;
      it.tiles_x = (it.W + cfg->tile_w - 1) / cfg->tile_w;
      it.tiles_y = (it.H + cfg->tile_h - 1) / cfg->tile_h;
      it.tile_base = (int32_t)tiles;
      it.pad = 0;
      it.pixel_base = pix;
      tiles += (int64_t)it.tiles_x * it.tiles_y;
      pix += (int64_t)it.W * it.H;
      if (tiles >= (int64_t)1 << 31) return GS_ERR_INVALID_ARG;
    }
  }
  if (n_pixels) *n_pixels = pix;
  if (n_tiles) *n_tiles = (int32_t)tiles;
  return n;
}

int gs_workspace_size(int kind, const gs_config* cfg, int32_t n_items, int64_t n_gauss, int32_t n_tiles,
                      int64_t dup_capacity, int64_t n_pixels, size_t* bytes) {
  if (!cfg_ok(cfg) || !bytes || n_items < 0 || n_gauss < 0 || n_tiles < 0 || dup_capacity < 0 || n_pixels < 0)
    return GS_ERR_INVALID_ARG;
  switch (kind) {
    case GS_WS_BIN_SORT:
      *bytes = bin_sort_workspace((int64_t)n_items * n_gauss, dup_capacity, n_tiles);
      return GS_OK;
    case GS_WS_RENDER_BWD:
      *bytes = align_up(sizeof(float) * kSortBwdRecord * (size_t)n_items * (size_t)n_gauss) + align_up(head_bwd_workspace()) +
               render_seg_workspace(n_tiles, dup_capacity, render_seg_len(*cfg));
      return GS_OK;
    case GS_WS_LOSS:
      *bytes = align_up(loss_workspace(n_items));
      return GS_OK;
    case GS_WS_RENDER_STATE:
      *bytes = render_state_bytes(n_tiles, dup_capacity, 4 + cfg->n_sem, render_seg_len(*cfg));
      return GS_OK;
    default:
      return GS_ERR_INVALID_ARG;
  }
}

int gs_preprocess(const gs_config* cfg, const gs_gaussians* g, const gs_view* views_dev, int32_t n_views,
                  const gs_item* items_dev, int32_t n_items, gs_projected* out, void* stream) {
  if (!cfg_ok(cfg) || !gauss_ok(g, false) || !out || n_views < 0 || n_items < 0) return GS_ERR_INVALID_ARG;
  if (g->n == 0 || n_items == 0) return GS_OK;
  if (!views_dev || !items_dev || !out->rec || !out->depth || !out->radius) return GS_ERR_INVALID_ARG;
  if ((int64_t)n_items * g->n >= (int64_t)1 << 32) return GS_ERR_UNSUPPORTED;
  return launch_preprocess(*cfg, *g, views_dev, n_views, items_dev, *out, (hipStream_t)stream);
}

int gs_bin_sort(const gs_config* cfg, const gs_projected* proj, const gs_item* items_dev, int32_t n_items,
                int64_t n_gauss, int32_t n_tiles, int64_t dup_capacity, void* workspace, size_t ws_bytes,
                uint64_t* keys, uint32_t* vals, uint32_t* ranges, int64_t* n_dup_dev, int32_t* status_dev,
                void* stream) {
  if (!cfg_ok(cfg) || !proj || n_items < 0 || n_gauss < 0 || n_tiles < 0 || dup_capacity < 0) return GS_ERR_INVALID_ARG;
  if (dup_capacity >= ((int64_t)1 << 32) - 1 || (int64_t)n_items * n_gauss >= (int64_t)1 << 32) return GS_ERR_UNSUPPORTED;
  if (n_tiles == 0) return GS_OK;
  if (!items_dev || !vals || !ranges) return GS_ERR_INVALID_ARG;
  if (n_items > 0 && n_gauss > 0 && (!proj->rec || !proj->depth || !proj->radius)) return GS_ERR_INVALID_ARG;
  if (ws_bytes < bin_sort_workspace((int64_t)n_items * n_gauss, dup_capacity, n_tiles) || !workspace) return GS_ERR_WORKSPACE;
  return launch_bin_sort(*cfg, *proj, items_dev, n_items, n_gauss, n_tiles, dup_capacity, workspace, keys, vals, ranges,
                         n_dup_dev, status_dev, (hipStream_t)stream);
}

int gs_render_fwd(const gs_config* cfg, const gs_gaussians* g, const gs_projected* proj, const gs_item* items_dev,
                  int32_t n_items, int32_t n_tiles, const uint32_t* vals, const uint32_t* ranges,
                  const gs_head* head, gs_images* out, void* stream) {
  if (!cfg_ok(cfg) || !gauss_ok(g, true) || !proj || !out || n_items < 0 || n_tiles < 0) return GS_ERR_INVALID_ARG;
  const bool learned = g->emb != nullptr;
  if (learned && cfg->n_sem != 16) return GS_ERR_INVALID_ARG;
  if (head && (!learned || !head_shape_ok(*head) || !out->logits || out->n_pixels < 0 || !items_dev))
    return GS_ERR_INVALID_ARG;
  if (learned && cfg->view_features) return GS_ERR_INVALID_ARG;
  if (!learned && cfg->n_sem > 0 && g->n > 0 && !g->sem) return GS_ERR_INVALID_ARG;
  if (n_tiles > 0) {
    if (!items_dev || !vals || !ranges || !out->color || !out->T || !out->n_contrib) return GS_ERR_INVALID_ARG;
    if (out->state && render_state_capacity(n_tiles, 4 + cfg->n_sem, render_seg_len(*cfg), out->state_bytes) < 0)
      return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  int st = launch_render_fwd(*cfg, *g, *proj, items_dev, n_items, n_tiles, vals, ranges, *out, s);
  if (st || !head) return st;
  return launch_head_fwd(items_dev, n_items, out->n_pixels, 4 + cfg->n_sem, *head, out->color, out->logits, s);
}

// Argument checks of gs_pyramid_loss other than the workspace's.
static int loss_args(const gs_config* cfg, const gs_item* items_dev, int32_t n_items, int64_t n_pixels,
                     int32_t n_classes, const gs_images* rendered, const gs_targets* targets, const gs_head* head,
                     const float* w, const float* loss_dev, const gs_images* grad_out, const gs_grads* head_grads) {
  if (!cfg_ok(cfg) || n_items < 0 || n_pixels < 0 || n_classes < 0 || !rendered || !targets || !w || !grad_out)
    return GS_ERR_INVALID_ARG;
  if (n_items == 0) return GS_OK;
  if (!items_dev || !loss_dev || !rendered->color || !grad_out->color || !targets->rgb || !targets->depth)
    return GS_ERR_INVALID_ARG;
  if (targets->sem_color) {
    // eq. 12: the semantic feature is a 3-channel colour, composited as channels 4..6
    if (cfg->n_sem != 3 || n_classes != 0 || head || rendered->logits) return GS_ERR_INVALID_ARG;
    return GS_OK;
  }
  if (n_classes > 0 && !targets->label) return GS_ERR_INVALID_ARG;
  if (head) {
    // the decode inside the loss: the embedding channels in, the head's gradients out
    if (cfg->n_sem != 16 || !head_shape_ok(*head) || head->n_classes != n_classes || !head_grads ||
        !head_grads->head_W1 || !head_grads->head_b1 || !head_grads->head_W2 || !head_grads->head_b2)
      return GS_ERR_INVALID_ARG;
  } else if (rendered->logits) {
    if (!grad_out->logits) return GS_ERR_INVALID_ARG;
  } else if (n_classes != cfg->n_sem) {
    return GS_ERR_INVALID_ARG;
  }
  return GS_OK;
}

int gs_pyramid_loss(const gs_config* cfg, const gs_item* items_dev, int32_t n_items, int64_t n_pixels,
                    int32_t n_classes, const gs_images* rendered, const gs_targets* targets, const gs_head* head,
                    const float* w, float* loss_dev, gs_images* grad_out, gs_grads* head_grads, void* workspace,
                    size_t ws_bytes, void* stream) {
  const int st = loss_args(cfg, items_dev, n_items, n_pixels, n_classes, rendered, targets, head, w, loss_dev,
                           grad_out, head_grads);
  if (st != GS_OK || n_items == 0) return st;
  if (!workspace || ws_bytes < loss_workspace(n_items)) return GS_ERR_WORKSPACE;
  return launch_loss(items_dev, n_items, n_pixels, 4 + cfg->n_sem, n_classes, rendered->color,
                     head ? nullptr : rendered->logits, *targets, head, w, cfg->ssim_lambda,
                     targets->sem_color ? cfg->sem_ssim_lambda : 0.0f, loss_dev, grad_out->color,
                     head ? nullptr : grad_out->logits, head_grads, (float*)workspace, (hipStream_t)stream);
}

// ---- the loss with library-held scratch ----------------------------------------
// gs_pyramid_loss_static runs gs_pyramid_loss's kernels with the workspace taken from this
// file-scope device array instead of a caller buffer, for callers that cannot allocate.
// Each GPU holds its own copy; its address is looked up once per device (the array's name
// is a host-side stand-in, never passed to a kernel).
constexpr size_t kLossScratchBytes = (size_t)16 << 20;
constexpr int32_t kLossScratchItems = 2048;
static __device__ __align__(256) unsigned char scratch[kLossScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on the calling thread's current device (nullptr and a
// recorded HIP error if it cannot be had).
void* scratch_on_current_device() {
  int dev = -1;
  if (hip_status(hipGetDevice(&dev)) != GS_OK || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hip_status(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != GS_OK) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int gs_pyramid_loss_static(const gs_config* cfg, const gs_item* items_dev, int32_t n_items,
                                      int64_t n_pixels, int32_t n_classes, const gs_images* rendered,
                                      const gs_targets* targets, const gs_head* head, const float* w, float* loss_dev,
                                      gs_images* grad_out, gs_grads* head_grads, void* stream) {
  const int st = loss_args(cfg, items_dev, n_items, n_pixels, n_classes, rendered, targets, head, w, loss_dev,
                           grad_out, head_grads);
  if (st != GS_OK || n_items == 0) return st;
  // more items than the scratch array holds the per-item sums of: refused before any launch
  if (n_items > kLossScratchItems || loss_workspace(n_items) > kLossScratchBytes) return GS_ERR_WORKSPACE;
  void* ws = scratch_on_current_device();
  if (!ws) return GS_ERR_HIP;
  return gs_pyramid_loss(cfg, items_dev, n_items, n_pixels, n_classes, rendered, targets, head, w, loss_dev, grad_out,
                         head_grads, ws, kLossScratchBytes, stream);
}

int gs_render_bwd(const gs_config* cfg, const gs_gaussians* g, const gs_projected* proj, const gs_view* views_dev,
                  int32_t n_views, const gs_item* items_dev, int32_t n_items, int32_t n_tiles,
                  const uint32_t* vals, const uint32_t* ranges, const gs_head* head, const gs_images* fwd,
                  const gs_images* grad_in, gs_grads* grads, void* workspace, size_t ws_bytes, void* stream) {
  // every argument is checked before the first launch: an invalid call enqueues nothing
  if (!cfg_ok(cfg) || !gauss_ok(g, true) || !proj || !fwd || !grad_in || !grads || n_views < 0 || n_items < 0 ||
      n_tiles < 0)
    return GS_ERR_INVALID_ARG;
  const bool learned = g->emb != nullptr;
  if (learned && (cfg->n_sem != 16 || !grads->emb)) return GS_ERR_INVALID_ARG;
  // with a head, the decode's logit gradient is taken back through it; without, the
  // embedding channels' gradient is used as given (and no logit gradient may be passed)
  if (head && (!learned || !head_shape_ok(*head) || !grads->head_W1 || !grads->head_b1 || !grads->head_W2 ||
               !grads->head_b2 || !fwd->color || !grad_in->logits || !grad_in->color || fwd->n_pixels < 0 ||
               !items_dev))
    return GS_ERR_INVALID_ARG;
  if (learned && !head && grad_in->logits) return GS_ERR_INVALID_ARG;
  if (learned && cfg->view_features) return GS_ERR_INVALID_ARG;
  if (!learned && cfg->n_sem > 0 && g->n > 0 && (!g->sem || !grads->sem)) return GS_ERR_INVALID_ARG;
  if (!grads->mean || !grads->log_scale || !grads->quat || !grads->opacity || !grads->rgb || !grads->pose)
    return GS_ERR_INVALID_ARG;
  if (g->n > 0 && n_items > 0 && (!views_dev || !items_dev || !proj->rec || !proj->radius)) return GS_ERR_INVALID_ARG;
  const bool render = g->n > 0 && n_tiles > 0;
  if (render) {
    if (!items_dev || !vals || !ranges || !fwd->T || !fwd->n_contrib || !grad_in->color) return GS_ERR_INVALID_ARG;
    if (fwd->state && render_state_capacity(n_tiles, 4 + cfg->n_sem, render_seg_len(*cfg), fwd->state_bytes) < 0)
      return GS_ERR_WORKSPACE;
  }
  const size_t rec_bytes = align_up(sizeof(float) * kSortBwdRecord * (size_t)n_items * (size_t)g->n);
  const size_t head_bytes = align_up(head_bwd_workspace());
  if (!workspace || ws_bytes < rec_bytes + head_bytes) return GS_ERR_WORKSPACE;
  // the rest holds the segment work list of the reverse pass, sized for a duplicate
  // capacity (0 still works: every tile is then one work item)
  const int64_t cap = render_seg_capacity(n_tiles, render_seg_len(*cfg), ws_bytes - rec_bytes - head_bytes);
  if (cap < 0) return GS_ERR_WORKSPACE;
  void* seg_ws = (char*)workspace + rec_bytes + head_bytes;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = g->n;
  gs_grads gr = *grads;
  if (learned) gr.sem = grads->emb;   // the semantic channels' gradient is the embedding's
  float* const zp[4] = {(float*)workspace, gr.rgb, cfg->n_sem > 0 ? gr.sem : nullptr, gr.pose};
  const int64_t fv = cfg->view_features ? n_views : 1;   // feature blocks (one per view, or shared)
  const int64_t zn[4] = {kSortBwdRecord * (int64_t)n_items * n, 3 * n * fv, (int64_t)cfg->n_sem * n * fv, 6ll * n_views};
  int st = launch_zero_f32(zp, zn, 4, s);
  if (st) return st;
  if (head) {
    st = launch_head_bwd(items_dev, n_items, fwd->n_pixels, 4 + cfg->n_sem, *head, fwd->color, grad_in->logits,
                         grad_in->color, (float*)((char*)workspace + rec_bytes), gr.head_W1, gr.head_b1, gr.head_W2,
                         gr.head_b2, s);
    if (st) return st;
  }
  if (n == 0) return GS_OK;
  if (render) {
    st = launch_render_bwd(*cfg, *g, *proj, items_dev, n_items, n_tiles, vals, ranges, *fwd, *grad_in, (float*)workspace,
                           gr, seg_ws, cap, s);
    if (st) return st;
  }
  return launch_preprocess_bwd(*cfg, *g, views_dev, n_views, items_dev, (const float*)workspace, proj->radius, gr, s);
}

int gs_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                 float eps, int32_t step, uint16_t* bf16_copy, void* stream) {
  if (n < 0 || step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return GS_ERR_INVALID_ARG;
  if (n > 0 && (!param || !grad || !m || !v)) return GS_ERR_INVALID_ARG;
  return launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, step, bf16_copy, (hipStream_t)stream);
}

static bool sh_ok(int32_t n_sem, const gs_gaussians* g, const gs_sh* sh) {
  if (!sh || !g || g->n < 0 || n_sem < 0 || n_sem > 60) return false;
  if (sh->rgb_degree < 0 || sh->rgb_degree > 3 || sh->sem_degree < 0 || sh->sem_degree > 3) return false;
  if (g->emb) return false;   // plain semantics only
  if (g->n == 0) return true;
  if (!g->mean || !g->rgb || (n_sem > 0 && !g->sem)) return false;
  if (sh->rgb_degree > 0 && !sh->rgb_rest) return false;
  if (n_sem > 0 && sh->sem_degree > 0 && !sh->sem_rest) return false;
  return true;
}

int gs_sh_features(int32_t n_sem, const gs_gaussians* g, const gs_sh* sh, const gs_view* views_dev, int32_t n_views,
                   float* rgb_out, float* sem_out, void* stream) {
  if (!sh_ok(n_sem, g, sh) || n_views < 0) return GS_ERR_INVALID_ARG;
  if (g->n == 0 || n_views == 0) return GS_OK;
  if (!views_dev || !rgb_out || (n_sem > 0 && !sem_out)) return GS_ERR_INVALID_ARG;
  return launch_sh_fwd(*g, *sh, n_sem, views_dev, n_views, rgb_out, sem_out, (hipStream_t)stream);
}

int gs_sh_features_bwd(int32_t n_sem, const gs_gaussians* g, const gs_sh* sh, const gs_view* views_dev,
                       int32_t n_views, const float* grad_rgb, const float* grad_sem, float* grad_rgb_dc,
                       float* grad_rgb_rest, float* grad_sem_dc, float* grad_sem_rest, float* grad_mean,
                       float* grad_pose, void* stream) {
  if (!sh_ok(n_sem, g, sh) || n_views < 0) return GS_ERR_INVALID_ARG;
  if (g->n == 0) return GS_OK;
  if (n_views > 0 && (!views_dev || !grad_rgb || (n_sem > 0 && !grad_sem))) return GS_ERR_INVALID_ARG;
  const bool dir = (sh->rgb_degree > 0 || (n_sem > 0 && sh->sem_degree > 0)) && n_views > 0;
  if (dir && (!grad_mean || !grad_pose)) return GS_ERR_INVALID_ARG;
  if (n_views == 0) return GS_ERR_INVALID_ARG;   // the constant-band gradient is a sum over views
  gs_sh s = *sh;
  if (n_sem == 0) s.sem_degree = 0;
  return launch_sh_bwd(*g, s, n_sem, views_dev, n_views, grad_rgb, grad_sem, grad_rgb_dc, grad_rgb_rest, grad_sem_dc,
                       grad_sem_rest, grad_mean, grad_pose, (hipStream_t)stream);
}

static bool adam_ok(const gs_adam_config* hp, int32_t step) {
  if (!hp || step < 1) return false;
  if (!(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) || !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) || !(hp->eps > 0.0f))
    return false;
  const float lr[8] = {hp->lr_mean, hp->lr_log_scale, hp->lr_quat, hp->lr_opacity, hp->lr_rgb, hp->lr_sem,
                       hp->lr_rho, hp->lr_phi};
  for (float x : lr)
    if (!(x >= 0.0f) || !std::isfinite(x)) return false;
  return true;
}

int gs_gaussians_adam(int64_t n, int32_t n_sem, const gs_param_arrays* params, const gs_grads* grads,
                      const gs_param_arrays* m, const gs_param_arrays* v, const gs_adam_config* hp, int32_t step,
                      void* stream) {
  if (n < 0 || n_sem < 0 || n_sem > 60 || !params || !grads || !m || !v || !adam_ok(hp, step)) return GS_ERR_INVALID_ARG;
  if (n == 0) return GS_OK;
  const float lr[6] = {hp->lr_mean, hp->lr_log_scale, hp->lr_quat, hp->lr_opacity, hp->lr_rgb, hp->lr_sem};
  const float* P[6] = {params->mean, params->log_scale, params->quat, params->opacity, params->rgb, params->sem};
  const float* G[6] = {grads->mean, grads->log_scale, grads->quat, grads->opacity, grads->rgb, grads->sem};
  const float* M[6] = {m->mean, m->log_scale, m->quat, m->opacity, m->rgb, m->sem};
  const float* V[6] = {v->mean, v->log_scale, v->quat, v->opacity, v->rgb, v->sem};
  for (int k = 0; k < 6; ++k) {
    if (lr[k] == 0.0f || (k == 5 && n_sem == 0)) continue;
    if (!P[k] || !G[k] || !M[k] || !V[k]) return GS_ERR_INVALID_ARG;
  }
  return launch_gaussians_adam(n, n_sem, *params, *grads, *m, *v, *hp, step, (hipStream_t)stream);
}

int gs_pose_adam(gs_view* views_dev, int32_t n_views, const float* grad_pose, float* m, float* v,
                 const gs_adam_config* hp, int32_t step, void* stream) {
  if (n_views < 0 || !adam_ok(hp, step)) return GS_ERR_INVALID_ARG;
  if (n_views == 0) return GS_OK;
  if (!views_dev || !grad_pose || !m || !v) return GS_ERR_INVALID_ARG;
  return launch_pose_adam(views_dev, n_views, grad_pose, m, v, *hp, step, (hipStream_t)stream);
}

int gs_pose_perturb(const gs_view* views_in, int32_t n_views, const float* xi, gs_view* views_out, void* stream) {
  if (n_views < 0) return GS_ERR_INVALID_ARG;
  if (n_views == 0) return GS_OK;
  if (!views_in || !xi || !views_out) return GS_ERR_INVALID_ARG;
  return launch_pose_perturb(views_in, n_views, xi, views_out, (hipStream_t)stream);
}

int gs_pose_perturb_bwd(const float* xi, int32_t n_views, const float* grad_pose, float* grad_xi, void* stream) {
  if (n_views < 0) return GS_ERR_INVALID_ARG;
  if (n_views == 0) return GS_OK;
  if (!xi || !grad_pose || !grad_xi || grad_pose == grad_xi) return GS_ERR_INVALID_ARG;
  return launch_pose_perturb_bwd(xi, n_views, grad_pose, grad_xi, (hipStream_t)stream);
}

int gs_distill_loss(const gs_item* items_dev, int32_t n_items, int64_t n_pixels, int32_t C, const float* teacher,
                    const float* student, float mse_w, float* loss_dev, float* grad, void* workspace, size_t ws_bytes,
                    void* stream) {
  if (n_items <= 0 || n_pixels < 0 || C < 1 || !items_dev || !teacher || !student || !loss_dev || !grad)
    return GS_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < 256) return GS_ERR_WORKSPACE;
  return launch_distill(items_dev, n_items, n_pixels, C, teacher, student, mse_w, loss_dev, grad, (float*)workspace,
                        (hipStream_t)stream);
}

int gs_argmax_agreement(const gs_item* items_dev, int32_t n_items, int64_t n_pixels, int32_t C, const float* a,
                        const float* b, uint64_t* counts_dev, void* stream) {
  if (n_items <= 0 || n_pixels < 0 || C < 1 || !items_dev || !a || !b || !counts_dev) return GS_ERR_INVALID_ARG;
  return launch_agree(items_dev, n_items, n_pixels, C, a, b, (unsigned long long*)counts_dev, (hipStream_t)stream);
}

int gs_graph_begin(void* stream) {
  if (!stream) return GS_ERR_INVALID_ARG;  // the legacy null stream cannot be captured
  return hip_status(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeRelaxed));
}

int gs_graph_end(void* stream, void** graph_exec) {
  if (!stream || !graph_exec) return GS_ERR_INVALID_ARG;
  hipGraph_t graph = nullptr;
  int st = hip_status(hipStreamEndCapture((hipStream_t)stream, &graph));
  if (st) return st;
  hipGraphExec_t exec = nullptr;
  st = hip_status(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  // the captured graph is not needed once instantiated
  const int dst = hip_status(hipGraphDestroy(graph));
  if (st) return st;
  if (dst) {
    (void)hipGraphExecDestroy(exec);
    return dst;
  }
  *graph_exec = (void*)exec;
  return GS_OK;
}

int gs_graph_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return GS_ERR_INVALID_ARG;
  return hip_status(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream));
}

int gs_graph_destroy(void* graph_exec) {
  if (!graph_exec) return GS_OK;
  return hip_status(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
}

int gs_pyramid_downsample(const gs_item* items_dev, int32_t n_items, int64_t n_pixels, int32_t max_level, int32_t K,
                          float* img, int32_t* labels, void* stream) {
  if (n_items < 0 || n_pixels < 0 || max_level < 0 || K < 4) return GS_ERR_INVALID_ARG;
  if (n_items == 0 || n_pixels == 0) return GS_OK;
  if (!items_dev || !img) return GS_ERR_INVALID_ARG;
  return launch_downsample(items_dev, n_items, n_pixels, max_level, K, img, labels, (hipStream_t)stream);
}

}  // extern "C"
