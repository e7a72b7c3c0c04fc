/*
 * gs.h -- C ABI of the MI355X (gfx950) pyramid Gaussian-splatting rasterizer.
 *
 * The library renders RGB, depth and per-class semantics from 3D Gaussians at
 * every level of an image pyramid, computes the per-level reconstruction loss,
 * and back-propagates it to every Gaussian parameter and to an SE(3) tangent of
 * every camera pose (RGBDS-SLAM, Sec. III-B to III-D, eq. 1-13).
 *
 * Conventions shared by every entry point
 *  - All pointers named *_dev, and every pointer inside the structs below, are
 *    device pointers (hipMalloc'd or torch-owned GPU memory) unless stated.
 *    The caller owns every buffer, including workspaces; the library never
 *    allocates, frees or waits on the host inside a call.
 *  - `stream` is a hipStream_t passed as void*. Every call only enqueues work on
 *    it and returns; results are ready when the stream is.
 *  - Return value: GS_OK (0) or a negative gs_status. Argument errors are
 *    detected on the host before anything is enqueued. No C++ exception crosses
 *    the ABI. The hot-path functions keep no state between calls (launch sizes
 *    are derived from the calling thread's current device at every call); the
 *    only state is the last HIP error code, kept per thread for gs_last_hip_error().
 *  - Work item ("item"): one (view, pyramid level) pair. Level l of a view with
 *    base size W x H has size (W >> l) x (H >> l) and intrinsics
 *    fx/2^l, fy/2^l, cx/2^l, cy/2^l (Sec. III-C, eq. 4-6: the pyramid).
 *    Items of one view are contiguous, in level order.
 *  - Images are planar per item: channel c of pixel (x, y) of item i lives at
 *    [pixel_base_i * C + c * W_i * H_i + y * W_i + x] for a C-channel image.
 *    Pixel (x, y) is sampled at (x + 1/2, y + 1/2).
 *  - Rendered channels: 0-2 RGB (eq. 7), 3 depth (eq. 8), 4.. semantics (eq. 9):
 *    n_sem class logits (plain mode) or the 16-wide embedding (learned mode).
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gs_status {
  GS_OK = 0,
  GS_ERR_INVALID_ARG = -1,   /* a size, pointer or config field is out of range */
  GS_ERR_WORKSPACE = -2,     /* workspace smaller than gs_workspace_size() asks */
  GS_ERR_CAPACITY = -3,      /* reported through status_dev: duplicates > capacity */
  GS_ERR_HIP = -4,           /* a HIP launch failed; gs_last_hip_error() has the code */
  GS_ERR_UNSUPPORTED = -5    /* valid, but not built into this library */
} gs_status;

/* Rasterizer configuration. gs_config_default() fills the values listed. */
typedef struct gs_config {
  int32_t tile_w, tile_h;  /* 16, 16: screen tile of 256 pixels: 8x32, 16x16, 32x8 or 64x4 */
  float z_near;            /* 0.2: cull Gaussians whose camera depth <= z_near */
  float eps_dilate;        /* 0.3: added to the 2D covariance diagonal (px^2) */
  float alpha_min;         /* 1/255: a Gaussian is skipped where alpha < alpha_min */
  float alpha_max;         /* 0.99: alpha is clamped to alpha_max */
  float t_min;             /* 1e-4: a pixel stops before T would fall below t_min */
  float guard;             /* 1.3: x/z, y/z clamped to +-guard*(W/2)/fx inside J */
  int32_t full_rect;       /* 0; 1 = every Gaussian covers every tile of its item */
  int32_t n_sem;           /* composited semantic channels, 0..60 (plain: classes; learned: 16) */
  int32_t variant;         /* render kernels: 0 automatic (= 3), 1 per-lane FMA (VALU), 2 single-precision
                              matrix cores, 3 bfloat16 matrix cores with hi/lo split operands
                              (single-precision accurate to about 2^-16 relative) */
  int32_t tile_order;      /* 0: coarse pyramid levels (longest tile lists) launched first; 1: item order */
  int32_t fwd_chunk;       /* 0: forward with a state (gs_images.state), variant 3: segments (seg_len)
                              walked per work item, 1..65535 (a transmittance pre-pass gives every
                              chunk but a list's first its starting T), or 0 = whole lists */
  float ssim_lambda;       /* 0: weight lambda of the SSIM term of the colour loss (eq. 10, read as
                              (1 - lambda) L1 + lambda (1 - SSIM)), 0..1; the paper trains with 0.2 */
  int32_t isotropic;       /* 0: EWA footprint of scale x rotation; 1: the literal primitive of eq. 1-3,
                              one scale r = exp(log_scale[0]) projected to standard deviation f r / d
                              along each image axis (plus eps_dilate); quat and log_scale[1..2] are
                              then unused and get zero gradient */
  int32_t view_features;   /* 0: g->rgb [n][3] and g->sem [n][n_sem] are shared by all views;
                              1: one block per view, [n_views][n][3] and [n_views][n][n_sem] (e.g.
                              view-dependent colours from gs_sh_features), and gs_render_bwd's
                              grads->rgb / grads->sem have the same per-view layout. Plain
                              semantics only (not with an embedding) */
  float sem_ssim_lambda;   /* 0: weight lambda_s of the SSIM term of the semantic colour loss (eq. 12,
                              read as (1 - lambda_s) L1 + lambda_s (1 - SSIM)), 0..1, used when the
                              targets carry a semantic colour image; the paper trains with 0.2 */
  int32_t seg_len;         /* 0: list positions per segment of a long tile list, variant 3 (a work item
                              of gs_render_bwd, and a point where a forward with a state saves it):
                              0 = 1024, else a multiple of 32 in 256..1048576. Longer segments save
                              less state and start fewer items; shorter ones balance long lists
                              across the GPU better */
  int32_t sort_mode;       /* 0: how gs_bin_sort orders the duplicates (the result is the same):
                              1 = radix passes (entries by (item, depth), then duplicates by tile);
                              2 = buckets: one counting pass by tile, then each tile's list sorted
                              by (depth, index) in LDS (few launches; made for short lists; up to
                              12288 tiles, else GS_ERR_UNSUPPORTED); 0 = automatic (2 up to 12288
                              tiles and 2^22 (item, Gaussian) entries, else 1) */
} gs_config;

/* One camera view: world -> camera transform x_c = R x_w + t (OpenCV axes,
 * x right, y down, z forward), R row-major; and its items in the item table. */
typedef struct gs_view {
  float R[9];
  float t[3];
  int32_t item_first, item_count;
} gs_view;

/* One (view, level) item. Filled by the caller (gs_make_items() does it on the host). */
typedef struct gs_item {
  float fx, fy, cx, cy;    /* intrinsics of this level, pixels */
  int32_t W, H;            /* level image size */
  int32_t view, level;
  int32_t tiles_x, tiles_y;
  int32_t tile_base;       /* first global tile index of the item */
  int32_t pad;
  int64_t pixel_base;      /* first pixel of the item in the concatenated images */
} gs_item;

/* Gaussian parameters, structure of arrays, float32 (Sec. III-B, generalised to a
 * per-axis scale and a rotation; the paper's isotropic primitive is the case of
 * three equal scales). */
typedef struct gs_gaussians {
  int64_t n;
  const float* mean;       /* [n][3] world position mu */
  const float* log_scale;  /* [n][3] log of the per-axis standard deviation */
  const float* quat;       /* [n][4] rotation (w, x, y, z), normalised inside */
  const float* opacity;    /* [n]    logit; o = sigmoid */
  const float* rgb;        /* [n][3] colour feature r (eq. 7) */
  const float* sem;        /* [n][n_sem] semantic feature s (eq. 9), plain mode */
  const uint16_t* emb;     /* [n][16] bfloat16 embedding, learned mode (else NULL) */
} gs_gaussians;

/* Per (item, Gaussian) projection, written by gs_preprocess, [n_items * n] each,
 * entry e = item * n + gaussian. */
typedef struct gs_projected {
  float* rec;       /* [E][8]: mean2d hi x, y; mean2d lo x, y (mean2d = hi + lo);
                       conic A, B, C (inverse 2D covariance [[A,B],[B,C]]); opacity */
  float* depth;     /* [E] camera-space depth of the mean (sort key, depth feature) */
  int32_t* radius;  /* [E] footprint radius in pixels; 0 = culled */
} gs_projected;

/* Rendered or gradient images. */
typedef struct gs_images {
  float* color;          /* [P * (4 + n_sem)] planar per item */
  float* T;              /* [P] final transmittance (forward only) */
  uint32_t* n_contrib;   /* [P] 1 + list position of the last blended Gaussian, 0 if none */
  float* logits;         /* [P * n_classes] learned mode decoded logits, else NULL */
  int64_t n_pixels;      /* P, the total pixel count of all items (read in learned mode) */
  /* Forward output, optional (NULL: none; ignored by render variants 1 and 2): a caller
   * buffer of state_bytes >= gs_workspace_size(GS_WS_RENDER_STATE) bytes. With it, the
   * forward cuts tile lists into segments of cfg->seg_len entries, walked fwd_chunk at a
   * time (a transmittance pre-pass gives each work item its starting T), and keeps, per
   * segment and pixel, what the reverse pass needs to start a segment: gs_render_bwd
   * given these images then skips its summary pass. Overwritten by every forward; read
   * by the backward, which must get the same images. */
  void* state;
  size_t state_bytes;
} gs_images;

/* Targets of the loss (the image pyramid of eq. 4-6). */
typedef struct gs_targets {
  const float* rgb;      /* [P * 3] planar per item */
  const float* depth;    /* [P]; <= 0 marks a missing depth */
  const int32_t* label;  /* [P] class index in [0, n_classes); any other value = unlabelled */
  const float* sem_color; /* [P * 3] planar per item: a semantic colour image (eq. 12), or NULL for
                             the cross-entropy on labels */
} gs_targets;

/* Learned semantic head: logits = W2 relu(W1 E + b1) + b2 (bfloat16 weights). */
typedef struct gs_head {
  int32_t d_in;          /* 16 */
  int32_t d_hidden;      /* 64 */
  int32_t n_classes;
  int32_t pad;
  const uint16_t* W1;    /* [d_hidden][d_in] bfloat16 */
  const float* b1;       /* [d_hidden] */
  const uint16_t* W2;    /* [n_classes][d_hidden] bfloat16 */
  const float* b2;       /* [n_classes] */
} gs_head;

/* Gradient outputs. Every non-NULL array is overwritten (zeroed by the callee first). */
typedef struct gs_grads {
  float* mean;       /* [n][3] */
  float* log_scale;  /* [n][3] */
  float* quat;       /* [n][4] */
  float* opacity;    /* [n] (with respect to the logit) */
  float* rgb;        /* [n][3] */
  float* sem;        /* [n][n_sem] plain mode */
  float* emb;        /* [n][16] learned mode, float32 */
  float* pose;       /* [n_views][6]: (rho, phi) of T_cw <- Exp(xi) T_cw at xi = 0 */
  float* head_W1;    /* learned mode: [64][16] */
  float* head_b1;    /* [64] */
  float* head_W2;    /* [n_classes][64] */
  float* head_b2;    /* [n_classes] */
} gs_grads;

enum gs_workspace_kind { GS_WS_BIN_SORT = 1, GS_WS_RENDER_BWD = 2, GS_WS_LOSS = 3, GS_WS_RENDER_STATE = 4 };

/* ---- helpers --------------------------------------------------------------- */
void gs_config_default(gs_config* cfg);
const char* gs_status_string(int status);
int gs_last_hip_error(void);
int gs_version(void);

/* Host helper: fills views[i].item_first/item_count and items[] (host memory) for
 * n_views views of base size W[v] x H[v], intrinsics K[v] = (fx, fy, cx, cy) and
 * levels[v] pyramid levels. W and H must be divisible by 2^(levels-1).
 * items must hold sum(levels) entries. Returns the item count, or a negative status.
 * n_pixels and n_tiles (host, may be NULL) receive the totals. */
int gs_make_items(const gs_config* cfg, int32_t n_views, gs_view* views, const int32_t* W, const int32_t* H,
                  const float* K, const int32_t* levels, gs_item* items, int64_t* n_pixels, int32_t* n_tiles);

/* Bytes of caller workspace a call needs (kind = gs_workspace_kind). GS_WS_RENDER_STATE
 * (the optional gs_images.state of a forward) depends on n_tiles, dup_capacity (the
 * bin_sort capacity the lists come from), cfg->n_sem and cfg->seg_len; GS_WS_RENDER_BWD
 * on n_items * n_gauss, n_tiles, dup_capacity and cfg->seg_len. Both hold at most one
 * segment per tile more than dup_capacity / seg_len, so a buffer sized for one segment
 * length holds fewer segments of a shorter one. A smaller buffer still works when the
 * lists' segments fit it, and makes every tile one item when they do not. */
int gs_workspace_size(int kind, const gs_config* cfg, int32_t n_items, int64_t n_gauss, int32_t n_tiles,
                      int64_t dup_capacity, int64_t n_pixels, size_t* bytes);

/* ---- the hot path ------------------------------------------------------------ */

/* Projection (eq. 2-3 in the EWA form): for every view and Gaussian, the camera-space
 * mean, the 2D covariance J W Sigma W^T J^T + eps I with Sigma = R(q) S^2 R(q)^T,
 * its inverse (conic), the projected mean K (W mu + t) / z, the opacity sigmoid(a),
 * the radius ceil(3 sqrt(lambda_max)) and, per level, the same for K_l.
 * A Gaussian is culled (radius 0) when z <= z_near, |q| = 0, det <= 0, or its
 * tile rectangle is empty. */
int gs_preprocess(const gs_config* cfg, const gs_gaussians* g, const gs_view* views_dev, int32_t n_views,
                  const gs_item* items_dev, int32_t n_items, gs_projected* out, void* stream);

/* Binning and depth order (the sorted set N of eq. 7-9): every visible (item, Gaussian)
 * is duplicated once per tile of its rectangle; the duplicates are ordered by
 * (global tile, float32 depth, Gaussian index) -- equivalently by the 64-bit key
 * tile << 32 | bits(depth), ties by index -- and ranges[2t], ranges[2t+1] receive
 * the first and one-past-last position of tile t ((0, 0) if empty).
 * vals[j] = Gaussian index of entry j; keys (may be NULL) = the 64-bit keys.
 * Every entry with radius > 0 must have depth > 0 (gs_preprocess gives depth > z_near).
 * n_dup_dev (device int64) receives the duplicate count. If it exceeds dup_capacity,
 * status_dev (device int32) is set to GS_ERR_CAPACITY and nothing past the capacity
 * is written (the lists are then incomplete); otherwise status_dev is set
 * to GS_OK. cfg->sort_mode picks the method; the workspace size covers both. */
int gs_bin_sort(const gs_config* cfg, const gs_projected* proj, const gs_item* items_dev, int32_t n_items,
                int64_t n_gauss, int32_t n_tiles, int64_t dup_capacity, void* workspace, size_t ws_bytes,
                uint64_t* keys, uint32_t* vals, uint32_t* ranges, int64_t* n_dup_dev, int32_t* status_dev,
                void* stream);

/* Front-to-back compositing (eq. 7-9) of every pixel of every item: over its tile's
 * list, alpha = min(alpha_max, o exp(-d^T conic d / 2)), skipped below alpha_min;
 * the pixel stops before the Gaussian that would take T below t_min; the colour,
 * depth and semantic channels accumulate f alpha T. Learned mode (g->emb != NULL,
 * n_sem = 16): the semantic channels composite the bfloat16 embedding in single
 * precision; with head != NULL, out->logits [P * head->n_classes] also receives the
 * head's decode W2 relu(W1 E + b1) + b2 of every pixel's embedding E (matrix cores,
 * bfloat16 weights, single-precision accumulation). */
int gs_render_fwd(const gs_config* cfg, const gs_gaussians* g, const gs_projected* proj, const gs_item* items_dev,
                  int32_t n_items, int32_t n_tiles, const uint32_t* vals, const uint32_t* ranges,
                  const gs_head* head, gs_images* out, void* stream);

/* Per-level loss (eq. 10-13): for each item, loss_dev[3i..3i+2] = L_rgb, mean |D - D_gt|
 * over pixels with D_gt > 0, and L_sem, where L_rgb = (1 - l) mean |R - R_gt| over 3HW +
 * l (1 - SSIM), l = cfg->ssim_lambda, and SSIM is the mean over the 3 colour channels and all
 * pixels of the structural similarity of Wang et al. (2004) with an 11 x 11 Gaussian window
 * of standard deviation 1.5 (weights summing to 1; both images taken as zero outside),
 * C1 = 0.01^2, C2 = 0.03^2. grad_out->color receives the gradient of
 * sum_i (w[0] L_rgb + w[1] L_depth + w[2] L_sem) with respect to every rendered channel.
 * w is a host array of 3. L_sem is one of:
 *  - targets->sem_color != NULL (eq. 12, the semantic feature a colour): plain mode with
 *    cfg->n_sem = 3 and n_classes = 0; channels 4..6 of rendered->color are the semantic
 *    colour image S and L_sem = (1 - l_s) mean |S - S_gt| over 3HW + l_s (1 - SSIM(S, S_gt)),
 *    l_s = cfg->sem_ssim_lambda, SSIM as above;
 *  - otherwise the mean over pixels of -log softmax(S)[label] (a label outside
 *    [0, n_classes) adds no term), with the class logits S, in plain mode, channels 4.. of
 *    rendered->color; in learned mode (cfg->n_sem = 16) either
 *  - head != NULL: the decode S = W2 relu(W1 E + b1) + b2 of the embedding channels E,
 *    evaluated inside the loss (matrix cores, as gs_render_fwd's) and differentiated there:
 *    grad_out->color channels 4..19 receive dL/dE and head_grads->head_W1 .. head_b2 the
 *    weight gradients (overwritten); no logits are read or written (rendered->logits and
 *    grad_out->logits are ignored); or
 *  - head == NULL: S = rendered->logits (gs_render_fwd's decode), whose gradient goes to
 *    grad_out->logits; channels 4..19 of grad_out->color get 0.
 * workspace: gs_workspace_size(GS_WS_LOSS); its contents are scratch between calls. */
int gs_pyramid_loss(const gs_config* cfg, const gs_item* items_dev, int32_t n_items, int64_t n_pixels,
                    int32_t n_classes, const gs_images* rendered, const gs_targets* targets, const gs_head* head,
                    const float* w, float* loss_dev, gs_images* grad_out, gs_grads* head_grads, void* workspace,
                    size_t ws_bytes, void* stream);

/* gs_pyramid_loss for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same computation
 * and arguments without the workspace, which is instead a 16 MiB array the library holds
 * in each GPU's memory (from the library's load until the process ends). The caller still
 * passes every input and output. At most 2048 items; more returns GS_ERR_WORKSPACE before
 * anything is enqueued. Nothing is allocated or freed by the call. Every call on one GPU
 * shares that GPU's array, which keeps the last call's contents (each call clears what it
 * sums into first), so calls that overlap in time on one GPU, on any streams, race and must
 * be ordered by the caller. */
int gs_pyramid_loss_static(const gs_config* cfg, const gs_item* items_dev, int32_t n_items, int64_t n_pixels,
                           int32_t n_classes, const gs_images* rendered, const gs_targets* targets, const gs_head* head,
                           const float* w, float* loss_dev, gs_images* grad_out, gs_grads* head_grads, void* stream);

/* Back-propagation (Sec. III-D) of an upstream gradient grad_in->color (and ->logits)
 * through compositing and projection to every Gaussian parameter and every view's
 * pose tangent. fwd must hold T and n_contrib of the matching gs_render_fwd.
 * Learned mode (g->emb != NULL): grads->emb receives the per-Gaussian embedding gradient
 * of the embedding channels' gradient, channels 4..19 of grad_in->color. With head != NULL
 * and grad_in->logits (a decode's logit gradient), the head is differentiated first: its
 * gradient with respect to the embedding image is added to channels 4..19 of
 * grad_in->color (the caller's buffer) and grads->head_* receive the weight gradients.
 * With head == NULL (grad_in->logits must be NULL) channels 4..19 are taken as they are,
 * e.g. from gs_pyramid_loss with its head. workspace: gs_workspace_size(GS_WS_RENDER_BWD). */
int gs_render_bwd(const gs_config* cfg, const gs_gaussians* g, const gs_projected* proj, const gs_view* views_dev,
                  int32_t n_views, const gs_item* items_dev, int32_t n_items, int32_t n_tiles,
                  const uint32_t* vals, const uint32_t* ranges, const gs_head* head, const gs_images* fwd,
                  const gs_images* grad_in, gs_grads* grads, void* workspace, size_t ws_bytes, void* stream);

/* Image pyramid (eq. 4-6): fills levels 1..max_level of every view from the level
 * above by 2x2 box means of a K-channel image; channel 3 (depth) averages only its
 * positive children (0 if none). labels (may be NULL) receives, for every pixel of
 * every item, the argmax over channels 4..K-1 (ties to the lowest index). */
int gs_pyramid_downsample(const gs_item* items_dev, int32_t n_items, int64_t n_pixels, int32_t max_level,
                          int32_t K, float* img, int32_t* labels, void* stream);

/* ---- view-dependent features (Sec. III-B, spherical harmonics) -------------- */

/* Higher SH bands of the colour and semantic features. The constant band is the plain
 * feature (gs_gaussians.rgb / .sem), so degree 0 needs no array here. Coefficients are
 * [n][(degree+1)^2 - 1][channels], band index j = l^2 + l + m (l >= 1), real harmonics in
 * the sign convention of the 3DGS renderer. */
typedef struct gs_sh {
  int32_t rgb_degree, sem_degree;   /* 0..3 */
  const float* rgb_rest;            /* [n][(rgb_degree+1)^2 - 1][3], NULL for degree 0 */
  const float* sem_rest;            /* [n][(sem_degree+1)^2 - 1][n_sem], NULL for degree 0 */
} gs_sh;

/* Per view v and Gaussian i: f_vic = dc_ic + sum_j Y_j(d_vi) k_ijc with d_vi the unit
 * direction from the camera centre -R_v^T t_v to the mean. Writes rgb_out [n_views][n][3]
 * and sem_out [n_views][n][n_sem] (device), the per-view feature blocks that gs_render_fwd
 * and gs_render_bwd read with cfg->view_features = 1. g supplies mean, rgb and sem (the
 * constant band); n_sem may be 0 (sem_out unused). One launch on `stream`. */
int gs_sh_features(int32_t n_sem, const gs_gaussians* g, const gs_sh* sh, const gs_view* views_dev, int32_t n_views,
                   float* rgb_out, float* sem_out, void* stream);

/* Backward of gs_sh_features for the per-view feature gradients grad_rgb [n_views][n][3]
 * and grad_sem [n_views][n][n_sem] (gs_render_bwd's grads->rgb / ->sem under
 * view_features): WRITES the constant-band gradients grad_rgb_dc [n][3], grad_sem_dc
 * [n][n_sem] and the band gradients grad_rgb_rest / grad_sem_rest (the layouts of gs_sh;
 * any may be NULL to skip it), and ADDS the direction's share to grad_mean [n][3] and to the
 * translation part of grad_pose [n_views][6] (the camera centre moves by -R^T rho under
 * T_cw <- Exp(xi) T_cw, and not with phi), so that it runs after gs_render_bwd. */
int gs_sh_features_bwd(int32_t n_sem, const gs_gaussians* g, const gs_sh* sh, const gs_view* views_dev,
                       int32_t n_views, const float* grad_rgb, const float* grad_sem, float* grad_rgb_dc,
                       float* grad_rgb_rest, float* grad_sem_dc, float* grad_sem_rest, float* grad_mean,
                       float* grad_pose, void* stream);

/* ---- mapping update (Sec. III-D) -------------------------------------------- */

/* Writable float32 arrays in the layouts of the gs_gaussians fields of the same name. */
typedef struct gs_param_arrays {
  float* mean;       /* [n][3] */
  float* log_scale;  /* [n][3] */
  float* quat;       /* [n][4] */
  float* opacity;    /* [n] logit */
  float* rgb;        /* [n][3] */
  float* sem;        /* [n][n_sem] (plain mode; NULL when n_sem = 0) */
} gs_param_arrays;

/* Adam hyper-parameters of a mapping step: one learning rate per parameter group and
 * for the translation (rho) and rotation (phi) parts of the pose tangent. A group whose
 * rate is 0 is left untouched (parameters and moments). */
typedef struct gs_adam_config {
  float lr_mean, lr_log_scale, lr_quat, lr_opacity, lr_rgb, lr_sem;
  float lr_rho, lr_phi;
  float beta1, beta2, eps;   /* 0 <= beta < 1, eps > 0 */
} gs_adam_config;

/* One Adam step (Kingma and Ba 2015, Algorithm 1, bias-corrected; step >= 1) on every
 * parameter group of n Gaussians at once: p <- p - lr m_hat / (sqrt(v_hat) + eps) with the
 * gradients of gs_render_bwd (grads->mean .. grads->sem; the other fields are not read).
 * m and v (device, same layouts, zero before the first step) hold the moments. In place on
 * `params`; one launch on `stream`. */
int gs_gaussians_adam(int64_t n, int32_t n_sem, const gs_param_arrays* params, const gs_grads* grads,
                      const gs_param_arrays* m, const gs_param_arrays* v, const gs_adam_config* hp, int32_t step,
                      void* stream);

/* Pose update of n_views views (device gs_view array, R and t rewritten in place): Adam on
 * each view's tangent gradient grad_pose [n_views][6] = (rho, phi) (as gs_grads.pose), with
 * moments m, v [n_views][6] (device, zero before the first step), gives the step delta;
 * then T_cw <- Exp(delta) T_cw, the left-multiplied SE(3) exponential, composed in double
 * precision and its rotation re-orthonormalised before it is stored. item_first and
 * item_count are not touched. */
int gs_pose_adam(gs_view* views_dev, int32_t n_views, const float* grad_pose, float* m, float* v,
                 const gs_adam_config* hp, int32_t step, void* stream);

/* Left perturbation of view poses at a nonzero tangent (the pose input of an autograd
 * wrapper; R12 of the readings: T_cw <- Exp(xi) T_cw, xi = (rho, phi), rho first):
 * views_out[i] = views_in[i] with R, t replaced by those of Exp(xi_i) T_cw, composed in
 * double precision and rounded once to single precision (not re-orthonormalised);
 * item_first and item_count are copied. xi [n_views][6] (device). views_out may equal
 * views_in. One launch on `stream`. */
int gs_pose_perturb(const gs_view* views_in, int32_t n_views, const float* xi, gs_view* views_out, void* stream);

/* Chain rule of gs_pose_perturb: grad_xi[i] = J_l(xi_i)^T grad_pose[i], where grad_pose is the
 * gradient with respect to a tangent at the perturbed pose (gs_render_bwd's grads->pose after
 * rendering with views_out) and J_l the left Jacobian of SE(3), Exp(xi + d) = Exp(J_l d) Exp(xi)
 * to first order in d. Arrays [n_views][6] (device); grad_xi must not alias grad_pose. */
int gs_pose_perturb_bwd(const float* xi, int32_t n_views, const float* grad_pose, float* grad_xi, void* stream);

/* ---- training helpers for the learned head ------------------------------- */

/* One Adam step on n float32 parameters in place (m, v: moment buffers, step >= 1,
 * bias-corrected). bf16_copy (may be NULL) receives the updated values rounded to
 * bfloat16 (nearest, ties to even). */
int gs_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                 float eps, int32_t step, uint16_t* bf16_copy, void* stream);

/* Distillation of decoded logits `student` onto the plain render's logits `teacher`
 * (both [P * C] planar per item): per item, the mean over pixels of the soft-target
 * cross-entropy -sum_c softmax(teacher)_c log softmax(student)_c plus mse_w times the
 * mean over pixels and classes of (student - teacher)^2; *loss_dev = sum over items.
 * grad receives d loss / d student. workspace: 256 bytes. */
int gs_distill_loss(const gs_item* items_dev, int32_t n_items, int64_t n_pixels, int32_t C, const float* teacher,
                    const float* student, float mse_w, float* loss_dev, float* grad, void* workspace, size_t ws_bytes,
                    void* stream);

/* counts_dev[i] (uint64) = number of pixels of item i whose argmax over the C planar
 * channels of a and b agree (ties to the lowest channel). */
int gs_argmax_agreement(const gs_item* items_dev, int32_t n_items, int64_t n_pixels, int32_t C, const float* a,
                        const float* b, uint64_t* counts_dev, void* stream);

/* ---- graph capture of a whole step (Sec. III-C/D: one mapping iteration) ----
 * Every hot-path call above only enqueues kernels and never synchronises, so a full
 * step (preprocess, bin_sort, render_fwd, pyramid_loss, render_bwd) can be captured
 * once and replayed. gs_graph_begin starts a capture of `stream` (relaxed mode);
 * gs_graph_end ends it and instantiates the graph into *graph_exec (host memory owned
 * by the library until gs_graph_destroy). Buffers referenced by the captured calls
 * must stay allocated and keep their addresses while the graph is replayed. */
int gs_graph_begin(void* stream);
int gs_graph_end(void* stream, void** graph_exec);
int gs_graph_launch(void* graph_exec, void* stream);
int gs_graph_destroy(void* graph_exec);

#ifdef __cplusplus
}
#endif
#endif /* GS_H */
