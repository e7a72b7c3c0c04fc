// Per-level reconstruction loss (paper eq. 10-13: L1 terms, the SSIM term of the colour
// loss, semantics as a per-pixel cross-entropy on the composited class logits or, when the
// semantic feature is a colour, eq. 12's L1 and SSIM on the semantic colour image) and the
// image pyramid of the targets (eq. 4-6, 2x2 box means). The L1 / cross-entropy pass and
// the pyramid are elementwise over pixels and bound by HBM traffic: one thread per pixel,
// planar channel reads coalesced along x. SSIM is a windowed filter: LDS-tiled, one
// 32 x 32 output tile of one colour channel per workgroup, forward and gradient fused.
#include "common.h"

namespace gs {
namespace {

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Partial sums are spread over kSlots addresses per item (slot = block index mod kSlots)
// so that thousands of blocks do not serialise on one atomic address; a one-block
// kernel folds the slots afterwards.
constexpr int kSlots = 64;

// out[i * stride + c] = sum over slots of in[(i * ncomp + c) * kSlots + slot].
__global__ void k_fold_slots(const float* __restrict__ in, int n_items, int ncomp, float* __restrict__ out) {
  for (int i = threadIdx.x; i < n_items * ncomp; i += blockDim.x) {
    const float* src = in + (int64_t)i * kSlots;
    float s = 0.0f;
    for (int k = 0; k < kSlots; ++k) s += src[k];
    out[i] = s;
  }
}

__device__ __forceinline__ float sgn(float d) { return (float)((d > 0.0f) - (d < 0.0f)); }

// Item of each lane's pixel. Items are ordered by pixel_base: the lanes read 64 bases at a
// time and the wave's first pixel lies in item (number of bases <= it) - 1, one memory round
// trip for up to 64 items; only a wave that straddles two items searches per lane.
struct PixItem {
  int item, W, H;
  int64_t pixel_base;
};

__device__ __forceinline__ PixItem lane_item(const gs_item* __restrict__ items, int n_items, int64_t wave_pix0,
                                             int64_t pix) {
  const int lane = (int)(threadIdx.x & 63);
  int count = 0;
  for (int b = 0; b < n_items; b += 64) {
    const int i = b + lane;
    const uint64_t m = __ballot(i < n_items && items[i].pixel_base <= wave_pix0);
    count += (int)__popcll(m);
    if (m != ~0ull) break;
  }
  const int first = __builtin_amdgcn_readfirstlane(count - 1);
  PixItem r{first, items[first].W, items[first].H, items[first].pixel_base};
  if (pix >= r.pixel_base + (int64_t)r.W * r.H) {
    r.item = item_of_pixel(items, n_items, pix);
    r.W = items[r.item].W;
    r.H = items[r.item].H;
    r.pixel_base = items[r.item].pixel_base;
  }
  return r;
}

// Per-item L1 colour, L1 depth over valid target depths, cross-entropy on the class
// logits, and their image gradients, in one pass over each pixel's channels (every load
// issued before the arithmetic). The depth gradient is written as sign(d) (or 0) and
// scaled by w1 / n_valid afterwards, once the valid counts are known; the logits of a
// pixel are held in registers (CM >= classes). With a semantic colour target (tsem, eq. 12;
// then CM = 0 and K = 7) the semantic term is instead the L1 mean of channels 4..6 against
// it, with its gradient written here unless the SSIM pass writes it (sem_grad false).
// Every input and output element is touched once: loads and stores are non-temporal.
template <int CM>
__global__ __launch_bounds__(256) void k_loss(const gs_item* __restrict__ items, int n_items, int64_t P, int K,
                                              int n_classes, const float* __restrict__ color,
                                              const float* __restrict__ logits, const float* __restrict__ trgb,
                                              const float* __restrict__ tdepth, const int32_t* __restrict__ tlabel,
                                              const float* __restrict__ tsem, float w0, float w2, bool rgb_grad,
                                              bool sem_grad, float* __restrict__ loss_slots,
                                              float* __restrict__ count_slots, float* __restrict__ gcolor,
                                              float* __restrict__ glogits) {
  const int slot = blockIdx.x % kSlots;
  const int64_t wave_pix0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  if (wave_pix0 >= P) return;
  const int64_t pix = wave_pix0 + (threadIdx.x & 63);
  const bool live = pix < P;
  const PixItem it = lane_item(items, n_items, wave_pix0, live ? pix : wave_pix0);
  const int item = it.item;
  float lr = 0.0f, ld = 0.0f, ls = 0.0f, nv = 0.0f;
  if (live) {
    const int64_t HW = (int64_t)it.W * it.H;
    const int64_t p = pix - it.pixel_base;
    const int64_t cb = it.pixel_base * K + p;
    const int64_t tb = it.pixel_base * 3 + p;
    const bool sem = CM > 0 && n_classes > 0;
    // plain mode: logits are colour channels 4..; learned mode: a separate C-plane image
    const int64_t lb = logits ? it.pixel_base * n_classes + p : cb + 4 * HW;
    const float* L = logits ? logits : color;
    float col[4], tr[3];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) col[ch] = __builtin_nontemporal_load(&color[cb + ch * HW]);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) tr[ch] = __builtin_nontemporal_load(&trgb[tb + ch * HW]);
    const float td = __builtin_nontemporal_load(&tdepth[pix]);
    const int y = sem ? __builtin_nontemporal_load(&tlabel[pix]) : -1;
    float x[CM > 0 ? CM : 1];
#pragma unroll
    for (int c = 0; c < CM; ++c) x[c] = c < n_classes ? __builtin_nontemporal_load(&L[lb + c * HW]) : -INFINITY;

    const float inv3 = 1.0f / (3.0f * (float)HW);
    float gc[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float d = col[ch] - tr[ch];
      lr += fabsf(d) * inv3;
      gc[ch] = w0 * sgn(d) * inv3;
    }
    float gd = 0.0f;
    if (td > 0.0f) {
      const float d = col[3] - td;
      ld = fabsf(d);
      nv = 1.0f;
      gd = sgn(d);
    }
    if (rgb_grad) {   // else the SSIM pass writes the colour gradient
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) __builtin_nontemporal_store(gc[ch], &gcolor[cb + ch * HW]);
    }
    __builtin_nontemporal_store(gd, &gcolor[cb + 3 * HW]);
    // learned mode: the loss has no direct term on the composited embedding channels
    // (the head's backward adds its input gradient there)
    if (logits)
      for (int ch = 4; ch < K; ++ch) __builtin_nontemporal_store(0.0f, &gcolor[cb + ch * HW]);
    if (CM == 0 && tsem) {
      // eq. 12's L1 part on the semantic colour channels 4..6
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float d = __builtin_nontemporal_load(&color[cb + (4 + ch) * HW]) -
                        __builtin_nontemporal_load(&tsem[tb + ch * HW]);
        ls += fabsf(d) * inv3;
        if (sem_grad) __builtin_nontemporal_store(w2 * sgn(d) * inv3, &gcolor[cb + (4 + ch) * HW]);
      }
    }
    if (sem) {
      float* G = logits ? glogits + lb : gcolor + lb;
      float m = -INFINITY;
#pragma unroll
      for (int c = 0; c < CM; ++c) m = fmaxf(m, x[c]);
      float xy = 0.0f, z = 0.0f;
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        xy = c == y ? x[c] : xy;
        x[c] = c < n_classes ? __expf(x[c] - m) : 0.0f;
        z += x[c];
      }
      const float invp = 1.0f / (float)HW;
      const bool labelled = y >= 0 && y < n_classes;   // outside [0, C): unlabelled, no semantic term
      if (labelled) ls = (m + __logf(z) - xy) * invp;
      const float sc = labelled ? w2 * invp / z : 0.0f;
      const float oh = labelled ? w2 * invp : 0.0f;
#pragma unroll
      for (int c = 0; c < CM; ++c)
        if (c < n_classes) __builtin_nontemporal_store(x[c] * sc - (c == y ? oh : 0.0f), &G[c * HW]);
    }
  }
  // wave-uniform item: one atomic per wave and quantity, else one per lane
  const int first = __shfl(item, 0, 64);
  const bool uniform = __ballot(item != first) == 0ull;
  float* loss = loss_slots + slot;
  float* count = count_slots + slot;
  if (uniform) {
    const float a = wave_sum(lr), b = wave_sum(ld), c = wave_sum(ls), v = wave_sum(nv);
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&loss[(3 * first + 0) * kSlots], a);
      if (v != 0.0f) {
        atomicAdd(&loss[(3 * first + 1) * kSlots], b);
        atomicAdd(&count[first * kSlots], v);
      }
      atomicAdd(&loss[(3 * first + 2) * kSlots], c);
    }
  } else if (live) {
    atomicAdd(&loss[(3 * item + 0) * kSlots], lr);
    if (nv != 0.0f) {
      atomicAdd(&loss[(3 * item + 1) * kSlots], ld);
      atomicAdd(&count[item * kSlots], nv);
    }
    atomicAdd(&loss[(3 * item + 2) * kSlots], ls);
  }
}

// Folds the slots: loss[i] = (colour term, L1 depth / n_valid, semantic term); n_valid[i].
// The colour term is (1 - lambda) L1 + lambda (1 - mean SSIM) (lambda = 0: the L1 mean); the
// semantic term is the cross-entropy, or the same form as the colour term with lambda_s on
// the semantic colour image (its SSIM sums in the second block of n_items slot rows).
__global__ void k_fold_loss(const float* __restrict__ loss_slots, const float* __restrict__ count_slots,
                            const float* __restrict__ ssim_slots, float lambda, float lambda_s, int n_items,
                            float* __restrict__ loss, float* __restrict__ nvalid) {
  for (int i = threadIdx.x; i < n_items * 4; i += blockDim.x) {
    const int item = i >> 2, comp = i & 3;
    const float* src = comp < 3 ? loss_slots + (int64_t)(3 * item + comp) * kSlots : count_slots + (int64_t)item * kSlots;
    float s = 0.0f;
    for (int k = 0; k < kSlots; ++k) s += src[k];
    if (comp == 3) {
      nvalid[item] = s;
    } else if (comp == 0 && lambda != 0.0f) {
      const float* ss = ssim_slots + (int64_t)item * kSlots;
      float m = 0.0f;
      for (int k = 0; k < kSlots; ++k) m += ss[k];
      loss[3 * item] = (1.0f - lambda) * s + lambda * (1.0f - m);
    } else if (comp == 2 && lambda_s != 0.0f) {
      const float* ss = ssim_slots + (int64_t)(n_items + item) * kSlots;
      float m = 0.0f;
      for (int k = 0; k < kSlots; ++k) m += ss[k];
      loss[3 * item + 2] = (1.0f - lambda_s) * s + lambda_s * (1.0f - m);
    } else if (comp != 1) {
      loss[3 * item + comp] = s;
    }
  }
  __syncthreads();
  for (int item = threadIdx.x; item < n_items; item += blockDim.x) {
    const float* src = loss_slots + (int64_t)(3 * item + 1) * kSlots;
    float s = 0.0f;
    for (int k = 0; k < kSlots; ++k) s += src[k];
    loss[3 * item + 1] = nvalid[item] > 0.0f ? s / nvalid[item] : 0.0f;
  }
}

// Depth-gradient plane *= w1 / n_valid of the pixel's item.
__global__ __launch_bounds__(256) void k_scale_depth(const gs_item* __restrict__ items, int n_items, int64_t P, int K,
                                                     float w1, const float* __restrict__ nvalid,
                                                     float* __restrict__ gcolor) {
  const int64_t wave_pix0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  if (wave_pix0 >= P) return;
  const int64_t pix = wave_pix0 + (threadIdx.x & 63);
  if (pix >= P) return;
  const PixItem it = lane_item(items, n_items, wave_pix0, pix);
  const int64_t HW = (int64_t)it.W * it.H;
  float* g = gcolor + it.pixel_base * K + 3 * HW + (pix - it.pixel_base);
  const float nv = nvalid[it.item];
  *g = nv > 0.0f ? *g * (w1 / nv) : 0.0f;
}

// ---- SSIM (Wang et al. 2004) of the colour loss ----------------------------------------
// Per channel, window sums with the 11 x 11 Gaussian of standard deviation 1.5 (weights
// normalised to 1, image taken as zero outside): mu_x, mu_y, E[x^2], E[y^2], E[xy] at every
// pixel q, S(q) = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)),
// C1 = 0.01^2, C2 = 0.03^2. With A, B, C the partial derivatives of S(q) with respect to
// the window sums of x, x^2 and xy, d mean(S) / d x(p) = (g*A + 2 x(p) g*B + y(p) g*C)(p) / HW,
// g* the same window (symmetric). A tile of 32 x 32 gradients therefore needs A, B, C on
// 42 x 42 positions and those the inputs on 52 x 52; the Gaussian is separable, so each
// filter is a horizontal then a vertical 11-tap pass.
constexpr int kSsT = 32;                      // output tile edge
constexpr int kSsR = 5;                       // window radius
constexpr int kSsN2 = kSsT + 2 * kSsR;        // 42: positions whose A, B, C a tile reads
constexpr int kSsN1 = kSsT + 4 * kSsR;        // 52: input extent
// Work units: a run of outputs along a row (horizontal passes) or a column (vertical).
constexpr int kSsH = 7;                       // outputs per unit, first horizontal pass (42 = 6 x 7)
constexpr int kSsV = 7;                       // outputs per unit, first vertical pass
constexpr int kSsH2 = 8;                      // outputs per unit, second horizontal pass (32 = 4 x 8)
constexpr int kSsV2 = 4;                      // outputs per unit, second vertical pass (32 = 8 x 4)
constexpr int kSsHA = kSsT + 1;               // row stride of the second horizontal pass's output
static_assert(kSsN2 % kSsH == 0 && kSsN2 % kSsV == 0 && kSsT % kSsH2 == 0 && kSsT % kSsV2 == 0, "ssim units");
static_assert(kSsN2 * (kSsN2 / kSsV) <= 256 && kSsT * (kSsT / kSsV2) == 256, "one unit per thread");

constexpr double cexp(double x) {   // exp for |x| <= 12.5 by range halving and a Taylor series
  int h = 0;
  while (x < -0.5 || x > 0.5) { x *= 0.5; ++h; }
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 30; ++k) { t *= x / k; s += t; }
  while (h-- > 0) s *= s;
  return s;
}
constexpr double ss_raw(int i) { return cexp(-double((i - kSsR) * (i - kSsR)) / (2.0 * 1.5 * 1.5)); }
constexpr double ss_norm() {
  double t = 0;
  for (int i = 0; i <= 2 * kSsR; ++i) t += ss_raw(i);
  return t;
}
struct SsTaps { float g[2 * kSsR + 1]; };
constexpr SsTaps ss_taps() {
  SsTaps t{};
  for (int i = 0; i <= 2 * kSsR; ++i) t.g[i] = (float)(ss_raw(i) / ss_norm());
  return t;
}
constexpr SsTaps kSsG = ss_taps();

// Per item, the first SSIM tile: prefix[i] = sum over items < i of ceil(W/32) ceil(H/32).
__global__ void k_ssim_prefix(const gs_item* __restrict__ items, int n_items, int64_t* __restrict__ prefix) {
  __shared__ int64_t s[256];
  int64_t carry = 0;
  for (int base = 0; base < n_items; base += 256) {
    const int i = base + (int)threadIdx.x;
    int64_t v = 0;
    if (i < n_items) {
      const gs_item it = items[i];
      v = (int64_t)((it.W + kSsT - 1) / kSsT) * ((it.H + kSsT - 1) / kSsT);
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const int64_t a = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < n_items) prefix[i + 1] = carry + s[threadIdx.x];
    if (i == 0) prefix[0] = 0;
    carry += s[255];
    __syncthreads();
  }
}

// Where one (tile, channel) unit of the SSIM pass sits. Channels 0..2 are the colour image
// (planes 0..2, targets trgb), 3..5 the semantic colour image of eq. 12 (planes 4..6,
// targets tsem); a launch covers the nch channels from c0.
struct SsUnit {
  int64_t tile, pixel_base;
  int item, ch, W, H, tx0, ty0;
};

__device__ __forceinline__ SsUnit ss_locate(const gs_item* __restrict__ items, int n_items,
                                            const int64_t* __restrict__ prefix, int64_t w, int nch, int c0) {
  SsUnit u;
  u.tile = w / nch;
  u.ch = c0 + (int)(w - nch * u.tile);
  int lo = 0, hi = n_items - 1;                   // last item with prefix <= tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= u.tile) lo = mid; else hi = mid - 1;
  }
  const gs_item it = items[lo];
  u.item = lo;
  u.W = it.W;
  u.H = it.H;
  u.pixel_base = it.pixel_base;
  const int ntx = (it.W + kSsT - 1) / kSsT;
  const int local = (int)(u.tile - prefix[lo]);
  u.tx0 = (local % ntx) * kSsT;
  u.ty0 = (local / ntx) * kSsT;
  return u;
}

constexpr int kSsLoads = (kSsN1 * kSsN1 + 255) / 256;   // input values per thread

// Inputs of a unit over [ty0 - 10, ty0 + 42) x [tx0 - 10, tx0 + 42), zero outside the image,
// all loads issued before any is used.
__device__ __forceinline__ void ss_fetch(const SsUnit& u, int K, const float* __restrict__ color,
                                         const float* __restrict__ trgb, const float* __restrict__ tsem,
                                         float (&px)[kSsLoads], float (&py)[kSsLoads]) {
  const int64_t HW = (int64_t)u.W * u.H;
  const bool semc = u.ch >= 3;
  const float* X = color + u.pixel_base * K + (semc ? u.ch + 1 : u.ch) * HW;
  const float* Y = (semc ? tsem : trgb) + u.pixel_base * 3 + (semc ? u.ch - 3 : u.ch) * HW;
#pragma unroll
  for (int k = 0; k < kSsLoads; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    const int r = e / kSsN1, c = e - r * kSsN1;
    const int gy = u.ty0 - 2 * kSsR + r, gx = u.tx0 - 2 * kSsR + c;
    const bool in = e < kSsN1 * kSsN1 && gx >= 0 && gx < u.W && gy >= 0 && gy < u.H;
    const int64_t q = in ? (int64_t)gy * u.W + gx : 0;
    px[k] = in ? X[q] : 0.0f;
    py[k] = in ? Y[q] : 0.0f;
  }
}

// Horizontal 11-tap pass of NQ quantities formed from x and y: rows 0..51 of the input
// block, output columns 0..41 (column c centred on input column c + 5), into sH planes.
// Q(x, y) gives the NQ quantities of one input pixel.
template <int NQ, class Q>
__device__ __forceinline__ void ss_hpass(const float* __restrict__ sX, const float* __restrict__ sY,
                                         float* __restrict__ sH, Q quant) {
  for (int u = threadIdx.x; u < kSsN1 * (kSsN2 / kSsH); u += 256) {
    const int r = u / (kSsN2 / kSsH), c0 = (u - r * (kSsN2 / kSsH)) * kSsH;
    float v[NQ][kSsH + 2 * kSsR];
#pragma unroll
    for (int t = 0; t < kSsH + 2 * kSsR; ++t) {
      float q[NQ];
      quant(sX[r * kSsN1 + c0 + t], sY[r * kSsN1 + c0 + t], q);
#pragma unroll
      for (int k = 0; k < NQ; ++k) v[k][t] = q[k];
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k)
#pragma unroll
      for (int j = 0; j < kSsH; ++j) {
        float a = 0.0f;
#pragma unroll
        for (int t = 0; t <= 2 * kSsR; ++t) a = fmaf(kSsG.g[t], v[k][j + t], a);
        sH[(k * kSsN1 + r) * kSsN2 + c0 + j] = a;
      }
  }
}

// Vertical 11-tap pass of NQ sH planes at the unit's 7 positions (rows r0..r0+6, column j).
template <int NQ>
__device__ __forceinline__ void ss_vpass(const float* __restrict__ sH, int r0, int j, float (&m)[NQ][kSsV]) {
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    float v[kSsV + 2 * kSsR];
#pragma unroll
    for (int t = 0; t < kSsV + 2 * kSsR; ++t) v[t] = sH[(k * kSsN1 + r0 + t) * kSsN2 + j];
#pragma unroll
    for (int i = 0; i < kSsV; ++i) {
      float a = 0.0f;
#pragma unroll
      for (int t = 0; t <= 2 * kSsR; ++t) a = fmaf(kSsG.g[t], v[i + t], a);
      m[k][i] = a;
    }
  }
}

// Persistent loop over the nch x tile-count (tile, channel) units; the next unit's inputs
// are loaded into registers while the current one is filtered. Writes the gradient
// w ((1 - lambda) sign(x - y) / (3HW) - lambda / 3 d mean(S) / dx) of the tile's pixels (w0 and
// lambda for the colour channels, w2 and lambda_s for the semantic colour ones) and adds
// S / (3HW) over them to the item's SSIM slots (semantic colour: rows n_items + item).
__global__ __launch_bounds__(256) void k_ssim(const gs_item* __restrict__ items, int n_items,
                                              const int64_t* __restrict__ prefix, int K, int nch, int c0,
                                              const float* __restrict__ color, const float* __restrict__ trgb,
                                              const float* __restrict__ tsem, float w0, float lambda, float w2,
                                              float lambda_s, float* __restrict__ ssim_slots,
                                              float* __restrict__ gcolor) {
  __shared__ float sXY[2 * kSsN1 * kSsN1];       // inputs; later the second horizontal pass
  __shared__ float sH[5 * kSsN1 * kSsN2];        // first horizontal pass; later A, B, C
  float* const sX = sXY;
  float* const sY = sXY + kSsN1 * kSsN1;
  float* const sABC = sH;                         // [3][42][42]
  float* const sHA = sXY;                         // [3][42][33]
  static_assert(3 * kSsN2 * kSsN2 <= 5 * kSsN1 * kSsN2 && 3 * kSsN2 * kSsHA <= 2 * kSsN1 * kSsN1,
                "ssim LDS aliasing");
  const int tid = threadIdx.x;
  const int64_t total = nch * prefix[n_items];
  const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
  int64_t w = blockIdx.x;
  if (w >= total) return;
  float px[kSsLoads], py[kSsLoads];
  SsUnit cur = ss_locate(items, n_items, prefix, w, nch, c0);
  ss_fetch(cur, K, color, trgb, tsem, px, py);
  const bool vunit = tid < kSsN2 * (kSsN2 / kSsV);
  const int vj = tid % kSsN2, vr0 = (tid / kSsN2) * kSsV;   // first vertical pass
  const int oj = tid % kSsT, or0 = (tid / kSsT) * kSsV2;    // second vertical pass and output
  for (; w < total; w += gridDim.x) {
#pragma unroll
    for (int k = 0; k < kSsLoads; ++k) {
      const int e = tid + 256 * k;
      if (e < kSsN1 * kSsN1) {
        sX[e] = px[k];
        sY[e] = py[k];
      }
    }
    __syncthreads();
    const int64_t wn = w + gridDim.x;
    SsUnit nxt = cur;
    if (wn < total) {
      nxt = ss_locate(items, n_items, prefix, wn, nch, c0);
      ss_fetch(nxt, K, color, trgb, tsem, px, py);
    }
    const int W = cur.W, H = cur.H;
    const int64_t HW = (int64_t)W * H;
    const int tx0 = cur.tx0, ty0 = cur.ty0;

    // window sums of x, y, xy, x^2, y^2 at the 42 x 42 positions (r, j), image pixel
    // (ty0 - 5 + r, tx0 - 5 + j)
    ss_hpass<5>(sX, sY, sH, [](float x, float y, float (&q)[5]) {
      q[0] = x; q[1] = y; q[2] = x * y; q[3] = x * x; q[4] = y * y;
    });
    __syncthreads();
    float abc[3][kSsV];
    float ssum = 0.0f;
    if (vunit) {
      float m1[3][kSsV], m2[2][kSsV];
      {
        float m[5][kSsV];
        ss_vpass<5>(sH, vr0, vj, m);
#pragma unroll
        for (int i = 0; i < kSsV; ++i) {
          m1[0][i] = m[0][i]; m1[1][i] = m[1][i]; m1[2][i] = m[2][i];
          m2[0][i] = m[3][i]; m2[1][i] = m[4][i];
        }
      }
      const int gx = tx0 - kSsR + vj;
      const bool colin = gx >= 0 && gx < W;
      const bool colc = vj >= kSsR && vj < kSsR + kSsT;
#pragma unroll
      for (int i = 0; i < kSsV; ++i) {
        const int r = vr0 + i, gy = ty0 - kSsR + r;
        const float mx = m1[0][i], my = m1[1][i];
        const float sxx = m2[0][i] - mx * mx, syy = m2[1][i] - my * my, sxy = m1[2][i] - mx * my;
        const float a = fmaf(2.0f * mx, my, C1), b = fmaf(2.0f, sxy, C2);
        const float c = fmaf(mx, mx, fmaf(my, my, C1)), d = sxx + syy + C2;
        // c >= C1 and d >= C2 (up to rounding) are the only divisors: S / a and S / b are
        // formed as b / (cd) and a / (cd), finite where a or b vanish
        const float ic = __builtin_amdgcn_rcpf(c), id = __builtin_amdgcn_rcpf(d);
        const float Sa = b * ic * id, Sb = a * ic * id, S = a * Sa;
        const bool in = colin && gy >= 0 && gy < H;
        abc[0][i] = in ? 2.0f * (my * (Sa - Sb) + mx * S * (id - ic)) : 0.0f;
        abc[1][i] = in ? -S * id : 0.0f;
        abc[2][i] = in ? 2.0f * Sb : 0.0f;
        if (in && colc && r >= kSsR && r < kSsR + kSsT) ssum += S;
      }
    }
    // x and y of this thread's output pixels, before the inputs' LDS is reused
    float ox[kSsV2], oy[kSsV2];
#pragma unroll
    for (int i = 0; i < kSsV2; ++i) {
      const int li = (or0 + i + 2 * kSsR) * kSsN1 + oj + 2 * kSsR;
      ox[i] = sX[li];
      oy[i] = sY[li];
    }
    __syncthreads();
    if (vunit) {
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int i = 0; i < kSsV; ++i) sABC[(q * kSsN2 + vr0 + i) * kSsN2 + vj] = abc[q][i];
    }
    __syncthreads();

    // horizontal pass of A, B, C: rows 0..41, columns 0..31 (column c centred on c + 5)
    for (int u = tid; u < kSsN2 * (kSsT / kSsH2); u += 256) {
      const int r = u / (kSsT / kSsH2), c0 = (u - r * (kSsT / kSsH2)) * kSsH2;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        float v[kSsH2 + 2 * kSsR];
#pragma unroll
        for (int t = 0; t < kSsH2 + 2 * kSsR; ++t) v[t] = sABC[(q * kSsN2 + r) * kSsN2 + c0 + t];
#pragma unroll
        for (int j = 0; j < kSsH2; ++j) {
          float a = 0.0f;
#pragma unroll
          for (int t = 0; t <= 2 * kSsR; ++t) a = fmaf(kSsG.g[t], v[j + t], a);
          sHA[(q * kSsN2 + r) * kSsHA + c0 + j] = a;
        }
      }
    }
    __syncthreads();

    // vertical pass and the gradient of pixel (ty0 + or0 + i, tx0 + oj)
    {
      float f[3][kSsV2];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        float v[kSsV2 + 2 * kSsR];
#pragma unroll
        for (int t = 0; t < kSsV2 + 2 * kSsR; ++t) v[t] = sHA[(q * kSsN2 + or0 + t) * kSsHA + oj];
#pragma unroll
        for (int i = 0; i < kSsV2; ++i) {
          float a = 0.0f;
#pragma unroll
          for (int t = 0; t <= 2 * kSsR; ++t) a = fmaf(kSsG.g[t], v[i + t], a);
          f[q][i] = a;
        }
      }
      const int gx = tx0 + oj;
      const float inv = 1.0f / (float)HW;
      const bool semc = cur.ch >= 3;
      const float wq = semc ? w2 : w0, lq = semc ? lambda_s : lambda;
      const float l1 = wq * (1.0f - lq) * inv * (1.0f / 3.0f);
      const float ls = -wq * lq * inv * (1.0f / 3.0f);
      float* G = gcolor + cur.pixel_base * K + (semc ? cur.ch + 1 : cur.ch) * HW;
#pragma unroll
      for (int i = 0; i < kSsV2; ++i) {
        const int gy = ty0 + or0 + i;
        if (gx < W && gy < H) {
          const float x = ox[i], y = oy[i];
          const float dS = fmaf(2.0f * x, f[1][i], fmaf(y, f[2][i], f[0][i]));
          G[(int64_t)gy * W + gx] = fmaf(ls, dS, l1 * sgn(x - y));
        }
      }
    }
    // the tile's S / (3HW), one atomic per wave
    const float part = wave_sum(ssum);
    if ((tid & 63) == 0 && part != 0.0f)
      atomicAdd(&ssim_slots[(int64_t)(cur.ch >= 3 ? n_items + cur.item : cur.item) * kSlots + (int)(cur.tile % kSlots)],
                part * (1.0f / (3.0f * (float)HW)));
    __syncthreads();                                // LDS is rewritten by the next unit
    cur = nxt;
  }
}

// Level `level` of every view from the level above (item - 1 of the same view).
__global__ void k_downsample(const gs_item* __restrict__ items, int n_items, int64_t P, int level, int K,
                             float* __restrict__ img) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= P) return;
  const int item = item_of_pixel(items, n_items, pix);
  const gs_item it = items[item];
  if (it.level != level) return;
  const gs_item up = items[item - 1];
  const int64_t HW = (int64_t)it.W * it.H, HWu = (int64_t)up.W * up.H;
  const int64_t p = pix - it.pixel_base;
  const int x = (int)(p % it.W), y = (int)(p / it.W);
  const int64_t q = (int64_t)(2 * y) * up.W + 2 * x;
  const float* src = img + up.pixel_base * K;
  float* dst = img + it.pixel_base * K;
  for (int ch = 0; ch < K; ++ch) {
    const float* s = src + ch * HWu + q;
    const float a = s[0], b = s[1], c = s[up.W], d = s[up.W + 1];
    float r;
    if (ch == 3) {
      float sum = 0.0f, cnt = 0.0f;
      if (a > 0.0f) { sum += a; cnt += 1.0f; }
      if (b > 0.0f) { sum += b; cnt += 1.0f; }
      if (c > 0.0f) { sum += c; cnt += 1.0f; }
      if (d > 0.0f) { sum += d; cnt += 1.0f; }
      r = cnt > 0.0f ? sum / cnt : 0.0f;
    } else {
      r = ((a + b) + (c + d)) * 0.25f;
    }
    dst[ch * HW + p] = r;
  }
}

__global__ void k_argmax_labels(const gs_item* __restrict__ items, int n_items, int64_t P, int K,
                                const float* __restrict__ img, int32_t* __restrict__ labels) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= P) return;
  const int item = item_of_pixel(items, n_items, pix);
  const gs_item it = items[item];
  const int64_t HW = (int64_t)it.W * it.H;
  const float* s = img + it.pixel_base * K + (pix - it.pixel_base) + 4 * HW;
  int best = 0;
  float bv = s[0];
  for (int c = 1; c < K - 4; ++c) {
    const float v = s[c * HW];
    if (v > bv) { bv = v; best = c; }
  }
  labels[pix] = best;
}

}  // namespace

// Zeroes up to four arrays in one launch (grid-stride over their concatenation).
struct ZeroList {
  float* p[4];
  int64_t end[4];   // running totals of the lengths
};
__global__ __launch_bounds__(256) void k_zero_multi(ZeroList z) {
  const int64_t tot = z.end[3];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (i >= z.end[0]) + (i >= z.end[1]) + (i >= z.end[2]);
    z.p[k][i - (k > 0 ? z.end[k - 1] : 0)] = 0.0f;
  }
}

int launch_zero_f32(float* const* p, const int64_t* n, int count, hipStream_t s) {
  ZeroList z{};
  int64_t run = 0;
  for (int k = 0; k < 4; ++k) {
    const bool use = k < count && p[k] && n[k] > 0;
    z.p[k] = use ? p[k] : nullptr;
    run += use ? n[k] : 0;
    z.end[k] = run;
  }
  if (run == 0) return GS_OK;
  const int64_t blocks = std::min<int64_t>(ceil_div(run, 256), 4096);
  hipLaunchKernelGGL(k_zero_multi, dim3((unsigned)blocks), dim3(256), 0, s, z);
  return launch_status();
}

int launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return GS_OK;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, p, n, v);
  return launch_status();
}

size_t head_bwd_workspace();
int launch_head_loss(const gs_item* items, int n_items, int64_t P, int K, const gs_head& h, const float* color,
                     const gs_targets& t, float w0, float w2, bool rgb_grad, int n_slots, float* loss_slots,
                     float* count_slots, float* gcolor, float* partial, float* gW1, float* gb1, float* gW2, float* gb2,
                     hipStream_t s);

// Workspace: count slots [n][kSlots], loss slots [n][3][kSlots], SSIM slots [2n][kSlots]
// (colour, then semantic colour), n_valid [n], then the SSIM tile prefix [n + 1] (int64,
// 8-byte aligned), then the learned head's per-block weight-gradient partials (256-byte
// aligned).
static size_t loss_prefix_offset(int n_items) {
  return (sizeof(float) * (size_t)std::max(n_items, 1) * (6 * kSlots + 1) + 7) / 8 * 8;
}
static size_t loss_head_offset(int n_items) {
  return align_up(loss_prefix_offset(n_items) + sizeof(int64_t) * ((size_t)n_items + 1));
}
size_t loss_workspace(int n_items) { return loss_head_offset(n_items) + head_bwd_workspace(); }

// lambda_s is used only with a semantic colour target (t.sem_color, eq. 12).
int launch_loss(const gs_item* items, int n_items, int64_t P, int K, int n_classes, const float* color,
                const float* logits, const gs_targets& t, const gs_head* head, const float* w, float lambda,
                float lambda_s, float* loss, float* gcolor, float* glogits, const gs_grads* head_grads, float* ws,
                hipStream_t s) {
  const unsigned pb = (unsigned)std::max<int64_t>(1, ceil_div(P, 256));
  float* count_slots = ws;                                   // [n_items][kSlots]
  float* loss_slots = ws + (int64_t)n_items * kSlots;        // [n_items][3][kSlots]
  float* ssim_slots = ws + (int64_t)n_items * 4 * kSlots;    // [2 n_items][kSlots]
  float* nvalid = ws + (int64_t)n_items * 6 * kSlots;        // [n_items]
  int64_t* prefix = (int64_t*)((char*)ws + loss_prefix_offset(n_items));
  const float* tsem = t.sem_color;
  if (!tsem) lambda_s = 0.0f;
  const bool ssim = lambda != 0.0f, ssim_s = lambda_s != 0.0f;
  launch_fill_f32(ws, (int64_t)n_items * 6 * kSlots, 0.0f, s);
#define GS_LOSS_ARGS items, n_items, P, K, n_classes, color, logits, t.rgb, t.depth, t.label, tsem, w[0], w[2], \
                     !ssim, !ssim_s, loss_slots, count_slots, gcolor, glogits
  if (head) {
    float* partial = (float*)((char*)ws + loss_head_offset(n_items));
    const int st = launch_head_loss(items, n_items, P, K, *head, color, t, w[0], w[2], !ssim, kSlots, loss_slots,
                                    count_slots, gcolor, partial, head_grads->head_W1, head_grads->head_b1,
                                    head_grads->head_W2, head_grads->head_b2, s);
    if (st) return st;
  } else if (n_classes == 0) hipLaunchKernelGGL(k_loss<0>, dim3(pb), dim3(256), 0, s, GS_LOSS_ARGS);
  else if (n_classes <= 16) hipLaunchKernelGGL(k_loss<16>, dim3(pb), dim3(256), 0, s, GS_LOSS_ARGS);
  else if (n_classes <= 32) hipLaunchKernelGGL(k_loss<32>, dim3(pb), dim3(256), 0, s, GS_LOSS_ARGS);
  else if (n_classes <= 64) hipLaunchKernelGGL(k_loss<64>, dim3(pb), dim3(256), 0, s, GS_LOSS_ARGS);
  else return GS_ERR_UNSUPPORTED;
#undef GS_LOSS_ARGS
  if (ssim || ssim_s) {
    // one launch over the colour channels (0..2), the semantic colour ones (3..5) or both
    const int c0 = ssim ? 0 : 3, nch = (ssim && ssim_s) ? 6 : 3;
    hipLaunchKernelGGL(k_ssim_prefix, dim3(1), dim3(256), 0, s, items, n_items, prefix);
    // a grid-stride loop covers every (tile, channel); the grid only needs to fill the chip
    const int resident = resident_blocks(k_ssim, 256, 512);
    const int64_t est = nch * (ceil_div(P, kSsT * kSsT) + n_items);
    const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(est, 1), resident);
    hipLaunchKernelGGL(k_ssim, dim3(grid), dim3(256), 0, s, items, n_items, prefix, K, nch, c0, color, t.rgb, tsem,
                       w[0], lambda, w[2], lambda_s, ssim_slots, gcolor);
  }
  hipLaunchKernelGGL(k_fold_loss, dim3(1), dim3(256), 0, s, loss_slots, count_slots, ssim_slots, lambda, lambda_s,
                     n_items, loss, nvalid);
  hipLaunchKernelGGL(k_scale_depth, dim3(pb), dim3(256), 0, s, items, n_items, P, K, w[1], nvalid, gcolor);
  return launch_status();
}

int launch_downsample(const gs_item* items, int n_items, int64_t P, int max_level, int K, float* img, int32_t* labels,
                      hipStream_t s) {
  const unsigned pb = (unsigned)std::max<int64_t>(1, ceil_div(P, 256));
  for (int l = 1; l <= max_level; ++l)
    hipLaunchKernelGGL(k_downsample, dim3(pb), dim3(256), 0, s, items, n_items, P, l, K, img);
  if (labels && K > 4) hipLaunchKernelGGL(k_argmax_labels, dim3(pb), dim3(256), 0, s, items, n_items, P, K, img, labels);
  return launch_status();
}

}  // namespace gs
