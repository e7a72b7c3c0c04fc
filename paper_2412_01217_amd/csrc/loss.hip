// Per-level reconstruction loss (paper eq. 10-13, L1 terms; semantics as a per-pixel
// cross-entropy on the composited class logits) and the image pyramid of the
// targets (eq. 4-6, 2x2 box means). Both are elementwise over pixels and bound by
// HBM traffic: one thread per pixel, planar channel reads coalesced along x.
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

// Item of each lane's pixel: one scalar lookup for the wave's first pixel, a per-lane
// search only where a wave straddles two items.
__device__ __forceinline__ int lane_item(const gs_item* __restrict__ items, int n_items, int64_t wave_pix0,
                                         int64_t pix) {
  const int first = item_of_pixel(items, n_items, wave_pix0);
  const gs_item it = items[first];
  const int64_t end = it.pixel_base + (int64_t)it.W * it.H;
  return pix < end ? first : item_of_pixel(items, n_items, pix);
}

// Per-item L1 colour, L1 depth over valid target depths, cross-entropy on the class
// logits, and their image gradients, in one pass over each pixel's channels. The depth
// gradient is written as sign(d) (or 0) and scaled by w1 / n_valid afterwards, once the
// valid counts are known; the logits of a pixel are held in registers (CM >= classes).
template <int CM>
__global__ __launch_bounds__(256) void k_loss(const gs_item* __restrict__ items, int n_items, int64_t P, int K,
                                              int n_classes, const float* __restrict__ color,
                                              const float* __restrict__ logits, const float* __restrict__ trgb,
                                              const float* __restrict__ tdepth, const int32_t* __restrict__ tlabel,
                                              float w0, float w2, float* __restrict__ loss_slots,
                                              float* __restrict__ count_slots, float* __restrict__ gcolor,
                                              float* __restrict__ glogits) {
  const int slot = blockIdx.x % kSlots;
  const int64_t wave_pix0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  if (wave_pix0 >= P) return;
  const int64_t pix = wave_pix0 + (threadIdx.x & 63);
  const bool live = pix < P;
  const int item = lane_item(items, n_items, wave_pix0, live ? pix : wave_pix0);
  float lr = 0.0f, ld = 0.0f, ls = 0.0f, nv = 0.0f;
  if (live) {
    const gs_item it = items[item];
    const int64_t HW = (int64_t)it.W * it.H;
    const int64_t p = pix - it.pixel_base;
    const int64_t cb = it.pixel_base * K + p;
    const float inv3 = 1.0f / (3.0f * (float)HW);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float d = color[cb + ch * HW] - trgb[it.pixel_base * 3 + ch * HW + p];
      lr += fabsf(d) * inv3;
      gcolor[cb + ch * HW] = w0 * sgn(d) * inv3;
    }
    const float td = tdepth[pix];
    float gd = 0.0f;
    if (td > 0.0f) {
      const float d = color[cb + 3 * HW] - td;
      ld = fabsf(d);
      nv = 1.0f;
      gd = sgn(d);
    }
    gcolor[cb + 3 * HW] = gd;
    if (CM > 0 && n_classes > 0) {
      // plain mode: logits are colour channels 4..; learned mode: a separate C-plane image
      const float* L = logits ? logits + it.pixel_base * n_classes + p : color + cb + 4 * HW;
      float* G = logits ? glogits + it.pixel_base * n_classes + p : gcolor + cb + 4 * HW;
      float x[CM > 0 ? CM : 1];
      float m = -INFINITY;
      const float* Lc = L;
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        x[c] = c < n_classes ? *Lc : -INFINITY;
        Lc += HW;
        m = fmaxf(m, x[c]);
      }
      const int y = tlabel[pix];
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
      float* Gc = G;
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        if (c < n_classes) *Gc = x[c] * sc - (c == y ? oh : 0.0f);
        Gc += HW;
      }
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

// Folds the slots: loss[i] = (L1 colour, L1 depth / n_valid, cross-entropy); n_valid[i].
__global__ void k_fold_loss(const float* __restrict__ loss_slots, const float* __restrict__ count_slots, int n_items,
                            float* __restrict__ loss, float* __restrict__ nvalid) {
  for (int i = threadIdx.x; i < n_items * 4; i += blockDim.x) {
    const int item = i >> 2, comp = i & 3;
    const float* src = comp < 3 ? loss_slots + (int64_t)(3 * item + comp) * kSlots : count_slots + (int64_t)item * kSlots;
    float s = 0.0f;
    for (int k = 0; k < kSlots; ++k) s += src[k];
    if (comp == 3) nvalid[item] = s;
    else if (comp != 1) loss[3 * item + comp] = s;
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
  const int item = lane_item(items, n_items, wave_pix0, pix);
  const gs_item it = items[item];
  const int64_t HW = (int64_t)it.W * it.H;
  float* g = gcolor + it.pixel_base * K + 3 * HW + (pix - it.pixel_base);
  const float nv = nvalid[item];
  *g = nv > 0.0f ? *g * (w1 / nv) : 0.0f;
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

size_t loss_workspace(int n_items) { return sizeof(float) * (size_t)std::max(n_items, 1) * (4 * kSlots + 1); }

int launch_loss(const gs_item* items, int n_items, int64_t P, int K, int n_classes, const float* color,
                const float* logits, const gs_targets& t, const float* w, float* loss, float* gcolor, float* glogits,
                float* ws, hipStream_t s) {
  const unsigned pb = (unsigned)std::max<int64_t>(1, ceil_div(P, 256));
  float* count_slots = ws;                                   // [n_items][kSlots]
  float* loss_slots = ws + (int64_t)n_items * kSlots;        // [n_items][3][kSlots]
  float* nvalid = ws + (int64_t)n_items * 4 * kSlots;        // [n_items]
  launch_fill_f32(ws, (int64_t)n_items * 4 * kSlots, 0.0f, s);
#define GS_LOSS_ARGS items, n_items, P, K, n_classes, color, logits, t.rgb, t.depth, t.label, w[0], w[2], loss_slots, \
                     count_slots, gcolor, glogits
  if (n_classes == 0) hipLaunchKernelGGL(k_loss<0>, dim3(pb), dim3(256), 0, s, GS_LOSS_ARGS);
  else if (n_classes <= 16) hipLaunchKernelGGL(k_loss<16>, dim3(pb), dim3(256), 0, s, GS_LOSS_ARGS);
  else if (n_classes <= 32) hipLaunchKernelGGL(k_loss<32>, dim3(pb), dim3(256), 0, s, GS_LOSS_ARGS);
  else if (n_classes <= 64) hipLaunchKernelGGL(k_loss<64>, dim3(pb), dim3(256), 0, s, GS_LOSS_ARGS);
  else return GS_ERR_UNSUPPORTED;
#undef GS_LOSS_ARGS
  hipLaunchKernelGGL(k_fold_loss, dim3(1), dim3(256), 0, s, loss_slots, count_slots, n_items, loss, nvalid);
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
