// Training helpers for the learned semantic head: an Adam step on float32 master
// parameters (optionally refreshing a bfloat16 copy), the distillation loss that
// fits decoded logits to the plain C-class render, and an argmax-agreement count.
// All elementwise over parameters or pixels.
#include "common.h"

namespace gs {
namespace {

__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t* __restrict__ bf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  if (bf) bf[i] = to_bf16(pi);
}

// Per pixel: soft-target cross-entropy of the student logits against softmax of the
// teacher logits, plus mse_w times the mean squared logit difference; both averaged
// over the item's pixels and summed over items. grad = d loss / d student.
__global__ __launch_bounds__(256) void k_distill(const gs_item* __restrict__ items, int n_items, int64_t P, int C,
                                                 const float* __restrict__ teacher, const float* __restrict__ student,
                                                 float mse_w, float* __restrict__ loss_slots,
                                                 float* __restrict__ grad) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (pix < P) {
    const gs_item it = items[item_of_pixel(items, n_items, pix)];
    const int64_t HW = (int64_t)it.W * it.H;
    const int64_t base = it.pixel_base * C + (pix - it.pixel_base);
    const float* t = teacher + base;
    const float* s = student + base;
    float mt = -INFINITY, ms = -INFINITY;
    for (int c = 0; c < C; ++c) {
      mt = fmaxf(mt, t[c * HW]);
      ms = fmaxf(ms, s[c * HW]);
    }
    float zt = 0.0f, zs = 0.0f;
    for (int c = 0; c < C; ++c) {
      zt += __expf(t[c * HW] - mt);
      zs += __expf(s[c * HW] - ms);
    }
    const float lzt = mt + __logf(zt), lzs = ms + __logf(zs);
    const float inv = 1.0f / (float)HW;
    const float wm = mse_w / (float)C;
    for (int c = 0; c < C; ++c) {
      const float pt = __expf(t[c * HW] - lzt);
      const float ps = __expf(s[c * HW] - lzs);
      const float d = s[c * HW] - t[c * HW];
      l += (-pt * (s[c * HW] - lzs) + wm * d * d) * inv;
      grad[base + c * HW] = (ps - pt + 2.0f * wm * d) * inv;
    }
  }
  l = wave_sum(l);
  if ((threadIdx.x & 63) == 0 && l != 0.0f) atomicAdd(&loss_slots[blockIdx.x & 63], l);
}

__global__ void k_sum_slots(const float* __restrict__ slots, float* __restrict__ out) {
  if (threadIdx.x == 0) {
    float s = 0.0f;
    for (int k = 0; k < 64; ++k) s += slots[k];
    *out = s;
  }
}

__global__ void k_fill0(float* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// Counts pixels whose argmax over C planar channels agrees between a and b
// (ties to the lowest index) into counts[item].
__global__ void k_agree(const gs_item* __restrict__ items, int n_items, int64_t P, int C, const float* __restrict__ a,
                        const float* __restrict__ b, unsigned long long* __restrict__ counts) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= P) return;
  const int item = item_of_pixel(items, n_items, pix);
  const gs_item it = items[item];
  const int64_t HW = (int64_t)it.W * it.H;
  const int64_t base = it.pixel_base * C + (pix - it.pixel_base);
  int ia = 0, ib = 0;
  float va = a[base], vb = b[base];
  for (int c = 1; c < C; ++c) {
    const float x = a[base + c * HW], y = b[base + c * HW];
    if (x > va) { va = x; ia = c; }
    if (y > vb) { vb = y; ib = c; }
  }
  if (ia == ib) atomicAdd(&counts[item], 1ull);
}

}  // namespace

int launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                int step, uint16_t* bf, hipStream_t s) {
  if (n == 0) return GS_OK;
  const float c1 = 1.0f / (1.0f - powf(b1, (float)step));
  const float c2 = 1.0f / (1.0f - powf(b2, (float)step));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2, bf);
  return launch_status();
}

int launch_distill(const gs_item* items, int n_items, int64_t P, int C, const float* teacher, const float* student,
                   float mse_w, float* loss, float* grad, float* slots, hipStream_t s) {
  hipLaunchKernelGGL(k_fill0, dim3(1), dim3(64), 0, s, slots, 64);
  if (P > 0)
    hipLaunchKernelGGL(k_distill, dim3((unsigned)ceil_div(P, 256)), dim3(256), 0, s, items, n_items, P, C, teacher,
                       student, mse_w, slots, grad);
  hipLaunchKernelGGL(k_sum_slots, dim3(1), dim3(64), 0, s, slots, loss);
  return launch_status();
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

int launch_agree(const gs_item* items, int n_items, int64_t P, int C, const float* a, const float* b,
                 unsigned long long* counts, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)ceil_div(std::max(n_items, 1), 256)), dim3(256), 0, s, counts, n_items);
  if (P == 0) return launch_status();
  hipLaunchKernelGGL(k_agree, dim3((unsigned)ceil_div(P, 256)), dim3(256), 0, s, items, n_items, P, C, a, b, counts);
  return launch_status();
}

}  // namespace gs
