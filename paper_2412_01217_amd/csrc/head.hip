// Learned semantic head: logits = W2 relu(W1 E + b1) + b2 per pixel, where E is the
// composited 16-wide embedding (eq. 9 with an embedding in place of class logits),
// W1 [64][16] and W2 [C][64] bfloat16, biases float32. Forward and backward run on
// matrix cores as v_mfma_f32_32x32x8bf16_1k. Single-precision activations enter the
// bfloat16 products as a hi + lo pair (x = bf16(x) + bf16(x - bf16(x))), which keeps
// the decode within ~2^-16 of single precision; products of two single-precision
// factors (weight gradients) use hi*hi + hi*lo + lo*hi.
//
// 32x32x8 bf16 operand layout (lane l): A[i][k]: i = l % 32, k = 4 (l / 32) + 0..3;
// B[k][j]: k = 4 (l / 32) + 0..3, j = l % 32; D as the 32x32 f32 layout
// (j = l % 32, i = 8 (r / 4) + 4 (l / 32) + r % 4). Computing the transposed
// activations H^T = W1 E^T leaves, in registers 4g..4g+3 of a lane, exactly the four
// hidden units that form the B operand of the next product's k-step g, so layers chain
// without a transpose.
#include "common.h"

namespace gs {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef short v4s __attribute__((ext_vector_type(4)));

constexpr int kDin = 16;
constexpr int kHid = 64;
constexpr int kHeadBlocksMax = 1024;
// per-block partial of the weight gradients: dW2 [64][64], dW1 [64][32] (column 16 = db1), db2 [64]
constexpr int kPartW2 = 64 * 64;
constexpr int kPartW1 = 64 * 32;
constexpr int kPartB2 = 64;
constexpr int kPart = kPartW2 + kPartW1 + kPartB2;

__device__ __forceinline__ int drow(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Splits four floats into hi and lo bfloat16 operands.
__device__ __forceinline__ void split4(const float* x, v4s& hi, v4s& lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint16_t h = bf16_rne(x[j]);
    hi[j] = (short)h;
    lo[j] = (short)bf16_rne(x[j] - bf16_f(h));
  }
}

__device__ __forceinline__ v16f mfma(v4s a, v4s b, v16f c) { return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0); }

__device__ __forceinline__ v16f zero16() {
  v16f z;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[r] = 0.0f;
  return z;
}

struct PixelRef {     // where one global pixel's channel c lives in a planar image
  int64_t base;       // pixel_base * channels + local index
  int64_t HW;
  bool live;
};

__device__ __forceinline__ PixelRef pixel_ref(const gs_item* items, int n_items, int64_t P, int64_t pix, int channels) {
  PixelRef r;
  r.live = pix < P;
  if (!r.live) { r.base = 0; r.HW = 0; return r; }
  const gs_item it = items[item_of_pixel(items, n_items, pix)];
  r.HW = (int64_t)it.W * it.H;
  r.base = it.pixel_base * channels + (pix - it.pixel_base);
  return r;
}

// Layer 1 for the wave's 64 pixels: H^T[hb][pb] = W1 E^T (pre-activation, bias added).
__device__ __forceinline__ void layer1(const gs_item* items, int n_items, int64_t P, int64_t wave_pix, int K,
                                       const float* __restrict__ color, const uint16_t* __restrict__ W1,
                                       const float* __restrict__ b1, v16f (&H)[2][2]) {
  const int lane = threadIdx.x & 63;
  // A = W1 (i = hidden l%32 + 32 hb, k = d 8 ks + 4 (l/32) + 0..3): exact bfloat16
  v4s a[2][2];
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        a[hb][ks][j] = (short)W1[((lane & 31) + 32 * hb) * kDin + 8 * ks + 4 * (lane >> 5) + j];
#pragma unroll
  for (int pb = 0; pb < 2; ++pb) {
    const PixelRef pr = pixel_ref(items, n_items, P, wave_pix + (lane & 31) + 32 * pb, K);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      float e[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) e[j] = pr.live ? color[pr.base + (4 + 8 * ks + 4 * (lane >> 5) + j) * pr.HW] : 0.0f;
      v4s hi, lo;
      split4(e, hi, lo);
#pragma unroll
      for (int hb = 0; hb < 2; ++hb) {
        if (ks == 0) H[hb][pb] = zero16();
        H[hb][pb] = mfma(a[hb][ks], hi, H[hb][pb]);
        H[hb][pb] = mfma(a[hb][ks], lo, H[hb][pb]);
      }
    }
  }
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float bias = b1[drow(r, lane) + 32 * hb];
      H[hb][0][r] += bias;
      H[hb][1][r] += bias;
    }
}

// B operand (k = hidden 8 ks + 4 (l/32) + 0..3, j = pixel) of k-step ks from H^T registers.
__device__ __forceinline__ void hidden_operand(const v16f (&X)[2][2], int pb, int ks, v4s& hi, v4s& lo) {
  const int hb = ks >> 2, g = ks & 3;
  float x[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = X[hb][pb][4 * g + j];
  split4(x, hi, lo);
}

__global__ __launch_bounds__(256) void k_head_fwd(const gs_item* __restrict__ items, int n_items, int64_t P, int K,
                                                  int C, const float* __restrict__ color,
                                                  const uint16_t* __restrict__ W1, const float* __restrict__ b1,
                                                  const uint16_t* __restrict__ W2, const float* __restrict__ b2,
                                                  float* __restrict__ logits) {
  const int lane = threadIdx.x & 63;
  const int64_t wave_pix = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
  if (wave_pix >= P) return;
  v16f H[2][2];
  layer1(items, n_items, P, wave_pix, K, color, W1, b1, H);
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
      for (int r = 0; r < 16; ++r) H[hb][pb][r] = fmaxf(H[hb][pb][r], 0.0f);
  // logits^T[cb][pb] = W2 h^T: A = W2 (i = class l%32 + 32 cb, k = hidden 8 ks + 4 (l/32) + 0..3)
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int cls = (lane & 31) + 32 * cb;
    v16f L[2] = {zero16(), zero16()};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      v4s a;
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = cls < C ? (short)W2[(int64_t)cls * kHid + 8 * ks + 4 * (lane >> 5) + j] : (short)0;
#pragma unroll
      for (int pb = 0; pb < 2; ++pb) {
        v4s hi, lo;
        hidden_operand(H, pb, ks, hi, lo);
        L[pb] = mfma(a, hi, L[pb]);
        L[pb] = mfma(a, lo, L[pb]);
      }
    }
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) {
      const PixelRef pr = pixel_ref(items, n_items, P, wave_pix + (lane & 31) + 32 * pb, C);
      if (!pr.live) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = drow(r, lane) + 32 * cb;
        if (c < C) logits[pr.base + c * pr.HW] = L[pb][r] + b2[c];
      }
    }
  }
}

// Writes the wave's 64 x 64 H^T-layout registers to LDS as [row][pixel] (row-major, 64 pixels).
__device__ __forceinline__ void store_T(float* sh, const v16f (&X)[2][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
      for (int r = 0; r < 16; ++r) sh[(drow(r, lane) + 32 * hb) * 65 + (lane & 31) + 32 * pb] = X[hb][pb][r];
}

// Backward of the head for one wave of 64 pixels. dE goes to the colour-gradient planes
// 4..19; the weight gradients accumulate into the block's LDS partial `acc`.
__global__ __launch_bounds__(256) void k_head_bwd(const gs_item* __restrict__ items, int n_items, int64_t P, int K,
                                                  int C, const float* __restrict__ color,
                                                  const float* __restrict__ glogits, const uint16_t* __restrict__ W1,
                                                  const float* __restrict__ b1, const uint16_t* __restrict__ W2,
                                                  float* __restrict__ gcolor, float* __restrict__ partial) {
  __shared__ float s_acc[kPart];
  __shared__ float s_t[4][64 * 65];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < kPart; i += 256) s_acc[i] = 0.0f;
  __syncthreads();
  float* sh = s_t[wave];
  const int64_t n_chunks = (P + 255) / 256;
  for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    const int64_t wave_pix = chunk * 256 + wave * 64;
    if (wave_pix >= P) continue;
    v16f H[2][2];
    layer1(items, n_items, P, wave_pix, K, color, W1, b1, H);
    // dH^T = W2^T dlogits^T: A = W2^T (i = hidden l%32 + 32 hb, k = class 8 ks + 4 (l/32) + 0..3)
    v16f dH[2][2];
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
#pragma unroll
      for (int pb = 0; pb < 2; ++pb) dH[hb][pb] = zero16();
    PixelRef prc[2];
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) prc[pb] = pixel_ref(items, n_items, P, wave_pix + (lane & 31) + 32 * pb, C);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      v4s a[2];
#pragma unroll
      for (int hb = 0; hb < 2; ++hb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int cls = 8 * ks + 4 * (lane >> 5) + j;
          a[hb][j] = cls < C ? (short)W2[(int64_t)cls * kHid + (lane & 31) + 32 * hb] : (short)0;
        }
#pragma unroll
      for (int pb = 0; pb < 2; ++pb) {
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int cls = 8 * ks + 4 * (lane >> 5) + j;
          x[j] = (prc[pb].live && cls < C) ? glogits[prc[pb].base + cls * prc[pb].HW] : 0.0f;
        }
        v4s hi, lo;
        split4(x, hi, lo);
#pragma unroll
        for (int hb = 0; hb < 2; ++hb) {
          dH[hb][pb] = mfma(a[hb], hi, dH[hb][pb]);
          dH[hb][pb] = mfma(a[hb], lo, dH[hb][pb]);
        }
      }
    }
    // ReLU' (0 at 0) and the activations h
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
#pragma unroll
      for (int pb = 0; pb < 2; ++pb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const bool on = H[hb][pb][r] > 0.0f;
          dH[hb][pb][r] = on ? dH[hb][pb][r] : 0.0f;
          H[hb][pb][r] = on ? H[hb][pb][r] : 0.0f;
        }
    // dE^T = W1^T dH^T: A = W1^T (i = d l%32, k = hidden 8 ks + 4 (l/32) + 0..3)
    {
      v16f dE[2] = {zero16(), zero16()};
      const int d = lane & 31;
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        v4s a;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          a[j] = d < kDin ? (short)W1[(8 * ks + 4 * (lane >> 5) + j) * kDin + d] : (short)0;
#pragma unroll
        for (int pb = 0; pb < 2; ++pb) {
          v4s hi, lo;
          hidden_operand(dH, pb, ks, hi, lo);
          dE[pb] = mfma(a, hi, dE[pb]);
          dE[pb] = mfma(a, lo, dE[pb]);
        }
      }
#pragma unroll
      for (int pb = 0; pb < 2; ++pb) {
        const PixelRef pr = pixel_ref(items, n_items, P, wave_pix + (lane & 31) + 32 * pb, K);
        if (!pr.live) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int dd = drow(r, lane);
          if (dd < kDin) gcolor[pr.base + (4 + dd) * pr.HW] = dE[pb][r];
        }
      }
    }
    // Weight gradients, contractions over the wave's pixels (k = pixel 8 ks + 4 (l/32) + 0..3).
    // dW2[c][h] = sum_p dlogits[c][p] h[h][p]; db2[c] = sum_p dlogits[c][p]
    store_T(sh, H);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int cls = (lane & 31) + 32 * cb;
      v16f dW[2] = {zero16(), zero16()};
      v16f dB = zero16();
      v4s ones;
#pragma unroll
      for (int j = 0; j < 4; ++j) ones[j] = (short)0x3F80;   // bfloat16 1.0
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const PixelRef pr = pixel_ref(items, n_items, P, wave_pix + 8 * ks + 4 * (lane >> 5) + j, C);
          x[j] = (pr.live && cls < C) ? glogits[pr.base + cls * pr.HW] : 0.0f;
        }
        v4s ahi, alo;
        split4(x, ahi, alo);
#pragma unroll
        for (int hb = 0; hb < 2; ++hb) {
          float y[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) y[j] = sh[((lane & 31) + 32 * hb) * 65 + 8 * ks + 4 * (lane >> 5) + j];
          v4s bhi, blo;
          split4(y, bhi, blo);
          dW[hb] = mfma(ahi, bhi, dW[hb]);
          dW[hb] = mfma(ahi, blo, dW[hb]);
          dW[hb] = mfma(alo, bhi, dW[hb]);
        }
        dB = mfma(ahi, ones, dB);
        dB = mfma(alo, ones, dB);
      }
      // D[c][h]: lane holds h = l%32 + 32 hb, c = drow(r, l) + 32 cb
#pragma unroll
      for (int hb = 0; hb < 2; ++hb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int c = drow(r, lane) + 32 * cb;
          atomicAdd(&s_acc[c * 64 + (lane & 31) + 32 * hb], dW[hb][r]);
        }
      if ((lane & 31) == 0)
#pragma unroll
        for (int r = 0; r < 16; ++r) atomicAdd(&s_acc[kPartW2 + kPartW1 + drow(r, lane) + 32 * cb], dB[r]);
    }
    // dW1[h][d] = sum_p dH[h][p] E[p][d]; column d = 16 carries db1 (E extended by a one)
    __builtin_amdgcn_wave_barrier();
    store_T(sh, dH);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
      v16f dW[2] = {zero16(), zero16()};
      const int d = lane & 31;
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        float e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t pix = wave_pix + 8 * ks + 4 * (lane >> 5) + j;
          const PixelRef pr = pixel_ref(items, n_items, P, pix, K);
          e[j] = !pr.live ? 0.0f : (d < kDin ? color[pr.base + (4 + d) * pr.HW] : (d == kDin ? 1.0f : 0.0f));
        }
        v4s bhi, blo;
        split4(e, bhi, blo);
#pragma unroll
        for (int hb = 0; hb < 2; ++hb) {
          float y[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) y[j] = sh[((lane & 31) + 32 * hb) * 65 + 8 * ks + 4 * (lane >> 5) + j];
          v4s ahi, alo;
          split4(y, ahi, alo);
          dW[hb] = mfma(ahi, bhi, dW[hb]);
          dW[hb] = mfma(ahi, blo, dW[hb]);
          dW[hb] = mfma(alo, bhi, dW[hb]);
        }
      }
      // D[h][d]: lane holds d = l%32, h = drow(r, l) + 32 hb
#pragma unroll
      for (int hb = 0; hb < 2; ++hb)
#pragma unroll
        for (int r = 0; r < 16; ++r) atomicAdd(&s_acc[kPartW2 + (drow(r, lane) + 32 * hb) * 32 + d], dW[hb][r]);
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  float* out = partial + (int64_t)blockIdx.x * kPart;
  for (int i = threadIdx.x; i < kPart; i += 256) out[i] = s_acc[i];
}

// Sums the per-block partials into the head's weight gradients.
__global__ void k_head_reduce(const float* __restrict__ partial, int n_blocks, int C, float* __restrict__ gW1,
                              float* __restrict__ gb1, float* __restrict__ gW2, float* __restrict__ gb2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kPart) return;
  float s = 0.0f;
  for (int b = 0; b < n_blocks; ++b) s += partial[(int64_t)b * kPart + i];
  if (i < kPartW2) {
    const int c = i / 64, h = i % 64;
    if (c < C) gW2[c * kHid + h] = s;
  } else if (i < kPartW2 + kPartW1) {
    const int h = (i - kPartW2) / 32, d = (i - kPartW2) % 32;
    if (d < kDin) gW1[h * kDin + d] = s;
    else if (d == kDin) gb1[h] = s;
  } else {
    const int c = i - kPartW2 - kPartW1;
    if (c < C) gb2[c] = s;
  }
}

}  // namespace

size_t head_bwd_workspace() { return sizeof(float) * (size_t)kHeadBlocksMax * kPart; }

int head_shape_ok(const gs_head& h) { return h.d_in == kDin && h.d_hidden == kHid && h.n_classes >= 1 && h.n_classes <= 64; }

int launch_head_fwd(const gs_item* items, int n_items, int64_t P, int K, const gs_head& h, const float* color,
                    float* logits, hipStream_t s) {
  if (P == 0) return GS_OK;
  const int64_t blocks = ceil_div(P, 256);
  hipLaunchKernelGGL(k_head_fwd, dim3((unsigned)blocks), dim3(256), 0, s, items, n_items, P, K, h.n_classes, color, h.W1,
                     h.b1, h.W2, h.b2, logits);
  return launch_status();
}

int launch_head_bwd(const gs_item* items, int n_items, int64_t P, int K, const gs_head& h, const float* color,
                    const float* glogits, float* gcolor, float* partial, float* gW1, float* gb1, float* gW2, float* gb2,
                    hipStream_t s) {
  if (P == 0) return GS_OK;
  const int blocks = (int)std::min<int64_t>(kHeadBlocksMax, ceil_div(P, 256));
  hipLaunchKernelGGL(k_head_bwd, dim3(blocks), dim3(256), 0, s, items, n_items, P, K, h.n_classes, color, glogits, h.W1,
                     h.b1, h.W2, gcolor, partial);
  hipLaunchKernelGGL(k_head_reduce, dim3((unsigned)ceil_div(kPart, 256)), dim3(256), 0, s, partial, blocks, h.n_classes,
                     gW1, gb1, gW2, gb2);
  return launch_status();
}

}  // namespace gs
