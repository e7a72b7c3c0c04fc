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
constexpr int kHeadBlocksMax = 512;
// per-block partial of the weight gradients: dW2 [64][64], dW1 [64][32] (column 16 = db1), db2 [64]
constexpr int kPartW2 = 64 * 64;
constexpr int kPartW1 = 64 * 32;
constexpr int kPartB2 = 64;
constexpr int kPart = kPartW2 + kPartW1 + kPartB2;
constexpr int kWtStride = kHid + 8;   // bfloat16 row stride of the transposed weights in LDS (16-byte rows)

__device__ __forceinline__ int drow(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Splits four floats into hi and lo bfloat16 operands (hardware round-to-nearest-even).
__device__ __forceinline__ void split4(const float* x, v4s& hi, v4s& lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const __bf16 h = (__bf16)x[j];
    const __bf16 l = (__bf16)(x[j] - (float)h);
    hi[j] = __builtin_bit_cast(short, h);
    lo[j] = __builtin_bit_cast(short, l);
  }
}

__device__ __forceinline__ v16f mfma(v4s a, v4s b, v16f c) { return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0); }

// Two consecutive k-steps of 32x32x8 as one v_mfma_f32_32x32x16_bf16 (twice the work per
// instruction on gfx950): lane (l % 32, h = l / 32) supplies k = 8 h + 0..7 of the 16; given
// k-step pairs whose lane h holds k = 8 (2s) + 4 h + 0..3 and 8 (2s + 1) + 4 h + 0..3 (the
// layout above), the concatenation [step 2s, step 2s + 1] covers each k of the pair once in
// both operands, so the product is the same sum over the 16 k.
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
__device__ __forceinline__ v16f mfma2(v8s a, v8s b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}
__device__ __forceinline__ v8s cat(v4s x0, v4s x1) { return __builtin_shufflevector(x0, x1, 0, 1, 2, 3, 4, 5, 6, 7); }
__device__ __forceinline__ v16f mfma2(v4s a0, v4s a1, v4s b0, v4s b1, v16f c) { return mfma2(cat(a0, a1), cat(b0, b1), c); }
__device__ __forceinline__ v16f mfma2(v8s a, v4s b0, v4s b1, v16f c) { return mfma2(a, cat(b0, b1), c); }
__device__ __forceinline__ v16f mfma2(v4s a0, v4s a1, v8s b, v16f c) { return mfma2(cat(a0, a1), b, c); }

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

// Walks the 64-pixel chunks of the concatenated items in increasing order. Chunks
// never straddle two items, so every pixel of a chunk shares one item's plane layout.
struct ChunkCursor {
  int item;
  int64_t first, end;   // chunks [first, end) belong to `item`
};

__device__ __forceinline__ int64_t item_chunks(const gs_item& it) { return ((int64_t)it.W * it.H + 63) / 64; }

// Moves the cursor forward to the item holding `chunk`; false once past the last item.
__device__ __forceinline__ bool seek_chunk(const gs_item* __restrict__ items, int n_items, int64_t chunk,
                                           ChunkCursor& cur) {
  while (chunk >= cur.end && cur.item + 1 < n_items) {
    ++cur.item;
    cur.first = cur.end;
    cur.end += item_chunks(items[cur.item]);
  }
  return chunk < cur.end;
}

// Backward of the head. Each wave takes 64-pixel chunks in a grid-stride loop. It
// stages the chunk's logit gradients in LDS ([class][pixel], classes >= C stay zero),
// then, per 32-pixel half,
//  (1) recomputes the hidden pre-activations for the ReLU mask,
//  (2) forms dH^T = W2^T dlogits^T (hidden in registers, pixels across lanes),
//  (3) adds (or stores) dE^T = W1^T dH^T to the colour-gradient planes 4..19,
//  (4) recomputes H and dH with pixels in registers and hidden units across lanes --
//      the layout in which a matrix-core product contracts over pixels -- and
//  (5) accumulates dW2 = dlogits^T relu(H), db2 and dW1 = dH^T [E, 1] (column 16 is
//      db1) in registers that live across the whole loop.
// The accumulators are summed over the block's waves in LDS once at the end and written
// as one partial per block; k_head_reduce adds the partials.
constexpr int kGst = 65;   // LDS row stride of the staged logit gradients

// The block's shared state of a head backward: transposed weights and the per-wave staging.
// The transposed weights' rows are stored with the contraction index k at kperm(k) (bits 2
// and 3 of k swapped), so that the 8 values a lane supplies to a 32x32x16 product of the
// k-step pair s (k = 16 s + 4 h + 0..3 and 16 s + 8 + 4 h + 0..3, see mfma2) are contiguous
// at 16 s + 8 h: one 16-byte LDS read.
__host__ __device__ constexpr int kperm(int k) { return (k & ~12) | ((k & 4) << 1) | ((k & 8) >> 1); }

struct alignas(16) HeadLds {
  float buf[4 * kHid * kGst];        // per wave [class][pixel]; the block's partial at the end
  uint16_t w2t[kHid * kWtStride];    // W2^T [hidden][kperm(class)], classes >= C zero
  uint16_t w1t[kDin * kWtStride];    // W1^T [d][kperm(hidden)]
  float b1[kHid];
};

// Per-lane accumulators of the weight gradients over a block's chunks.
struct HeadAcc {
  v16f W2[2][2], W1[2];   // W2[cb][hb]: D[c][h]; W1[hb]: D[h][d]
  float B2[2];            // class l32 + 32 cb, this lane's pixels
};

__device__ __forceinline__ void head_setup(HeadLds& L, int C, const uint16_t* __restrict__ W1,
                                           const float* __restrict__ b1, const uint16_t* __restrict__ W2,
                                           HeadAcc& acc, v4s (&w1a)[2][2], float (&b1l)[2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5, l32 = lane & 31;
  for (int i = threadIdx.x; i < kHid * kHid; i += 256) {
    const int c = i / kHid, h = i % kHid;
    L.w2t[h * kWtStride + kperm(c)] = c < C ? W2[c * kHid + h] : (uint16_t)0;
  }
  for (int i = threadIdx.x; i < kHid * kDin; i += 256) {
    const int h = i / kDin, d = i % kDin;
    L.w1t[d * kWtStride + kperm(h)] = W1[h * kDin + d];
  }
  if (threadIdx.x < kHid) L.b1[threadIdx.x] = b1[threadIdx.x];
  float* sg = L.buf + wave * kHid * kGst;
  for (int i = C * kGst + lane; i < kHid * kGst; i += 64) sg[i] = 0.0f;   // rows of absent classes
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    acc.W1[i] = zero16();
    acc.W2[i][0] = zero16();
    acc.W2[i][1] = zero16();
    acc.B2[i] = 0.0f;
  }
  // W1 as A (i = hidden l32 + 32 hb, k = d 8 ks + 4 half + j), which is also W1^T as B (k = d, j = hidden)
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int j = 0; j < 4; ++j) w1a[hb][ks][j] = (short)W1[(l32 + 32 * hb) * kDin + 8 * ks + 4 * half + j];
  b1l[0] = L.b1[l32];
  b1l[1] = L.b1[l32 + 32];
}

// Steps (1)-(5) for one 64-pixel chunk whose logit gradients are staged in sg [class][pixel].
// Eb: pixel 0 of plane 0 of the chunk's embedding, plane d at Eb + d es (es = HW in global
// memory; the row stride when staged in LDS, whose 64 entries per row are all readable);
// dEb: the chunk's gradient planes (plane d at dEb + d HW). on_in (LDS_E, the fused loss):
// the ReLU masks its decode formed, [half][hb] bit r for hidden unit drow(r) + 32 hb, in
// place of step (1)'s recomputation.
template <bool ADD, bool LDS_E>
__device__ __forceinline__ void head_chunk_backward(const HeadLds& L, const float* sg, const float* Eb, int64_t es,
                                                    float* dEb, int64_t HW, int nlive, const v4s (&w1a)[2][2],
                                                    const float (&b1l)[2], HeadAcc& acc,
                                                    const uint32_t (*on_in)[2] = nullptr) {
  const int lane = threadIdx.x & 63, half = lane >> 5, l32 = lane & 31;
#pragma unroll 1
  for (int pb = 0; pb < 2; ++pb) {
    const int q = l32 + 32 * pb;
    const bool qlive = q < nlive;
    const float* Eq = Eb + 4 * half * es + min(q, nlive - 1);   // plane 8 ks + 4 half + j at Eq + (8 ks + j) es
    const float* Gq = sg + 4 * half * kGst + q;                 // class 8 ks + 4 half + j at Gq + (8 ks + j) kGst
    // (1) E with d in registers, pixels across lanes; the sign of the hidden pre-activations
    v4s ehi[2], elo[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      float e[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float v = Eq[(8 * ks + j) * es];
        e[j] = qlive ? v : 0.0f;
      }
      split4(e, ehi[ks], elo[ks]);
    }
    uint32_t on[2];   // bit r: hidden unit drow(r) + 32 hb is active at this pixel
    if constexpr (LDS_E) {
      on[0] = pb ? on_in[1][0] : on_in[0][0];
      on[1] = pb ? on_in[1][1] : on_in[0][1];
    } else {
#pragma unroll
      for (int hb = 0; hb < 2; ++hb) {
        v16f h;
#pragma unroll
        for (int r = 0; r < 16; ++r) h[r] = L.b1[drow(r, lane) + 32 * hb];
        h = mfma2(w1a[hb][0], w1a[hb][1], ehi[0], ehi[1], h);
        h = mfma2(w1a[hb][0], w1a[hb][1], elo[0], elo[1], h);
        uint32_t bits = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) bits |= (h[r] > 0.0f ? 1u : 0u) << r;
        on[hb] = bits;
      }
    }

    // (2) dH^T = W2^T dlogits^T: A = W2^T (i = hidden l32 + 32 hb, k = class 8 ks + 4 half + j)
    v16f dHT[2] = {zero16(), zero16()};
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      v4s hi[2], lo[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ks = 2 * s2 + u;
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = Gq[(8 * ks + j) * kGst];
        split4(x, hi[u], lo[u]);
      }
#pragma unroll
      for (int hb = 0; hb < 2; ++hb) {
        const v8s a = *reinterpret_cast<const v8s*>(L.w2t + (l32 + 32 * hb) * kWtStride + 16 * s2 + 8 * half);
        dHT[hb] = mfma2(a, hi[0], hi[1], dHT[hb]);
        dHT[hb] = mfma2(a, lo[0], lo[1], dHT[hb]);
      }
    }
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
#pragma unroll
      for (int r = 0; r < 16; ++r) dHT[hb][r] = ((on[hb] >> r) & 1u) ? dHT[hb][r] : 0.0f;

    // (3) dE^T = W1^T dH^T: A = W1^T (i = d l32, k = hidden 8 ks + 4 half + j); B from the
    // dH^T registers 4 (ks % 4) .. +3 of block ks / 4
    {
      v16f dE = zero16();
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        v8s a = {0, 0, 0, 0, 0, 0, 0, 0};
        if (l32 < kDin) a = *reinterpret_cast<const v8s*>(L.w1t + l32 * kWtStride + 16 * s2 + 8 * half);
        v4s hi[2], lo[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int ks = 2 * s2 + u;
          float x[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) x[j] = dHT[ks >> 2][4 * (ks & 3) + j];
          split4(x, hi[u], lo[u]);
        }
        dE = mfma2(a, hi[0], hi[1], dE);
        dE = mfma2(a, lo[0], lo[1], dE);
      }
      // rows 0..15 = d: added to what the caller's gradient holds there, or stored
      if (qlive)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          float* dst = dEb + (int64_t)drow(r, lane) * HW + q;
          if constexpr (ADD) *dst += dE[r];
          else *dst = dE[r];
        }
    }

    // Reloading from LDS below is cheaper than keeping (2)'s operands alive through (3).
    asm volatile("" ::: "memory");
    // (4) H with pixels in registers: A = E (i = pixel), B = W1^T (k = d, j = hidden l32 + 32 hb)
    v16f H[2];
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      H[hb] = mfma2(ehi[0], ehi[1], w1a[hb][0], w1a[hb][1], zero16());
      H[hb] = mfma2(elo[0], elo[1], w1a[hb][0], w1a[hb][1], H[hb]);
#pragma unroll
      for (int r = 0; r < 16; ++r) H[hb][r] = fmaxf(H[hb][r] + b1l[hb], 0.0f);
    }
    // (5a) dW2[c][h] += sum_p dlogits[c][p] relu(H)[p][h] over the half's pixels
    // p = 32 pb + 8 kk + 4 half + j (registers 4 kk + j): A = dlogits (i = class l32 + 32 cb, k = p)
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) {
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        v4s ahi[2], alo[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int p0 = 32 * pb + 8 * (2 * k2 + u) + 4 * half;
          float x[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) x[j] = sg[(l32 + 32 * cb) * kGst + p0 + j];
          acc.B2[cb] += (x[0] + x[1]) + (x[2] + x[3]);
          split4(x, ahi[u], alo[u]);
        }
#pragma unroll
        for (int hb = 0; hb < 2; ++hb) {
          v4s bhi[2], blo[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            float y[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) y[j] = H[hb][4 * (2 * k2 + u) + j];
            split4(y, bhi[u], blo[u]);
          }
          acc.W2[cb][hb] = mfma2(ahi[0], ahi[1], bhi[0], bhi[1], acc.W2[cb][hb]);
          acc.W2[cb][hb] = mfma2(ahi[0], ahi[1], blo[0], blo[1], acc.W2[cb][hb]);
          acc.W2[cb][hb] = mfma2(alo[0], alo[1], bhi[0], bhi[1], acc.W2[cb][hb]);
        }
      }
    }
    uint32_t onH[2];   // bit r: hidden unit l32 + 32 hb is active at pixel drow(r) of the half
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      uint32_t bits = 0;
#pragma unroll
      for (int r = 0; r < 16; ++r) bits |= (H[hb][r] > 0.0f ? 1u : 0u) << r;
      onH[hb] = bits;
    }
    // (4b) dH with pixels in registers: A = dlogits (i = pixel, k = class), B = W2 (j = hidden)
    v16f dH[2] = {zero16(), zero16()};
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      v4s hi[2], lo[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ks = 2 * s2 + u;
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = Gq[(8 * ks + j) * kGst];
        split4(x, hi[u], lo[u]);
      }
#pragma unroll
      for (int hb = 0; hb < 2; ++hb) {
        const v8s b = *reinterpret_cast<const v8s*>(L.w2t + (l32 + 32 * hb) * kWtStride + 16 * s2 + 8 * half);
        dH[hb] = mfma2(hi[0], hi[1], b, dH[hb]);
        dH[hb] = mfma2(lo[0], lo[1], b, dH[hb]);
      }
    }
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
#pragma unroll
      for (int r = 0; r < 16; ++r) dH[hb][r] = ((onH[hb] >> r) & 1u) ? dH[hb][r] : 0.0f;
    // (5b) dW1[h][d] += sum_p dH[p][h] [E, 1][p][d]: A = dH (i = hidden l32 + 32 hb, k = p), B = [E, 1] (j = d l32)
    const float* Ed = Eb + (int64_t)min(l32, kDin - 1) * es;
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) {
      v4s bhi[2], blo[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int p0 = 32 * pb + 8 * (2 * k2 + u) + 4 * half;
        float e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = Ed[LDS_E ? p0 + j : min(p0 + j, nlive - 1)];
          e[j] = p0 + j >= nlive ? 0.0f : (l32 < kDin ? v : (l32 == kDin ? 1.0f : 0.0f));
        }
        split4(e, bhi[u], blo[u]);
      }
#pragma unroll
      for (int hb = 0; hb < 2; ++hb) {
        v4s ahi[2], alo[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          float y[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) y[j] = dH[hb][4 * (2 * k2 + u) + j];
          split4(y, ahi[u], alo[u]);
        }
        acc.W1[hb] = mfma2(ahi[0], ahi[1], bhi[0], bhi[1], acc.W1[hb]);
        acc.W1[hb] = mfma2(ahi[0], ahi[1], blo[0], blo[1], acc.W1[hb]);
        acc.W1[hb] = mfma2(alo[0], alo[1], bhi[0], bhi[1], acc.W1[hb]);
      }
    }
  }
}

// Sums the block's four waves' accumulators in LDS and writes the block's partial.
__device__ __forceinline__ void head_write_partial(HeadLds& L, const HeadAcc& acc, float* __restrict__ partial) {
  const int lane = threadIdx.x & 63, l32 = lane & 31;
  float* s_acc = L.buf;
  __syncthreads();
  for (int i = threadIdx.x; i < kPart; i += 256) s_acc[i] = 0.0f;
  __syncthreads();
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = drow(r, lane) + 32 * cb;   // D[c][h]: h = l32 + 32 hb
        atomicAdd(&s_acc[c * 64 + l32 + 32 * hb], acc.W2[cb][hb][r]);
      }
    atomicAdd(&s_acc[kPartW2 + kPartW1 + l32 + 32 * cb], acc.B2[cb]);
  }
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int r = 0; r < 16; ++r) atomicAdd(&s_acc[kPartW2 + (drow(r, lane) + 32 * hb) * 32 + l32], acc.W1[hb][r]);
  __syncthreads();
  float* out = partial + (int64_t)blockIdx.x * kPart;
  for (int i = threadIdx.x; i < kPart; i += 256) out[i] = s_acc[i];
}

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256, 1) void k_head_bwd(const gs_item* __restrict__ items, int n_items, int K, int C,
                                                     const float* __restrict__ color,
                                                     const float* __restrict__ glogits,
                                                     const uint16_t* __restrict__ W1, const float* __restrict__ b1,
                                                     const uint16_t* __restrict__ W2, float* __restrict__ gcolor,
                                                     float* __restrict__ partial) {
  __shared__ HeadLds L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  HeadAcc acc;
  v4s w1a[2][2];
  float b1l[2];
  head_setup(L, C, W1, b1, W2, acc, w1a, b1l);
  float* sg = L.buf + wave * kHid * kGst;
  ChunkCursor cur;
  cur.item = 0;
  cur.first = 0;
  cur.end = item_chunks(items[0]);
  for (int64_t chunk = (int64_t)blockIdx.x * 4 + wave;; chunk += (int64_t)gridDim.x * 4) {
    if (!seek_chunk(items, n_items, chunk, cur)) break;
    const gs_item it = items[cur.item];
    const int64_t HW = (int64_t)it.W * it.H;
    const int64_t local0 = (chunk - cur.first) * 64;
    const int nlive = (int)min((int64_t)64, HW - local0);
    {
      // stage: lane = pixel, one coalesced row per class; dead pixels are zero
      // (16 rows' loads in flight per round trip)
      const bool live = lane < nlive;
      const float* g = glogits + it.pixel_base * C + local0 + min(lane, nlive - 1);
      for (int c0 = 0; c0 < C; c0 += 16) {
        float v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = c0 + k < C ? g[(int64_t)(c0 + k) * HW] : 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (c0 + k < C) sg[(c0 + k) * kGst + lane] = live ? v[k] : 0.0f;
      }
    }
    wave_fence();
    head_chunk_backward<true, false>(L, sg, color + it.pixel_base * K + 4 * HW + local0, HW,
                                     gcolor + it.pixel_base * K + 4 * HW + local0, HW, nlive, w1a, b1l, acc);
    // every lane is past this chunk's reads of the staged rows before the next chunk writes them
    wave_fence();
  }
  head_write_partial(L, acc, partial);
}

// Learned-mode loss with the decode fused in (paper eq. 10-13 with the semantic term a
// cross-entropy on the head's logits): per 64-pixel chunk of one item, the L1 colour and
// depth terms (lane = pixel, as in the plain loss), the decode logits = W2 relu(W1 E + b1)
// + b2 on the matrix cores, the cross-entropy against the label and its logit gradient
// w2 (softmax - onehot) / HW, staged in LDS, then the head's backward (steps (1)-(5) above)
// storing dL/dE in the colour-gradient planes 4..19 and accumulating the weight gradients.
// No logits touch global memory. Loss partial sums go to the same per-item slots as the
// plain loss's.
//
// At one wave per SIMD nothing hides a load's latency, so every input a chunk reads (the
// 16 embedding planes, colour and depth, the targets) comes from LDS: while a wave works
// on one chunk, direct global-to-LDS loads fill the other of its two staging buffers with
// its next chunk. The buffers are two separate LDS arrays and the loop handles two chunks
// per iteration, one from each, so that the compiler's wait for a buffer's loads never
// waits for the other's.
constexpr int kEst = 68;   // row stride (floats) of a staged embedding plane

struct ChunkStage {        // one wave's staged chunk: 64 pixels of every input plane
  float E[kDin][kEst];
  float col[4][64];
  float tr[3][64];
  float td[64];
  int32_t lab[64];
};

struct ChunkInfo {
  int64_t chunk, pixel_base, HW, local0;
  int item, nlive;
};

// The item table read through the constant address space: the chunk walk is wave-uniform,
// and its reads become scalar loads, which do not wait behind the vector memory queue
// (where the staging loads are in flight).
typedef const __attribute__((address_space(4))) gs_item* ConstItems;

__device__ __forceinline__ bool seek_chunk_c(ConstItems items, int n_items, int64_t chunk, ChunkCursor& cur) {
  while (chunk >= cur.end && cur.item + 1 < n_items) {
    ++cur.item;
    cur.first = cur.end;
    cur.end += ((int64_t)items[cur.item].W * items[cur.item].H + 63) / 64;
  }
  return chunk < cur.end;
}

// The chunk's place in the item table (false once past the last item).
__device__ __forceinline__ bool chunk_info(ConstItems items, int n_items, int64_t chunk, ChunkCursor& cur,
                                           ChunkInfo& ci) {
  if (!seek_chunk_c(items, n_items, chunk, cur)) return false;
  ci.chunk = chunk;
  ci.item = cur.item;
  ci.pixel_base = items[cur.item].pixel_base;
  ci.HW = (int64_t)items[cur.item].W * items[cur.item].H;
  ci.local0 = (chunk - cur.first) * 64;
  ci.nlive = (int)min((int64_t)64, ci.HW - ci.local0);
  return true;
}

constexpr int kStageLoads = kDin + 4 + 3 + 1 + 1;   // direct-to-LDS loads per staged chunk

// Waits until at most kStageLoads vector memory operations are in flight: those are the
// other buffer's loads, issued last, so everything before them -- this buffer's loads and
// the previous chunk's stores -- is complete. Vector memory operations complete in issue
// order. (s_waitcnt encoding: vmcnt 25 in bits 3:0 and 15:14, expcnt and lgkmcnt not
// waited for.)
__device__ __forceinline__ void wait_own_stage() {
  static_assert(kStageLoads == 25, "the wait below encodes vmcnt(25)");
  __builtin_amdgcn_s_waitcnt((1 << 14) | (0xF << 8) | (0x7 << 4) | 9);
}

// Issues the direct-to-LDS loads of chunk ci into S (lane l fills entry l of every row;
// lanes past the item's last pixel load that pixel again).
__device__ __forceinline__ void stage_chunk(ChunkStage& S, const ChunkInfo& ci, int K, const float* color,
                                            const float* trgb, const float* tdepth, const int32_t* tlabel) {
  const int lane = threadIdx.x & 63;
  const int64_t p = ci.local0 + min(lane, ci.nlive - 1);
  const float* cb = color + ci.pixel_base * K + p;
  // the previous chunk's reads of S are complete before the loads overwrite it
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int d = 0; d < kDin; ++d)
    __builtin_amdgcn_global_load_lds(cb + (int64_t)(4 + d) * ci.HW, &S.E[d][0], 4, 0, 0);
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) __builtin_amdgcn_global_load_lds(cb + (int64_t)ch * ci.HW, &S.col[ch][0], 4, 0, 0);
  const float* tb = trgb + ci.pixel_base * 3 + p;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) __builtin_amdgcn_global_load_lds(tb + (int64_t)ch * ci.HW, &S.tr[ch][0], 4, 0, 0);
  __builtin_amdgcn_global_load_lds(tdepth + ci.pixel_base + p, &S.td[0], 4, 0, 0);
  __builtin_amdgcn_global_load_lds(tlabel + ci.pixel_base + p, &S.lab[0], 4, 0, 0);
}

// Everything k_head_loss does for one staged chunk.
__device__ __forceinline__ void head_loss_chunk(const HeadLds& L, const uint16_t* w2r, const ChunkStage& S,
                                                const ChunkInfo& ci, float* sg, int K, int C, float w0, float w2,
                                                bool rgb_grad, int n_slots, const float (&b2r)[2][16],
                                                const v4s (&w1a)[2][2], const float (&b1l)[2], HeadAcc& acc,
                                                float* __restrict__ loss_slots, float* __restrict__ count_slots,
                                                float* __restrict__ gcolor) {
  const int lane = threadIdx.x & 63, l32 = lane & 31;
  const int64_t HW = ci.HW;
  const int nlive = ci.nlive;
  const float invp = 1.0f / (float)HW;
  wait_own_stage();
  // L1 colour and depth, lane = pixel
  const bool live = lane < nlive;
  const int64_t cbase = ci.pixel_base * K + ci.local0 + min(lane, nlive - 1);
  float col[4], tr[3];
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) col[ch] = S.col[ch][lane];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) tr[ch] = S.tr[ch][lane];
  const float td = S.td[lane];
  const int y_own = S.lab[lane];
  float lr = 0.0f, ld = 0.0f, nv = 0.0f, ls = 0.0f;
  {
    const float inv3 = 1.0f / (3.0f * (float)HW);
    float gc[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float d = col[ch] - tr[ch];
      lr += fabsf(d) * inv3;
      gc[ch] = w0 * (float)((d > 0.0f) - (d < 0.0f)) * inv3;
    }
    float gd = 0.0f;
    if (td > 0.0f) {
      const float d = col[3] - td;
      ld = fabsf(d);
      nv = 1.0f;
      gd = (float)((d > 0.0f) - (d < 0.0f));
    }
    if (live) {
      if (rgb_grad)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) __builtin_nontemporal_store(gc[ch], &gcolor[cbase + ch * HW]);
      __builtin_nontemporal_store(gd, &gcolor[cbase + 3 * HW]);
    } else {
      lr = ld = nv = 0.0f;
    }
  }
  // decode and cross-entropy per 32-pixel half: logits^T[cb][.] in D layout, lane l holding
  // pixel 32 pb + l32, classes drow(r) + 32 cb; each pixel's classes span lanes l32 and l32 + 32.
  // The hidden layer's ReLU masks are kept for the backward (the same D layout); the halves
  // are unrolled so that the masks stay in registers.
  uint32_t onb[2][2];
#pragma unroll
  for (int pb = 0; pb < 2; ++pb) {
    const int q = l32 + 32 * pb;
    const bool qlive = q < nlive;
    const int y = __shfl(y_own, q, 64);
    v16f H[2];
    {
      v4s ehi[2], elo[2];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        float e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = S.E[8 * ks + 4 * (lane >> 5) + j][q];
          e[j] = qlive ? v : 0.0f;
        }
        split4(e, ehi[ks], elo[ks]);
      }
#pragma unroll
      for (int hb = 0; hb < 2; ++hb) {
        H[hb] = mfma2(w1a[hb][0], w1a[hb][1], ehi[0], ehi[1], zero16());
        H[hb] = mfma2(w1a[hb][0], w1a[hb][1], elo[0], elo[1], H[hb]);
      }
#pragma unroll
      for (int hb = 0; hb < 2; ++hb) {
        uint32_t bits = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float pre = H[hb][r] + L.b1[drow(r, lane) + 32 * hb];
          bits |= (pre > 0.0f ? 1u : 0u) << r;
          H[hb][r] = fmaxf(pre, 0.0f);
        }
        onb[pb][hb] = bits;
      }
    }
    v16f Lg[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      Lg[cb] = zero16();
      const uint16_t* wrow = w2r + (l32 + 32 * cb) * kWtStride + 8 * (lane >> 5);
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        // A = W2 (i = class l32 + 32 cb, k = hidden 8 ks + 4 (l / 32) + j, ks = 2 s2, 2 s2 + 1);
        // rows >= C are zero
        const v8s a = *reinterpret_cast<const v8s*>(wrow + 16 * s2);
        v4s hi[2], lo[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int ks = 2 * s2 + u;
          float x[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) x[j] = H[ks >> 2][4 * (ks & 3) + j];
          split4(x, hi[u], lo[u]);
        }
        Lg[cb] = mfma2(a, hi[0], hi[1], Lg[cb]);
        Lg[cb] = mfma2(a, lo[0], lo[1], Lg[cb]);
      }
    }
    // softmax over the pixel's classes: this lane's 32, then the partner lane's
    float m = -INFINITY;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = drow(r, lane) + 32 * cb;
        const float v = c < C ? Lg[cb][r] + b2r[cb][r] : -INFINITY;
        Lg[cb][r] = v;
        m = fmaxf(m, v);
      }
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    float z = 0.0f, xy = 0.0f;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = drow(r, lane) + 32 * cb;
        xy = c == y ? Lg[cb][r] : xy;
        const float e = c < C ? __expf(Lg[cb][r] - m) : 0.0f;
        Lg[cb][r] = e;
        z += e;
      }
    z += __shfl_xor(z, 32, 64);
    xy += __shfl_xor(xy, 32, 64);
    const bool labelled = qlive && y >= 0 && y < C;   // outside [0, C): unlabelled, no semantic term
    if (labelled && lane < 32) ls += (m + __logf(z) - xy) * invp;
    const float sc = labelled ? w2 * invp / z : 0.0f;
    const float oh = labelled ? w2 * invp : 0.0f;
    // dlogits to LDS [class][pixel] (rows of absent classes stay zero)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = drow(r, lane) + 32 * cb;
        if (c < C) sg[c * kGst + q] = Lg[cb][r] * sc - (c == y ? oh : 0.0f);
      }
  }
  wave_fence();
  head_chunk_backward<false, true>(L, sg, &S.E[0][0], kEst, gcolor + ci.pixel_base * K + 4 * HW + ci.local0, HW,
                                   nlive, w1a, b1l, acc, onb);
  wave_fence();
  // loss partial sums: one atomic per wave and quantity (a chunk lies in one item)
  const float a = wave_sum(lr), bsum = wave_sum(ld), c = wave_sum(ls), v = wave_sum(nv);
  if (lane == 0) {
    const int slot = (int)(ci.chunk % n_slots);
    float* loss = loss_slots + slot;
    atomicAdd(&loss[(3 * ci.item + 0) * n_slots], a);
    if (v != 0.0f) {
      atomicAdd(&loss[(3 * ci.item + 1) * n_slots], bsum);
      atomicAdd(&count_slots[ci.item * n_slots + slot], v);
    }
    atomicAdd(&loss[(3 * ci.item + 2) * n_slots], c);
  }
}

__global__ __launch_bounds__(256, 1) void k_head_loss(const gs_item* __restrict__ items, int n_items, int K, int C,
                                                      const float* __restrict__ color, const float* __restrict__ trgb,
                                                      const float* __restrict__ tdepth,
                                                      const int32_t* __restrict__ tlabel,
                                                      const uint16_t* __restrict__ W1, const float* __restrict__ b1,
                                                      const uint16_t* __restrict__ W2, const float* __restrict__ b2,
                                                      float w0, float w2, bool rgb_grad, int n_slots,
                                                      float* __restrict__ loss_slots, float* __restrict__ count_slots,
                                                      float* __restrict__ gcolor, float* __restrict__ partial) {
  __shared__ HeadLds L;
  __shared__ __align__(16) uint16_t w2r[kHid * kWtStride];   // W2 [class][kperm(hidden)], rows >= C zero
  __shared__ ChunkStage SA[4];
  __shared__ ChunkStage SB[4];
  const int lane = threadIdx.x & 63;
  // wave-uniform: the chunk walk and the item table reads stay in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < kHid * kHid; i += 256) {
    const int c = i / kHid, h = i % kHid;
    w2r[c * kWtStride + kperm(h)] = c < C ? W2[c * kHid + h] : (uint16_t)0;
  }
  HeadAcc acc;
  v4s w1a[2][2];
  float b1l[2];
  head_setup(L, C, W1, b1, W2, acc, w1a, b1l);   // ends in a block barrier: w2r is complete
  float* sg = L.buf + wave * kHid * kGst;
  // b2 of this lane's classes drow(r) + 32 cb
  float b2r[2][16];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int c = drow(r, lane) + 32 * cb;
      b2r[cb][r] = c < C ? b2[c] : 0.0f;
    }
  ConstItems citems = (ConstItems)items;
  ChunkCursor cur;
  cur.item = 0;
  cur.first = 0;
  cur.end = ((int64_t)citems[0].W * citems[0].H + 63) / 64;
  const int64_t stride = (int64_t)gridDim.x * 4;
  // Every iteration issues the same loads whether or not a next chunk exists (past the end
  // the current chunk is loaded again and not used), so the number of loads in flight is
  // the same on every path and each buffer's wait covers exactly its own loads.
  ChunkInfo ca, cb;
  bool have = chunk_info(citems, n_items, (int64_t)blockIdx.x * 4 + wave, cur, ca);
  if (!have) {
    head_write_partial(L, acc, partial);
    return;
  }
  stage_chunk(SA[wave], ca, K, color, trgb, tdepth, tlabel);
  for (;;) {
    const bool hb = chunk_info(citems, n_items, ca.chunk + stride, cur, cb);
    if (!hb) cb = ca;
    stage_chunk(SB[wave], cb, K, color, trgb, tdepth, tlabel);
    head_loss_chunk(L, w2r, SA[wave], ca, sg, K, C, w0, w2, rgb_grad, n_slots, b2r, w1a, b1l, acc, loss_slots,
                    count_slots, gcolor);
    if (!hb) break;
    const bool ha = chunk_info(citems, n_items, cb.chunk + stride, cur, ca);
    if (!ha) ca = cb;
    stage_chunk(SA[wave], ca, K, color, trgb, tdepth, tlabel);
    head_loss_chunk(L, w2r, SB[wave], cb, sg, K, C, w0, w2, rgb_grad, n_slots, b2r, w1a, b1l, acc, loss_slots,
                    count_slots, gcolor);
    if (!ha) break;
  }
  // the last iteration's loads into the unused buffer are complete before the block's LDS
  // is reused below
  __builtin_amdgcn_s_waitcnt(0);
  head_write_partial(L, acc, partial);
}

// Sums the per-block partials into the head's weight gradients: block = 64 columns,
// four thread groups over interleaved partials, combined in LDS.
__global__ __launch_bounds__(256) void k_head_reduce(const float* __restrict__ partial, int n_blocks, int C,
                                                     float* __restrict__ gW1, float* __restrict__ gb1,
                                                     float* __restrict__ gW2, float* __restrict__ gb2) {
  __shared__ float s_sum[4][64];
  const int col = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + col;
  float s = 0.0f;
  if (i < kPart)
    for (int b = grp; b < n_blocks; b += 4) s += partial[(int64_t)b * kPart + i];
  s_sum[grp][col] = s;
  __syncthreads();
  if (grp != 0 || i >= kPart) return;
  s = (s_sum[0][col] + s_sum[1][col]) + (s_sum[2][col] + s_sum[3][col]);
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
  // at most one 64-pixel chunk per item is partial, so P / 64 + n_items bounds the chunk count;
  // the blocks walk the chunks grid-stride, so the grid is the resident count (one wave per
  // SIMD: the register file holds the weight-gradient accumulators without spilling)
  const int resident = resident_blocks(k_head_bwd, 256, kHeadBlocksMax);
  const int blocks = (int)std::min<int64_t>(std::min(kHeadBlocksMax, resident), ceil_div(ceil_div(P, 64) + n_items, 4));
  hipLaunchKernelGGL(k_head_bwd, dim3(blocks), dim3(256), 0, s, items, n_items, K, h.n_classes, color, glogits, h.W1,
                     h.b1, h.W2, gcolor, partial);
  hipLaunchKernelGGL(k_head_reduce, dim3((unsigned)ceil_div(kPart, 64)), dim3(256), 0, s, partial, blocks, h.n_classes,
                     gW1, gb1, gW2, gb2);
  return launch_status();
}

int launch_head_loss(const gs_item* items, int n_items, int64_t P, int K, const gs_head& h, const float* color,
                     const gs_targets& t, float w0, float w2, bool rgb_grad, int n_slots, float* loss_slots,
                     float* count_slots, float* gcolor, float* partial, float* gW1, float* gb1, float* gW2, float* gb2,
                     hipStream_t s) {
  if (P == 0) return GS_OK;
  const int resident = resident_blocks(k_head_loss, 256, kHeadBlocksMax);
  const int blocks = (int)std::min<int64_t>(std::min(kHeadBlocksMax, resident), ceil_div(ceil_div(P, 64) + n_items, 4));
  hipLaunchKernelGGL(k_head_loss, dim3(blocks), dim3(256), 0, s, items, n_items, K, h.n_classes, color, t.rgb, t.depth,
                     t.label, h.W1, h.b1, h.W2, h.b2, w0, w2, rgb_grad, n_slots, loss_slots, count_slots, gcolor,
                     partial);
  hipLaunchKernelGGL(k_head_reduce, dim3((unsigned)ceil_div(kPart, 64)), dim3(256), 0, s, partial, blocks, h.n_classes,
                     gW1, gb1, gW2, gb2);
  return launch_status();
}

}  // namespace gs
