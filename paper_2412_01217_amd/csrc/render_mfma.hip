// Tile compositing (eq. 7-9) and its reverse pass with the channel work on matrix cores.
//
// Per pixel, compositing is a scalar recurrence over the tile's depth-ordered list
// (alpha, transmittance, stop test), followed by a K-channel accumulation
//   out[p][c] = sum_i w[p][i] f[i][c],        w[p][i] = alpha_i(p) T_i(p),
// which for a 16x16 tile and a batch of 32 Gaussians is a dense (pixels x Gaussians)
// by (Gaussians x channels) product. Likewise the backward's feature gradient
//   dF[i][c] = sum_p w[p][i] g[p][c]
// is a (Gaussians x pixels) by (pixels x channels) product. Each wave runs the scalar
// recurrence for its 64 pixels (one per lane), writes w to LDS, and the contraction
// runs as v_mfma_f32_32x32x2f32 (single precision in and out, so results match the
// per-lane FMA chain to rounding). The geometric gradients (mean2d, conic, opacity)
// are reduced over each 16-pixel row with DPP and summed over rows in LDS.
//
// MFMA 32x32x2 f32 operand layout (lane l, 0..63):
//   A[i][k]: i = l % 32, k = l / 32      B[k][j]: k = l / 32, j = l % 32
//   D[i][j] in 16 registers r: j = l % 32, i = 8 (r / 4) + 4 (l / 32) + r % 4
#include "common.h"

namespace gs {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kBatch = 32;          // Gaussians per LDS batch
constexpr int kWst = kBatch + 1;    // LDS row stride of the weight tile (bank-conflict padding)
constexpr int kPairs = 32;          // pixel pairs per wave (64 pixels, two per MFMA k-step)

template <int NS>
struct MShape {
  static constexpr int K = 4 + NS;
  static constexpr int KB = (K + 31) / 32;   // 32-channel blocks
  static constexpr int KP = KB * 32;
  static constexpr int FST = KP + 4;         // LDS row stride of the feature batch
};

__device__ __forceinline__ int mfma_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// Batch staging, double-buffered through registers: thread t stages Gaussian q = t / 8
// of the batch, channels [(t % 8) * CPT, +CPT) of its features and, for t % 8 < 2,
// half of its 8-float record. fetch() issues the global loads; commit() writes LDS.
template <int NS>
struct Stage {
  static constexpr int CPT = MShape<NS>::KP / 8;
  float4 r;
  float f[CPT];

  __device__ __forceinline__ void fetch(const uint32_t* __restrict__ vals, uint32_t b, int cnt, int item, int64_t n,
                                        const float* __restrict__ rec, const float* __restrict__ depth,
                                        const float* __restrict__ rgb, const float* __restrict__ sem,
                                        const uint16_t* __restrict__ emb, int n_sem, int64_t foff) {
    const int q = threadIdx.x >> 3, part = threadIdx.x & 7;
    const bool live = q < cnt;
    const uint32_t g = live ? vals[b + q] : 0u;
    const int64_t e = (int64_t)item * n + g;
    r = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live && part < 2) r = reinterpret_cast<const float4*>(rec + kRecFloats * e)[part];
    const int Kr = 4 + n_sem;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int k = part * CPT + j;
      float v = 0.0f;
      if (live && k < Kr) {
        if (k < 3) v = rgb[3 * ((int64_t)g + foff) + k];
        else if (k == 3) v = depth[e];
        else if (emb) v = __uint_as_float((uint32_t)emb[(int64_t)n_sem * ((int64_t)g + foff) + (k - 4)] << 16);
        else v = sem[(int64_t)n_sem * ((int64_t)g + foff) + (k - 4)];
      }
      f[j] = v;
    }
  }

  __device__ __forceinline__ void commit(float4* s_rec, float* s_feat) const {
    const int q = threadIdx.x >> 3, part = threadIdx.x & 7;
    if (part < 2) s_rec[2 * q + part] = r;
#pragma unroll
    for (int j = 0; j < CPT; ++j) s_feat[q * MShape<NS>::FST + part * CPT + j] = f[j];
  }
};

template <int NS>
__global__ __launch_bounds__(256) void k_render_fwd_mfma(gs_config cfg, const float* __restrict__ rgb,
                                                         const float* __restrict__ sem,
                                                         const uint16_t* __restrict__ emb, int n_sem,
                                                         const float* __restrict__ rec, const float* __restrict__ depth,
                                                         int64_t n, const gs_item* __restrict__ items, int n_items,
                                                         const uint32_t* __restrict__ vals,
                                                         const uint32_t* __restrict__ ranges, float* __restrict__ color,
                                                         float* __restrict__ Tout, uint32_t* __restrict__ ncout) {
  using S = MShape<NS>;
  constexpr int KB = S::KB, FST = S::FST;
  __shared__ float4 s_rec[2 * kBatch];
  __shared__ float s_feat[kBatch * FST];
  __shared__ float s_w[4][64 * kWst];
  const Ctx c = make_ctx(items, n_items, ranges, cfg.tile_order, tile_shift(cfg));
  const int64_t foff = feature_offset(cfg, c.view, n);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  int u, v;
  tile_pixel(c, tid, u, v);
  const bool inside = u < c.W && v < c.H;
  const float px = u + 0.5f, py = v + 0.5f;
  v16f acc[KB][2];
#pragma unroll
  for (int cb = 0; cb < KB; ++cb)
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[cb][pb][r] = 0.0f;
  float T = 1.0f;
  bool done = !inside;
  uint32_t last = 0;
  const float amin = cfg.alpha_min, amax = cfg.alpha_max, tmin = cfg.t_min;
  float* W = s_w[wave];
  Stage<NS> st;
  if (c.start < c.end) st.fetch(vals, c.start, (int)min((uint32_t)kBatch, c.end - c.start), c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
  for (uint32_t b = c.start; b < c.end; b += kBatch) {
    // every wave is past the previous batch's LDS reads; stop once every pixel has
    if (__syncthreads_count(!done) == 0) break;
    st.commit(s_rec, s_feat);
    __syncthreads();
    const int cnt = (int)min((uint32_t)kBatch, c.end - b);
    if (b + kBatch < c.end)
      st.fetch(vals, b + kBatch, (int)min((uint32_t)kBatch, c.end - b - kBatch), c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
    // front-to-back recurrence, branch-free: the alpha of successive Gaussians is
    // independent, only T carries from one to the next
    uint32_t nz = 0;  // bit q: some lane of this wave blends Gaussian q
    const uint32_t base = b - c.start;
#pragma unroll 8
    for (int q = 0; q < kBatch; ++q) {
      const float4 r0 = s_rec[2 * q], r1 = s_rec[2 * q + 1];
      float dx, dy;
      const float pw = footprint_power(px, py, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, dx, dy);
      const float araw = r1.w * fast_exp(pw);
      const bool ok = (q < cnt) & !done & (araw >= amin);
      const float a = fminf(amax, araw);
      const float Tn = T * (1.0f - a);
      const bool stop = ok & (Tn < tmin);
      const bool take = ok & !stop;
      W[lane * kWst + q] = take ? a * T : 0.0f;
      T = take ? Tn : T;
      done = done | stop;
      last = take ? base + q + 1 : last;
      nz |= (__ballot(take) != 0ull ? 1u : 0u) << q;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // out^T[c][p] += sum_i F^T[c][i] W^T[i][p]: A = F^T (c = l%32, i = 2s + l/32), B = W^T (i = 2s + l/32, p = l%32)
    for (int s = 0; s < kBatch / 2; ++s) {
      if (((nz >> (2 * s)) & 3u) == 0u) continue;
      const int qi = 2 * s + (lane >> 5);
      float a[KB];
#pragma unroll
      for (int cb = 0; cb < KB; ++cb) a[cb] = s_feat[qi * FST + (lane & 31) + 32 * cb];
#pragma unroll
      for (int pb = 0; pb < 2; ++pb) {
        const float bw = W[((lane & 31) + 32 * pb) * kWst + qi];
#pragma unroll
        for (int cb = 0; cb < KB; ++cb) acc[cb][pb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[cb], bw, acc[cb][pb], 0, 0, 0);
      }
    }
  }
  // D[c][p]: lane holds pixel p = l%32 + 32 pb of this wave, channels mfma_row(r, l) + 32 cb
  const int Kr = 4 + n_sem;
#pragma unroll
  for (int pb = 0; pb < 2; ++pb) {
    const int t = wave * 64 + (lane & 31) + 32 * pb;
    int pu, pv;
    tile_pixel(c, t, pu, pv);
    if (pu >= c.W || pv >= c.H) continue;
    const int64_t pbase = c.pixel_base * Kr + (int64_t)pv * c.W + pu;
#pragma unroll
    for (int cb = 0; cb < KB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ch = mfma_row(r, lane) + 32 * cb;
        if (ch < Kr) color[pbase + ch * c.HW] = acc[cb][pb][r];
      }
  }
  if (!inside) return;
  const int64_t pix = c.pixel_base + (int64_t)v * c.W + u;
  Tout[pix] = T;
  ncout[pix] = last;
}

template <int NS>
__global__ __launch_bounds__(256) void k_render_bwd_mfma(gs_config cfg, const float* __restrict__ rgb,
                                                         const float* __restrict__ sem,
                                                         const uint16_t* __restrict__ emb, int n_sem,
                                                         const float* __restrict__ rec, const float* __restrict__ depth,
                                                         int64_t n, const gs_item* __restrict__ items, int n_items,
                                                         const uint32_t* __restrict__ vals,
                                                         const uint32_t* __restrict__ ranges,
                                                         const float* __restrict__ Tfin, const uint32_t* __restrict__ ncin,
                                                         const float* __restrict__ gcolor, float* __restrict__ g2d,
                                                         float* __restrict__ grgb, float* __restrict__ gsem) {
  using S = MShape<NS>;
  constexpr int K = S::K, KB = S::KB, KP = S::KP, FST = S::FST;
  __shared__ float4 s_rec[2 * kBatch];
  __shared__ float s_feat[kBatch * FST];
  __shared__ float s_w[4][64 * kWst];
  __shared__ float s_df[kBatch * KP];
  __shared__ float s_geo[kBatch * 6 * 16];
  __shared__ uint32_t s_lmax;
  const Ctx c = make_ctx(items, n_items, ranges, cfg.tile_order, tile_shift(cfg));
  const int64_t foff = feature_offset(cfg, c.view, n);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int Kr = 4 + n_sem;
  int u, v;
  tile_pixel(c, tid, u, v);
  const bool inside = u < c.W && v < c.H;
  const float px = u + 0.5f, py = v + 0.5f;
  const int64_t cb0 = c.pixel_base * Kr + (int64_t)v * c.W + u;
  // own pixel's upstream gradient, for g . f
  float gp[K];
#pragma unroll
  for (int k = 0; k < K; ++k) gp[k] = (inside && k < Kr) ? gcolor[cb0 + k * c.HW] : 0.0f;
  // the wave's 64 x KP upstream gradient in MFMA B layout: pixel 2s + l/32, channel l%32 + 32 cb
  float gB[kPairs][KB];
#pragma unroll
  for (int s = 0; s < kPairs; ++s) {
    const int t = wave * 64 + 2 * s + (lane >> 5);
    int pu, pv;
    tile_pixel(c, t, pu, pv);
    const bool in = pu < c.W && pv < c.H;
    const int64_t base = c.pixel_base * Kr + (int64_t)pv * c.W + pu;
#pragma unroll
    for (int cb = 0; cb < KB; ++cb) {
      const int ch = (lane & 31) + 32 * cb;
      gB[s][cb] = (in && ch < Kr) ? gcolor[base + ch * c.HW] : 0.0f;
    }
  }
  float T = inside ? Tfin[c.pixel_base + (int64_t)v * c.W + u] : 1.0f;
  // n_contrib comes from the matching forward; clamp so that a mismatched call stays in range
  const uint32_t len = c.end - c.start;
  const uint32_t last = inside ? min(ncin[c.pixel_base + (int64_t)v * c.W + u], len) : 0u;
  if (tid == 0) s_lmax = 0;
  __syncthreads();
  atomicMax(&s_lmax, last);
  __syncthreads();
  const uint32_t lmax = s_lmax;
  float suffix = 0.0f;   // sum over later Gaussians of (g . f) alpha T
  const float amin = cfg.alpha_min, amax = cfg.alpha_max;
  float* W = s_w[wave];
  Stage<NS> st;
  if (lmax > 0) {
    const int lo0 = max(0, (int)lmax - kBatch);
    st.fetch(vals, c.start + lo0, (int)lmax - lo0, c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
  }
  for (int hi = (int)lmax; hi > 0; hi -= kBatch) {
    const int lo = max(0, hi - kBatch);
    const int cnt = hi - lo;
    __syncthreads();
    st.commit(s_rec, s_feat);
    for (int i = tid; i < kBatch * KP; i += 256) s_df[i] = 0.0f;
    for (int i = tid; i < kBatch * 6 * 16; i += 256) s_geo[i] = 0.0f;
    __syncthreads();
    if (lo > 0) {
      const int lo2 = max(0, lo - kBatch);
      st.fetch(vals, c.start + lo2, lo - lo2, c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
    }
    bool wave_any = false;
#pragma unroll 2
    for (int q = kBatch - 1; q >= 0; --q) {
      const float4 r0 = s_rec[2 * q], r1 = s_rec[2 * q + 1];
      float dx, dy;
      const float pw = footprint_power(px, py, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, dx, dy);
      const float G = fast_exp(pw);
      const float araw = r1.w * G;
      const bool act = (q < cnt) & ((uint32_t)(lo + q) < last) & (araw >= amin);
      const float a = fminf(amax, araw);
      const float rom = __builtin_amdgcn_rcpf(1.0f - a);
      const float Tq = act ? T * rom : T;   // transmittance in front of this Gaussian
      const float w = act ? a * Tq : 0.0f;
      const float* f = s_feat + q * FST;
      float gf = 0.0f;
#pragma unroll
      for (int k = 0; k < K; ++k) gf = __builtin_fmaf(gp[k], f[k], gf);
      const float dalpha = Tq * gf - suffix * rom;
      suffix = act ? __builtin_fmaf(gf, w, suffix) : suffix;
      T = Tq;
      const float dpow = (act & (araw < amax)) ? dalpha * araw : 0.0f;
      const float dop = (act & (araw < amax)) ? dalpha * G : 0.0f;
      W[lane * kWst + q] = w;
      if (__ballot(act) != 0ull) {
        wave_any = true;
        const float s0 = row_sum16(dpow * (r1.x * dx + r1.y * dy));   // d/d mean2d.x
        const float s1 = row_sum16(dpow * (r1.z * dy + r1.y * dx));   // d/d mean2d.y
        const float s2 = row_sum16(-0.5f * dpow * dx * dx);           // d/dA
        const float s3 = row_sum16(-dpow * dx * dy);                  // d/dB
        const float s4 = row_sum16(-0.5f * dpow * dy * dy);           // d/dC
        const float s5 = row_sum16(dop);                              // d/d opacity
        if ((lane & 15) == 0) {
          float* dst = s_geo + q * 96 + wave * 4 + (lane >> 4);
          dst[0] = s0; dst[16] = s1; dst[32] = s2; dst[48] = s3; dst[64] = s4; dst[80] = s5;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (wave_any) {
      // dF[i][c] = sum_p W^T[i][p] G[p][c]: A = W^T (i = l%32, p = 2s + l/32), B = G (p = 2s + l/32, c = l%32)
      v16f d[KB];
#pragma unroll
      for (int cb = 0; cb < KB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) d[cb][r] = 0.0f;
#pragma unroll
      for (int s = 0; s < kPairs; ++s) {
        const float aw = W[(2 * s + (lane >> 5)) * kWst + (lane & 31)];
#pragma unroll
        for (int cb = 0; cb < KB; ++cb) d[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(aw, gB[s][cb], d[cb], 0, 0, 0);
      }
#pragma unroll
      for (int cb = 0; cb < KB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float val = d[cb][r];
          if (val != 0.0f) atomicAdd(&s_df[mfma_row(r, lane) * KP + (lane & 31) + 32 * cb], val);
        }
    }
    __syncthreads();
    for (int idx = tid; idx < cnt * KP; idx += 256) {
      const int q = idx / KP, k = idx - q * KP;
      const float val = s_df[idx];
      if (val == 0.0f || k >= Kr) continue;
      const uint32_t g = vals[c.start + lo + q];
      if (k < 3) atomicAdd(&grgb[3 * ((int64_t)g + foff) + k], val);
      else if (k == 3) atomicAdd(&g2d[8 * ((int64_t)c.item * n + g) + 6], val);
      else atomicAdd(&gsem[(int64_t)n_sem * ((int64_t)g + foff) + (k - 4)], val);
    }
    for (int idx = tid; idx < cnt * 6; idx += 256) {
      const int q = idx / 6, comp = idx - q * 6;
      const float* src = s_geo + q * 96 + comp * 16;
      float sum = 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) sum += src[r];
      if (sum != 0.0f) {
        const uint32_t g = vals[c.start + lo + q];
        atomicAdd(&g2d[8 * ((int64_t)c.item * n + g) + comp], sum);
      }
    }
  }
}

template <int NS>
int launch_fwd_m(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items, int n_items,
                 int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& out, hipStream_t s) {
  hipLaunchKernelGGL(k_render_fwd_mfma<NS>, dim3(n_tiles), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb, cfg.n_sem, p.rec,
                     p.depth, g.n, items, n_items, vals, ranges, out.color, out.T, out.n_contrib);
  return launch_status();
}

template <int NS>
int launch_bwd_m(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items, int n_items,
                 int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& fwd,
                 const gs_images& gin, float* g2d, const gs_grads& gr, hipStream_t s) {
  hipLaunchKernelGGL(k_render_bwd_mfma<NS>, dim3(n_tiles), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb, cfg.n_sem, p.rec,
                     p.depth, g.n, items, n_items, vals, ranges, fwd.T, fwd.n_contrib, gin.color, g2d, gr.rgb, gr.sem);
  return launch_status();
}

}  // namespace

int launch_render_fwd_mfma(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items,
                           int n_items, int n_tiles, const uint32_t* vals, const uint32_t* ranges,
                           const gs_images& out, hipStream_t s) {
  const int ns = cfg.n_sem;
  if (ns <= 8) return launch_fwd_m<8>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 20) return launch_fwd_m<20>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 28) return launch_fwd_m<28>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 52) return launch_fwd_m<52>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 60) return launch_fwd_m<60>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  return GS_ERR_UNSUPPORTED;
}

int launch_render_bwd_mfma(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items,
                           int n_items, int n_tiles, const uint32_t* vals, const uint32_t* ranges,
                           const gs_images& fwd, const gs_images& gin, float* g2d, const gs_grads& gr, hipStream_t s) {
  const int ns = cfg.n_sem;
  if (ns <= 8) return launch_bwd_m<8>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (ns <= 20) return launch_bwd_m<20>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (ns <= 28) return launch_bwd_m<28>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (ns <= 52) return launch_bwd_m<52>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (ns <= 60) return launch_bwd_m<60>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  return GS_ERR_UNSUPPORTED;
}

}  // namespace gs
