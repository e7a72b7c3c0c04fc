// Tile compositing (paper eq. 7-9) and its reverse pass.
//
// One 256-thread workgroup per 16x16 screen tile, one pixel per thread. The tile's
// depth-ordered Gaussians are staged through LDS in batches; every lane reads the
// same record at the same time (LDS broadcast). This file holds the plain VALU
// variant, which accumulates the 4 + n_sem channels per pixel in registers.
#include "common.h"

namespace gs {
namespace {

template <int NS>
struct Shape {
  static constexpr int K = 4 + NS;                       // composited channels
  static constexpr int STRIDE = (12 + NS + 3) & ~3;      // LDS floats per Gaussian
  static constexpr int FWD_BATCH = (STRIDE * 4 * 256 <= 32768) ? 256 : ((STRIDE * 4 * 128 <= 32768) ? 128 : 64);
  static constexpr int NV = 6 + K;                       // reduced values per Gaussian in the backward
  static constexpr int NVP = (NV + 3) & ~3;
  static constexpr int BWD_BATCH = ((STRIDE + NVP) * 4 * 128 <= 32768) ? 128 : 64;
};

struct TileCtx {
  int item, view, tx, ty, u, v;
  bool inside;
  float px, py;
  int64_t pix;      // global pixel index
  int64_t HW;
  int64_t cbase;    // first float of the item's colour planes
  uint32_t start, end;
};

__device__ __forceinline__ TileCtx tile_ctx(const gs_item* items, int n_items, const uint32_t* ranges, int K, int tws) {
  TileCtx c;
  const int tile = blockIdx.x;
  c.item = item_of_tile(items, n_items, tile);
  const gs_item it = items[c.item];
  c.view = it.view;
  const int lt = tile - it.tile_base;
  c.tx = lt % it.tiles_x;
  c.ty = lt / it.tiles_x;
  c.u = (c.tx << tws) + (threadIdx.x & ((1 << tws) - 1));
  c.v = c.ty * (kTilePx >> tws) + (threadIdx.x >> tws);
  c.inside = c.u < it.W && c.v < it.H;
  c.px = c.u + 0.5f;
  c.py = c.v + 0.5f;
  c.HW = (int64_t)it.W * it.H;
  const int64_t local = (int64_t)c.v * it.W + c.u;
  c.pix = it.pixel_base + local;
  c.cbase = it.pixel_base * K + local;
  c.start = ranges[2 * (int64_t)tile];
  c.end = ranges[2 * (int64_t)tile + 1];
  return c;
}

// Stages Gaussian `g` of item `item` into sm[0..STRIDE): rec(8) rgb(3) depth(1) sem(NS).
template <int NS>
__device__ __forceinline__ void stage(float* sm, uint32_t g, int item, int64_t n, const float* __restrict__ rec,
                                      const float* __restrict__ depth, const float* __restrict__ rgb,
                                      const float* __restrict__ sem, const uint16_t* __restrict__ emb, int n_sem,
                                      int64_t foff) {
  const int64_t e = (int64_t)item * n + g;
  const float4* r = reinterpret_cast<const float4*>(rec + kRecFloats * e);
  float4* d = reinterpret_cast<float4*>(sm);
  d[0] = r[0];
  d[1] = r[1];
  d[2] = make_float4(rgb[3 * ((int64_t)g + foff)], rgb[3 * ((int64_t)g + foff) + 1], rgb[3 * ((int64_t)g + foff) + 2], depth[e]);
  const float* s = sem + (int64_t)n_sem * ((int64_t)g + foff);
  const uint16_t* es = emb + (int64_t)n_sem * ((int64_t)g + foff);
#pragma unroll
  for (int c = 0; c < NS; ++c)
    sm[12 + c] = c >= n_sem ? 0.0f : (emb ? __uint_as_float((uint32_t)es[c] << 16) : s[c]);
}

template <int NS>
__global__ __launch_bounds__(256) void k_render_fwd(gs_config cfg, const float* __restrict__ rgb, const float* __restrict__ sem,
                                                    const uint16_t* __restrict__ emb, int n_sem, const float* __restrict__ rec,
                                                    const float* __restrict__ depth, int64_t n,
                                                    const gs_item* __restrict__ items, int n_items,
                                                    const uint32_t* __restrict__ vals, const uint32_t* __restrict__ ranges,
                                                    float* __restrict__ color, float* __restrict__ Tout,
                                                    uint32_t* __restrict__ ncout) {
  using S = Shape<NS>;
  constexpr int K = S::K, STRIDE = S::STRIDE, BATCH = S::FWD_BATCH;
  __shared__ float4 smem[BATCH * STRIDE / 4];
  float* sm = reinterpret_cast<float*>(smem);
  const int Kr = 4 + n_sem;
  const TileCtx c = tile_ctx(items, n_items, ranges, Kr, tile_shift(cfg));
  const int64_t foff = feature_offset(cfg, c.view, n);
  float acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0f;
  float T = 1.0f;
  bool done = !c.inside;
  uint32_t last = 0;
  const float amin = cfg.alpha_min, amax = cfg.alpha_max, tmin = cfg.t_min;
  for (uint32_t b = c.start; b < c.end; b += BATCH) {
    if (__syncthreads_count(!done) == 0) break;
    const int cnt = (int)min((uint32_t)BATCH, c.end - b);
    for (int q = threadIdx.x; q < cnt; q += 256) stage<NS>(sm + q * STRIDE, vals[b + q], c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
    __syncthreads();
    if (!done) {
      for (int q = 0; q < cnt; ++q) {
        const float4* g4 = reinterpret_cast<const float4*>(sm + q * STRIDE);
        const float4 r0 = g4[0], r1 = g4[1];
        float dx, dy;
        const float pw = footprint_power(c.px, c.py, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, dx, dy);
        const float araw = r1.w * fast_exp(pw);
        if (araw < amin) continue;
        const float a = fminf(amax, araw);
        const float Tn = T * (1.0f - a);
        if (Tn < tmin) {
          done = true;
          break;
        }
        const float w = a * T;
#pragma unroll
        for (int k4 = 0; k4 < (K + 3) / 4; ++k4) {
          const float4 f = g4[2 + k4];
          if (4 * k4 + 0 < K) acc[4 * k4 + 0] = __builtin_fmaf(w, f.x, acc[4 * k4 + 0]);
          if (4 * k4 + 1 < K) acc[4 * k4 + 1] = __builtin_fmaf(w, f.y, acc[4 * k4 + 1]);
          if (4 * k4 + 2 < K) acc[4 * k4 + 2] = __builtin_fmaf(w, f.z, acc[4 * k4 + 2]);
          if (4 * k4 + 3 < K) acc[4 * k4 + 3] = __builtin_fmaf(w, f.w, acc[4 * k4 + 3]);
        }
        T = Tn;
        last = b - c.start + q + 1;
      }
    }
  }
  if (!c.inside) return;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (k < Kr) color[c.cbase + k * c.HW] = acc[k];
  Tout[c.pix] = T;
  ncout[c.pix] = last;
}

template <int NS>
__global__ __launch_bounds__(256) void k_render_bwd(gs_config cfg, const float* __restrict__ rgb, const float* __restrict__ sem,
                                                    const uint16_t* __restrict__ emb, int n_sem, const float* __restrict__ rec,
                                                    const float* __restrict__ depth, int64_t n,
                                                    const gs_item* __restrict__ items, int n_items,
                                                    const uint32_t* __restrict__ vals, const uint32_t* __restrict__ ranges,
                                                    const float* __restrict__ Tfin, const uint32_t* __restrict__ ncin,
                                                    const float* __restrict__ gcolor, float* __restrict__ g2d,
                                                    float* __restrict__ grgb, float* __restrict__ gsem) {
  using S = Shape<NS>;
  constexpr int K = S::K, STRIDE = S::STRIDE, BATCH = S::BWD_BATCH, NV = S::NV, NVP = S::NVP;
  __shared__ float4 smem[BATCH * STRIDE / 4];
  __shared__ float red[BATCH * NVP];
  __shared__ uint32_t s_lmax;
  float* sm = reinterpret_cast<float*>(smem);
  const int Kr = 4 + n_sem;
  const TileCtx c = tile_ctx(items, n_items, ranges, Kr, tile_shift(cfg));
  const int64_t foff = feature_offset(cfg, c.view, n);
  const int lane = threadIdx.x & 63;
  float gp[K];
#pragma unroll
  for (int k = 0; k < K; ++k) gp[k] = (c.inside && k < Kr) ? gcolor[c.cbase + k * c.HW] : 0.0f;
  float T = c.inside ? Tfin[c.pix] : 1.0f;
  // n_contrib comes from the matching forward; clamp so that a mismatched call stays in range
  const uint32_t len = c.end - c.start;
  const uint32_t last = c.inside ? min(ncin[c.pix], len) : 0u;
  if (threadIdx.x == 0) s_lmax = 0;
  __syncthreads();
  atomicMax(&s_lmax, last);
  __syncthreads();
  const uint32_t lmax = s_lmax;
  float suffix = 0.0f;   // sum over later Gaussians of (g . f) alpha T
  const float amin = cfg.alpha_min, amax = cfg.alpha_max;
  for (int hi = (int)lmax; hi > 0; hi -= BATCH) {
    const int lo = max(0, hi - BATCH);
    const int cnt = hi - lo;
    __syncthreads();
    for (int q = threadIdx.x; q < cnt; q += 256)
      stage<NS>(sm + q * STRIDE, vals[c.start + lo + q], c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
    for (int q = threadIdx.x; q < cnt * NVP; q += 256) red[q] = 0.0f;
    __syncthreads();
    for (int q = cnt - 1; q >= 0; --q) {
      const uint32_t pos = (uint32_t)(lo + q);
      float out[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = 0.0f;
      bool contrib = false;
      if (pos < last) {
        const float4* g4 = reinterpret_cast<const float4*>(sm + q * STRIDE);
        const float4 r0 = g4[0], r1 = g4[1];
        float dx, dy;
        const float pw = footprint_power(c.px, c.py, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, dx, dy);
        const float G = fast_exp(pw);
        const float araw = r1.w * G;
        if (araw >= amin) {
          contrib = true;
          const float a = fminf(amax, araw);
          const float om = 1.0f - a;
          T = T / om;                     // transmittance in front of this Gaussian
          const float w = a * T;
          float gf = 0.0f;
#pragma unroll
          for (int k4 = 0; k4 < (K + 3) / 4; ++k4) {
            const float4 f = g4[2 + k4];
            if (4 * k4 + 0 < K) { gf = __builtin_fmaf(gp[4 * k4 + 0], f.x, gf); out[6 + 4 * k4 + 0] = w * gp[4 * k4 + 0]; }
            if (4 * k4 + 1 < K) { gf = __builtin_fmaf(gp[4 * k4 + 1], f.y, gf); out[6 + 4 * k4 + 1] = w * gp[4 * k4 + 1]; }
            if (4 * k4 + 2 < K) { gf = __builtin_fmaf(gp[4 * k4 + 2], f.z, gf); out[6 + 4 * k4 + 2] = w * gp[4 * k4 + 2]; }
            if (4 * k4 + 3 < K) { gf = __builtin_fmaf(gp[4 * k4 + 3], f.w, gf); out[6 + 4 * k4 + 3] = w * gp[4 * k4 + 3]; }
          }
          const float dalpha = T * gf - suffix / om;
          suffix = __builtin_fmaf(gf, w, suffix);
          if (araw < amax) {
            const float dpow = dalpha * araw;
            out[0] = dpow * (r1.x * dx + r1.y * dy);     // d/d mean2d.x
            out[1] = dpow * (r1.z * dy + r1.y * dx);     // d/d mean2d.y
            out[2] = -0.5f * dpow * dx * dx;             // d/dA
            out[3] = -dpow * dx * dy;                    // d/dB
            out[4] = -0.5f * dpow * dy * dy;             // d/dC
            out[5] = dalpha * G;                         // d/d opacity
          }
        }
      }
      if (__ballot(contrib) != 0ull) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const float s = wave_sum(out[v]);
          if (lane == 0 && s != 0.0f) atomicAdd(&red[q * NVP + v], s);
        }
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < cnt * NV; idx += 256) {
      const int q = idx / NV, v = idx - q * NV;
      const float s = red[q * NVP + v];
      if (s == 0.0f) continue;
      const uint32_t g = vals[c.start + lo + q];
      const int64_t e = (int64_t)c.item * n + g;
      if (v < 6) atomicAdd(&g2d[8 * e + v], s);
      else if (v < 9) atomicAdd(&grgb[3 * ((int64_t)g + foff) + (v - 6)], s);
      else if (v == 9) atomicAdd(&g2d[8 * e + 6], s);
      else if (v - 10 < n_sem) atomicAdd(&gsem[(int64_t)n_sem * ((int64_t)g + foff) + (v - 10)], s);
    }
  }
}

template <int NS>
int launch_fwd_t(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items, int n_items,
                 int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& out, hipStream_t s) {
  hipLaunchKernelGGL(k_render_fwd<NS>, dim3(n_tiles), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb, cfg.n_sem, p.rec, p.depth,
                     g.n, items, n_items, vals, ranges, out.color, out.T, out.n_contrib);
  return launch_status();
}

template <int NS>
int launch_bwd_t(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items, int n_items,
                 int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& fwd,
                 const gs_images& gin, float* g2d, const gs_grads& gr, hipStream_t s) {
  hipLaunchKernelGGL(k_render_bwd<NS>, dim3(n_tiles), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb, cfg.n_sem, p.rec, p.depth,
                     g.n, items, n_items, vals, ranges, fwd.T, fwd.n_contrib, gin.color, g2d, gr.rgb, gr.sem);
  return launch_status();
}

}  // namespace

int launch_render_fwd_valu(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items,
                      int n_items, int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& out,
                      hipStream_t s) {
  if (n_tiles == 0) return GS_OK;
  const int ns = cfg.n_sem;
  if (ns <= 8) return launch_fwd_t<8>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 16) return launch_fwd_t<16>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 20) return launch_fwd_t<20>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 32) return launch_fwd_t<32>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 52) return launch_fwd_t<52>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 64) return launch_fwd_t<64>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  return GS_ERR_UNSUPPORTED;
}

int launch_render_bwd_valu(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items,
                      int n_items, int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& fwd,
                      const gs_images& gin, float* g2d, const gs_grads& gr, hipStream_t s) {
  if (n_tiles == 0) return GS_OK;
  const int ns = cfg.n_sem;
  if (ns <= 8) return launch_bwd_t<8>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (ns <= 16) return launch_bwd_t<16>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (ns <= 20) return launch_bwd_t<20>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (ns <= 32) return launch_bwd_t<32>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (ns <= 52) return launch_bwd_t<52>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  if (ns <= 64) return launch_bwd_t<64>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, s);
  return GS_ERR_UNSUPPORTED;
}

}  // namespace gs
