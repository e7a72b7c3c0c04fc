// Internal helpers of the gfx950 rasterizer library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs.h"

namespace gs {

constexpr int kTile = 16;          // default screen tile edge (pixels)
constexpr int kTilePx = 256;       // pixels per tile: every shape is tile_w x (256 / tile_w)

// Tile width as a shift: tiles are 8x32, 16x16, 32x8 or 64x4 pixels (one pixel per
// thread of a 256-thread block; tile-local pixel t sits at (t % tile_w, t / tile_w)).
__host__ __device__ inline int tile_shift(const gs_config& cfg) {
  return cfg.tile_w == 8 ? 3 : cfg.tile_w == 32 ? 5 : cfg.tile_w == 64 ? 6 : 4;
}
constexpr int kRecFloats = 8;      // per (item, Gaussian) render record

// Records the last HIP error for gs_last_hip_error(); returns GS_ERR_HIP if e != success.
int hip_status(hipError_t e);
int launch_status();  // hipGetLastError() folded into a gs_status

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Blocks of a persistent (grid-stride or work-queue) launch that fill the calling thread's
// current device: resident blocks per CU times CUs. Computed at every call (nothing is
// cached, so a second device or a changed current device is sized correctly); `fallback`
// (0: report failure) if the runtime cannot tell.
template <class F>
int resident_blocks(F kernel, int threads, int fallback) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess)
    return fallback;
  return (cus > 0 ? cus : 1) * (per > 0 ? per : 1);
}
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Item owning a global tile index (items are ordered by tile_base).
__device__ __forceinline__ int item_of_tile(const gs_item* items, int n_items, int tile) {
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Item owning a global pixel index (items are ordered by pixel_base).
__device__ __forceinline__ int item_of_pixel(const gs_item* items, int n_items, int64_t pix) {
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (items[mid].pixel_base <= pix) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Exponent of the 2D footprint, eq. 3 in conic form: -(d^T Q d)/2, d = p - mean2d.
// mean2d is carried as hi + lo so that d keeps full single precision far from the
// image origin. A positive-definite conic gives a value <= 0; rounding can make it
// slightly positive, which is clamped. The forward and the backward call this same
// sequence (contraction is disabled for the library) so that both see the same alpha.
__device__ __forceinline__ float footprint_power(float px, float py, float mhx, float mhy, float mlx, float mly,
                                                 float A, float B, float C, float& dx, float& dy) {
  dx = (px - mhx) - mlx;
  dy = (py - mhy) - mly;
  float q = __builtin_fmaf(A * dx, dx, (C * dy) * dy);
  float p = __builtin_fmaf(-0.5f, q, -((B * dx) * dy));
  return fminf(p, 0.0f);
}

struct Rect {
  int x0, y0, x1, y1;
};

// Tiles of an item met by the footprint square [mean2d - r, mean2d + r]^2 (half-open
// tile ranges); m = (mean2d hi, mean2d lo) as the render record stores it. Binning and
// the reverse pass both use this one definition.
__device__ __forceinline__ Rect tile_rect(const gs_config& cfg, int tiles_x, int tiles_y, float4 m, int r) {
  const double mx = (double)m.x + (double)m.z, my = (double)m.y + (double)m.w;
  Rect R;
  if (cfg.full_rect) {
    R.x0 = 0; R.y0 = 0; R.x1 = tiles_x; R.y1 = tiles_y;
    return R;
  }
  // tile sides are powers of two, so the products by their reciprocals are the quotients exactly
  const double iw = 1.0 / 256.0 * (double)(256 / cfg.tile_w), ih = 1.0 / 256.0 * (double)(256 / cfg.tile_h);
  R.x0 = min(tiles_x, max(0, (int)floor((mx - r) * iw)));
  R.y0 = min(tiles_y, max(0, (int)floor((my - r) * ih)));
  R.x1 = min(tiles_x, max(0, (int)floor((mx + r) * iw) + 1));
  R.y1 = min(tiles_y, max(0, (int)floor((my + r) * ih) + 1));
  return R;
}

// DPP lane moves within a row of 16 lanes (every source lane exists, so bound_ctrl only
// lets the compiler fold the move into the consuming add as one v_add_f32_dpp).
__device__ __forceinline__ float dpp_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_ror8(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_half_mirror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_mirror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, true));
}
// Sum over the 16 lanes of each DPP row; every lane of the row receives the sum.
__device__ __forceinline__ float row_sum16(float v) {
  v += dpp_xor1(v);
  v += dpp_xor2(v);
  v += dpp_half_mirror(v);
  v += dpp_mirror(v);
  return v;
}

// Workgroup barrier that orders LDS only: global stores and atomics issued before it stay
// in flight (nothing in the block reads them back), so their latency overlaps later work.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One tile of one item, as a render block sees it (tile width 1 << tws, height 256 >> tws).
struct Ctx {
  int item, view, tx, ty, tiles_x, tiles_y, tws;
  int W, H;
  int64_t HW, pixel_base;
  uint32_t start, end;
};

// Tiles are launched coarse pyramid levels first: their lists are the longest, and
// starting them early lets the many short fine-level tiles fill in around them.
__device__ __forceinline__ Ctx make_ctx_of(const gs_item* items, int n_items, const uint32_t* ranges, int tile,
                                           int tws) {
  Ctx c;
  c.tws = tws;
  c.item = item_of_tile(items, n_items, tile);
  const gs_item it = items[c.item];
  c.view = it.view;
  const int lt = tile - it.tile_base;
  c.tx = lt % it.tiles_x;
  c.ty = lt / it.tiles_x;
  c.tiles_x = it.tiles_x;
  c.tiles_y = it.tiles_y;
  c.W = it.W;
  c.H = it.H;
  c.HW = (int64_t)it.W * it.H;
  c.pixel_base = it.pixel_base;
  c.start = ranges[2 * (int64_t)tile];
  c.end = ranges[2 * (int64_t)tile + 1];
  return c;
}

__device__ __forceinline__ Ctx make_ctx(const gs_item* items, int n_items, const uint32_t* ranges, int order, int tws) {
  return make_ctx_of(items, n_items, ranges, order ? (int)blockIdx.x : (int)gridDim.x - 1 - (int)blockIdx.x, tws);
}

// First feature entry of a tile's Gaussians: with per-view features (cfg.view_features) the
// rgb / sem arrays (and their gradients) hold one [n][channels] block per view.
__device__ __forceinline__ int64_t feature_offset(const gs_config& cfg, int view, int64_t n) {
  return cfg.view_features ? (int64_t)view * n : 0;
}

// Tile-local pixel index t (0..255, row-major in the tile) -> image coordinates.
__device__ __forceinline__ void tile_pixel(const Ctx& c, int t, int& u, int& v) {
  u = (c.tx << c.tws) + (t & ((1 << c.tws) - 1));
  v = c.ty * (kTilePx >> c.tws) + (t >> c.tws);
}
// The image coordinates of the tile's middle pixel (tile_w / 2, tile_h / 2).
__device__ __forceinline__ int tile_mid_x(const Ctx& c) { return (c.tx << c.tws) + (1 << (c.tws - 1)); }
__device__ __forceinline__ int tile_mid_y(const Ctx& c) { return c.ty * (kTilePx >> c.tws) + (128 >> c.tws); }

__device__ __forceinline__ float fast_exp(float x) { return __expf(x); }

// Wave64 helpers.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace gs
