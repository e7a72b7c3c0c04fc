// Tile compositing (eq. 7-9) and its reverse pass, with every dense contraction on the
// bfloat16 matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16, 2.5 PFLOP/s) and single
// precision kept by splitting each operand x = hi + lo, hi = bf16(x), lo = bf16(x - hi):
//   a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi      (relative error about 2^-16)
//
// Forward, per batch of 32 depth-ordered Gaussians and per wave of 64 pixels:
//   each lane runs its pixel's transmittance recurrence and writes w[p][i] = alpha_i T_i
//   to LDS, then out^T[c][p] += sum_i F^T[c][i] W^T[i][p] on the matrix cores.
// Backward, per batch (back to front):
//   GF^T[i][p] = sum_c F[i][c] G^T[c][p]  (g . f of every pixel-Gaussian pair) on the
//     single-precision matrix cores (v_mfma_f32_16x16x4f32: it decides dL/dalpha, in
//     which terms cancel); a 4x4 block transpose across lane rows (permlane swaps) hands every
//     lane its own pixel's 32 values;
//   each lane runs the reverse recurrence (T recovered with the reciprocal of 1 - alpha)
//     and writes w[i][p] to LDS, Gaussian-major;
//   dF[i][c] = sum_p W^T[i][p] G[p][c]                       (feature gradients)
//   the 2D mean, conic and opacity gradients are summed per pair in single precision
//   (row sums over 16 lanes, then over rows and waves in LDS): expanding them into
//   moments about a fixed centre would lose accuracy for compact Gaussians.
//
// 16x16x32 bf16 operand layout (lane l, verified on the device):
//   A[i][k]: i = l % 16, k = 8 (l / 16) + 0..7     B[k][j]: k = 8 (l / 16) + 0..7, j = l % 16
//   D[i][j]: j = l % 16, i = 4 (l / 16) + r, r = 0..3
#include "common.h"

namespace gs {

int64_t scan_partials_needed(int64_t n);
int scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partial, uint64_t* total, hipStream_t s);

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kB = 32;          // Gaussians per batch
constexpr int kWs = kB + 4;     // dword stride of a pixel-major row of 32 Gaussians
constexpr int kPs = 64 + 4;     // dword stride of a Gaussian-major row of a wave's 64 pixels

template <int NS>
struct SShape {
  static constexpr int K = 4 + NS;
  static constexpr int KP = (K + 31) / 32 * 32;   // channels padded to whole 32-wide k-steps
  static constexpr int KS = KP / 32;
  static constexpr int CB = KP / 16;              // 16-channel blocks
  static constexpr int CPT = KP / 8;              // channels staged per thread
  static constexpr int FST = KP + 4;              // dword stride of a Gaussian-major feature row
};

// x -> (bf16(x) << 16) | bf16(x - bf16(x))
__device__ __forceinline__ uint32_t pack_hl(float x) {
  const float h = (float)(__bf16)x;
  const bf2 v = __builtin_convertvector((f2){x - h, x}, bf2);
  return __builtin_bit_cast(uint32_t, v);
}

// Eight packed values -> the hi and lo bfloat16 operands.
__device__ __forceinline__ void unpack8(const uint4 a, const uint4 b, v8bf& hi, v8bf& lo) {
  const uint32_t d[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  uint4 h, l;
  h.x = __builtin_amdgcn_perm(d[1], d[0], 0x07060302u);
  h.y = __builtin_amdgcn_perm(d[3], d[2], 0x07060302u);
  h.z = __builtin_amdgcn_perm(d[5], d[4], 0x07060302u);
  h.w = __builtin_amdgcn_perm(d[7], d[6], 0x07060302u);
  l.x = __builtin_amdgcn_perm(d[1], d[0], 0x05040100u);
  l.y = __builtin_amdgcn_perm(d[3], d[2], 0x05040100u);
  l.z = __builtin_amdgcn_perm(d[5], d[4], 0x05040100u);
  l.w = __builtin_amdgcn_perm(d[7], d[6], 0x05040100u);
  hi = __builtin_bit_cast(v8bf, h);
  lo = __builtin_bit_cast(v8bf, l);
}

__device__ __forceinline__ void load_op(const uint32_t* p, v8bf& hi, v8bf& lo) {
  const uint4 a = *reinterpret_cast<const uint4*>(p);
  const uint4 b = *reinterpret_cast<const uint4*>(p + 4);
  unpack8(a, b, hi, lo);
}

// Splits eight floats into hi and lo operands, two values per conversion.
__device__ __forceinline__ void split8(const float* x, v8bf& hi, v8bf& lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t hb = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){x[2 * k], x[2 * k + 1]}, bf2));
    const float h0 = __uint_as_float(hb << 16), h1 = __uint_as_float(hb & 0xffff0000u);
    h[k] = hb;
    l[k] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){x[2 * k] - h0, x[2 * k + 1] - h1}, bf2));
  }
  hi = __builtin_bit_cast(v8bf, make_uint4(h[0], h[1], h[2], h[3]));
  lo = __builtin_bit_cast(v8bf, make_uint4(l[0], l[1], l[2], l[3]));
}

// The render record as the compositing loops read it from LDS, per Gaussian two float4:
//   (mx, my, -, -)  mean2d relative to the centre of the tile's first pixel, so that a
//                   pixel's offset is its integer position in the tile minus (mx, my);
//   (a, b, c, o)    the conic scaled so that a dx^2 + b dx dy + c dy^2 is the exponent of
//                   eq. 4 in base 2: a = -A log2(e) / 2, b = -B log2(e), c = -C log2(e) / 2.
// The mean's hi + lo sum is rounded once, after the exact subtraction of the tile origin.
constexpr float kLog2e = 1.4426950408889634f;
__device__ __forceinline__ float4 local_rec(const float4 r, int part, float ox, float oy) {
  if (part == 0) return make_float4((r.x - ox) + r.z, (r.y - oy) + r.w, 0.0f, 0.0f);
  return make_float4(-0.5f * kLog2e * r.x, -kLog2e * r.y, -0.5f * kLog2e * r.z, r.w);
}

// Base-2 footprint exponent at tile-local pixel (lx, ly), clamped at zero; dx, dy are the
// pixel's offsets from the mean and t = a dx + b dy.
__device__ __forceinline__ float local_power2(float lx, float ly, const float4 r0, const float4 r1, float& dx,
                                              float& dy, float& t) {
  dx = lx - r0.x;
  dy = ly - r0.y;
  t = __builtin_fmaf(r1.x, dx, r1.y * dy);
  return fminf(__builtin_fmaf(t, dx, (r1.z * dy) * dy), 0.0f);
}

__device__ __forceinline__ v4f mma(v8bf a, v8bf b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
__device__ __forceinline__ v4f mma3(v8bf ah, v8bf al, v8bf bh, v8bf bl, v4f c) {
  c = mma(ah, bh, c);
  c = mma(ah, bl, c);
  c = mma(al, bh, c);
  return c;
}
__device__ __forceinline__ v4f zero4() { return (v4f){0.0f, 0.0f, 0.0f, 0.0f}; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Batch staging, double-buffered through registers: thread t stages Gaussian q = t / 8
// of the batch, channels [(t % 8) CPT, +CPT) of its features and, for t % 8 < 2, half of
// its 8-float record.
template <int NS>
struct SStage {
  static constexpr int CPT = SShape<NS>::CPT;
  float4 r;
  uint32_t gid;
  float f[CPT];

  __device__ __forceinline__ void fetch(const uint32_t* __restrict__ vals, uint32_t b, int cnt, int item, int64_t n,
                                        const float* __restrict__ rec, const float* __restrict__ depth,
                                        const float* __restrict__ rgb, const float* __restrict__ sem,
                                        const uint16_t* __restrict__ emb, int n_sem) {
    const int q = threadIdx.x >> 3, part = threadIdx.x & 7;
    const bool live = q < cnt;
    const uint32_t g = live ? vals[b + q] : 0u;
    gid = g;
    const int64_t e = (int64_t)item * n + g;
    r = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live && part < 2) r = reinterpret_cast<const float4*>(rec + kRecFloats * e)[part];
    const int Kr = 4 + n_sem;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int k = part * CPT + j;
      float v = 0.0f;
      if (live && k < Kr) {
        if (k < 3) v = rgb[3 * (int64_t)g + k];
        else if (k == 3) v = depth[e];
        else if (emb) v = __uint_as_float((uint32_t)emb[(int64_t)n_sem * g + (k - 4)] << 16);
        else v = sem[(int64_t)n_sem * g + (k - 4)];
      }
      f[j] = v;
    }
  }
  // features Gaussian-major, single precision: s_f[q][c]; Gaussian ids to s_gid[q]
  __device__ __forceinline__ void commit_rows(float4* s_rec, float* s_f, uint32_t* s_gid, float ox, float oy) const {
    const int q = threadIdx.x >> 3, part = threadIdx.x & 7;
    if (part < 2) s_rec[2 * q + part] = local_rec(r, part, ox, oy);
    if (part == 0) s_gid[q] = gid;
    float* dst = s_f + q * SShape<NS>::FST + part * CPT;
#pragma unroll
    for (int j = 0; j < CPT; j += 4) *reinterpret_cast<float4*>(dst + j) = make_float4(f[j], f[j + 1], f[j + 2], f[j + 3]);
  }
  // features channel-major: s_f[c][q]
  __device__ __forceinline__ void commit_cols(float4* s_rec, uint32_t* s_f, float ox, float oy) const {
    const int q = threadIdx.x >> 3, part = threadIdx.x & 7;
    if (part < 2) s_rec[2 * q + part] = local_rec(r, part, ox, oy);
#pragma unroll
    for (int j = 0; j < CPT; ++j) s_f[(part * CPT + j) * kWs + q] = pack_hl(f[j]);
  }
};

// ------------------------------------------------------------------------- forward
template <int NS>
__global__ __launch_bounds__(256, 3) void k_render_fwd_split(gs_config cfg, const float* __restrict__ rgb,
                                                          const float* __restrict__ sem,
                                                          const uint16_t* __restrict__ emb, int n_sem,
                                                          const float* __restrict__ rec,
                                                          const float* __restrict__ depth, int64_t n,
                                                          const gs_item* __restrict__ items, int n_items,
                                                          const uint32_t* __restrict__ vals,
                                                          const uint32_t* __restrict__ ranges, float* __restrict__ color,
                                                          float* __restrict__ Tout, uint32_t* __restrict__ ncout) {
  using S = SShape<NS>;
  constexpr int CB = S::CB, KP = S::KP;
  __shared__ float4 s_rec[2 * kB];
  __shared__ uint32_t s_f[KP * kWs];          // F^T, packed hi|lo, [channel][Gaussian]
  __shared__ float s_w[4][64 * kWs];          // per wave W, [pixel][Gaussian]
  const Ctx c = make_ctx(items, n_items, ranges, cfg.tile_order);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, g4 = lane >> 4;
  int u, v;
  tile_pixel(c, tid, u, v);
  const bool inside = u < c.W && v < c.H;
  const float lx = (float)(tid & 15), ly = (float)(tid >> 4);
  const float ox = (float)(c.tx * kTile) + 0.5f, oy = (float)(c.ty * kTile) + 0.5f;
  v4f acc[CB][4];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) acc[cb][pb] = zero4();
  float T = 1.0f;
  bool done = !inside;
  uint32_t last = 0;
  const float amin = cfg.alpha_min, amax = cfg.alpha_max, tmin = cfg.t_min;
  float* W = s_w[wave];
  SStage<NS> st;
  if (c.start < c.end)
    st.fetch(vals, c.start, (int)min((uint32_t)kB, c.end - c.start), c.item, n, rec, depth, rgb, sem, emb, n_sem);
  for (uint32_t b = c.start; b < c.end; b += kB) {
    // every wave is past the previous batch's LDS reads; stop once every pixel has
    if (__syncthreads_count(!done) == 0) break;
    st.commit_cols(s_rec, s_f, ox, oy);
    __syncthreads();
    const int cnt = (int)min((uint32_t)kB, c.end - b);
    if (b + kB < c.end)
      st.fetch(vals, b + kB, (int)min((uint32_t)kB, c.end - b - kB), c.item, n, rec, depth, rgb, sem, emb, n_sem);
    // front-to-back recurrence, branch-free; only T carries from one Gaussian to the next
    bool took = false;
    const uint32_t base = b - c.start;
#pragma unroll
    for (int q4 = 0; q4 < kB; q4 += 4) {
      float wq[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = q4 + e;
        const float4 r0 = s_rec[2 * q], r1 = s_rec[2 * q + 1];
        float dx, dy, t;
        const float araw = r1.w * __builtin_amdgcn_exp2f(local_power2(lx, ly, r0, r1, dx, dy, t));
        const bool ok = (q < cnt) & !done & (araw >= amin);
        const float w = fminf(amax, araw) * T;
        const float Tn = T - w;
        const bool stop = ok & (Tn < tmin);
        const bool take = ok & !stop;
        wq[e] = take ? w : 0.0f;
        T = take ? Tn : T;
        done = done | stop;
        last = take ? base + q + 1 : last;
        took |= take;
      }
      *reinterpret_cast<float4*>(W + lane * kWs + q4) = make_float4(wq[0], wq[1], wq[2], wq[3]);
    }
    wave_sync();
    if (__ballot(took) == 0ull) continue;
    // out^T[c][p] += F^T[c][i] W^T[i][p]: A = F^T (i = channel 16 cb + l16, k = Gaussian 8 g4 + e),
    // B = W^T (k = Gaussian, j = pixel 16 pb + l16)
    v8bf ah[CB], al[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) load_op(s_f + (16 * cb + l16) * kWs + 8 * g4, ah[cb], al[cb]);
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) {
      const float* src = W + (16 * pb + l16) * kWs + 8 * g4;
      const float4 w0 = *reinterpret_cast<const float4*>(src), w1 = *reinterpret_cast<const float4*>(src + 4);
      const float x[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
      v8bf bh, bl;
      split8(x, bh, bl);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[cb][pb] = mma3(ah[cb], al[cb], bh, bl, acc[cb][pb]);
    }
  }
  // D[c][p]: lane holds pixel 16 pb + l16 of this wave, channels 16 cb + 4 g4 + r
  const int Kr = 4 + n_sem;
#pragma unroll
  for (int pb = 0; pb < 4; ++pb) {
    int pu, pv;
    tile_pixel(c, wave * 64 + 16 * pb + l16, pu, pv);
    if (pu >= c.W || pv >= c.H) continue;
    const int64_t pbase = c.pixel_base * Kr + (int64_t)pv * c.W + pu;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ch = 16 * cb + 4 * g4 + r;
        if (ch < Kr) color[pbase + ch * c.HW] = acc[cb][pb][r];
      }
  }
  if (!inside) return;
  const int64_t pix = c.pixel_base + (int64_t)v * c.W + u;
  Tout[pix] = T;
  ncout[pix] = last;
}

// ------------------------------------------------------------------------- backward
// Swaps the 4x4 blocks (lane row R, register group X[pb]) -> (lane row pb, group R):
// permlane32 exchanges rows 0,1 with 2,3, permlane16 rows 0 with 1 and 2 with 3.
__device__ __forceinline__ void block_transpose(uint32_t (&X)[4][8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    auto s02 = __builtin_amdgcn_permlane32_swap(X[0][k], X[2][k], false, false);
    auto s13 = __builtin_amdgcn_permlane32_swap(X[1][k], X[3][k], false, false);
    X[0][k] = s02[0];
    X[2][k] = s02[1];
    X[1][k] = s13[0];
    X[3][k] = s13[1];
    auto s01 = __builtin_amdgcn_permlane16_swap(X[0][k], X[1][k], false, false);
    auto s23 = __builtin_amdgcn_permlane16_swap(X[2][k], X[3][k], false, false);
    X[0][k] = s01[0];
    X[1][k] = s01[1];
    X[2][k] = s23[0];
    X[3][k] = s23[1];
  }
}

// Long tile lists are cut into segments of kSeg list positions, each a work item of its
// own, so that the longest list no longer sets the length of the launch. Walking a
// segment backwards needs, per pixel, the transmittance after it and the suffix
// sum over every later Gaussian of w (g . f). A summary pass gives every segment s of a
// long list, per pixel,
//   P_s  = prod over its blended Gaussians of (1 - alpha)            (front to back)
//   GC_s = sum over its blended Gaussians of alpha T_loc (g . f),     T_loc from 1
// and then T_after(s) = prod_{s' <= s} P_s' and suffix(s) = sum_{s' > s} T_before(s') GC_s'.
constexpr int kSeg = 256;

// With the exponent E = a dx^2 + b dx dy + c dy^2 of the local record (E = log2(e) power),
// d power/d mean2d = -(dE/d dx, dE/d dy) / log2(e) and d power/d(A, B, C) =
// -(dx^2 / 2, dx dy, dy^2 / 2); the reverse pass sums dE/d dx, dE/d dy, dx^2, dx dy, dy^2
// (times dL/d power) and applies these factors once per Gaussian.
__constant__ float kGeoScale[6] = {-1.0f / kLog2e, -1.0f / kLog2e, -0.5f, -1.0f, -0.5f, 1.0f};

// One block per tile: the tile's list length in use (largest n_contrib) and its segment
// count, stored in work order (coarse pyramid levels first unless tile_order = 1).
__global__ __launch_bounds__(256) void k_seg_count(const gs_item* __restrict__ items, int n_items,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ ncin, int n_tiles, int order,
                                                   uint32_t* __restrict__ tile_lmax, uint32_t* __restrict__ cnt_ord) {
  __shared__ uint32_t s_m;
  const int tile = blockIdx.x;
  const int item = item_of_tile(items, n_items, tile);
  const gs_item it = items[item];
  const int lt = tile - it.tile_base;
  const int u = (lt % it.tiles_x) * kTile + (threadIdx.x & 15), v = (lt / it.tiles_x) * kTile + (threadIdx.x >> 4);
  const uint32_t len = ranges[2 * (int64_t)tile + 1] - ranges[2 * (int64_t)tile];
  const uint32_t last = (u < it.W && v < it.H) ? min(ncin[it.pixel_base + (int64_t)v * it.W + u], len) : 0u;
  if (threadIdx.x == 0) s_m = 0;
  __syncthreads();
  atomicMax(&s_m, last);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t m = s_m;
    tile_lmax[tile] = m;
    cnt_ord[order ? tile : n_tiles - 1 - tile] = m == 0 ? 0u : (m <= (uint32_t)kSeg ? 1u : (m + kSeg - 1) / kSeg);
  }
}

// Work list: (tile, segment | segment count << 16). If the segments do not fit the
// workspace, every tile becomes a single item. Also resets the two work counters.
__global__ void k_seg_list(const uint32_t* __restrict__ cnt_ord, const uint32_t* __restrict__ base_ord,
                           const uint64_t* __restrict__ total, int n_tiles, int order, int64_t max_segs,
                           uint2* __restrict__ work, uint32_t* __restrict__ ctl) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t tot = *total;
  const bool fits = tot <= (uint64_t)max_segs;
  if (o == 0) {
    ctl[0] = fits ? (uint32_t)tot : (uint32_t)n_tiles;
    ctl[1] = 0;
    ctl[2] = 0;
  }
  if (o >= n_tiles) return;
  const uint32_t tile = order ? o : n_tiles - 1 - o;
  if (fits) {
    const uint32_t c = cnt_ord[o], b = base_ord[o];
    for (uint32_t k = 0; k < c; ++k) work[b + k] = make_uint2(tile, k | (c << 16));
  } else {
    work[o] = make_uint2(tile, 1u << 16);
  }
}

// SUMMARY = false: the reverse pass proper over one work item (a whole tile list, or one
// segment of it). SUMMARY = true: the per-segment P and GC of the segments of long lists.
// Persistent blocks take work items from a counter until the list is exhausted.
template <int NS, bool SUMMARY>
__global__ __launch_bounds__(256, 2) void k_render_bwd_split(gs_config cfg, const float* __restrict__ rgb,
                                                          const float* __restrict__ sem,
                                                          const uint16_t* __restrict__ emb, int n_sem,
                                                          const float* __restrict__ rec,
                                                          const float* __restrict__ depth, int64_t n,
                                                          const gs_item* __restrict__ items, int n_items,
                                                          const uint32_t* __restrict__ vals,
                                                          const uint32_t* __restrict__ ranges,
                                                          const float* __restrict__ Tfin,
                                                          const uint32_t* __restrict__ ncin,
                                                          const float* __restrict__ gcolor, float* __restrict__ g2d,
                                                          float* __restrict__ grgb, float* __restrict__ gsem,
                                                          const uint2* __restrict__ work, uint32_t* __restrict__ ctl,
                                                          const uint32_t* __restrict__ tile_lmax,
                                                          float* __restrict__ segP, float* __restrict__ segGC) {
  using S = SShape<NS>;
  constexpr int KP = S::KP, CB = S::CB, FST = S::FST;
  __shared__ float4 s_rec[2 * kB];
  __shared__ float s_f[kB * FST];             // F, [Gaussian][channel]
  __shared__ float s_w[SUMMARY ? 1 : 4][16 * kPs];      // per wave, 16 Gaussians: W, [Gaussian][pixel]
  __shared__ float s_df[SUMMARY ? 1 : kB * KP];
  __shared__ float s_geo[SUMMARY ? 1 : kB * 6 * 16];     // [Gaussian][component][row slot]
  __shared__ uint32_t s_wi;
  __shared__ uint32_t s_gid[kB];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int Kr = 4 + n_sem;
  const float amin = cfg.alpha_min, amax = cfg.alpha_max;
  const uint32_t n_work = ctl[0];
  for (;;) {
    if (tid == 0) s_wi = atomicAdd(&ctl[SUMMARY ? 1 : 2], 1u);
    lds_barrier();
    const uint32_t wi = s_wi;
    lds_barrier();
    if (wi >= n_work) break;
    const uint2 wk = work[wi];
    const int tile = (int)wk.x;
    const int seg = (int)(wk.y & 0xffffu), nseg = (int)(wk.y >> 16);
    if (SUMMARY && nseg < 2) continue;
    const Ctx c = make_ctx_of(items, n_items, ranges, tile);
    int u, v;
    tile_pixel(c, tid, u, v);
    const bool inside = u < c.W && v < c.H;
    const float lx = (float)(tid & 15), ly = (float)(tid >> 4);
    const float ox = (float)(c.tx * kTile) + 0.5f, oy = (float)(c.ty * kTile) + 0.5f;
    const int64_t pix = c.pixel_base + (int64_t)v * c.W + u;
    // n_contrib comes from the matching forward; clamp so that a mismatched call stays in range
    const uint32_t len = c.end - c.start;
    const uint32_t last = inside ? min(ncin[pix], len) : 0u;
    const int lmax = (int)tile_lmax[tile];
    const int a0 = nseg == 1 ? 0 : seg * kSeg;
    const int b0 = nseg == 1 ? lmax : min(lmax, a0 + kSeg);

    // upstream gradient of a wave pixel (0..63) and channel, zero outside the image
    auto gval = [&](int wp, int ch) -> float {
      int pu, pv;
      tile_pixel(c, wave * 64 + wp, pu, pv);
      if (pu >= c.W || pv >= c.H || ch >= Kr) return 0.0f;
      return gcolor[c.pixel_base * Kr + (int64_t)pv * c.W + pu + ch * c.HW];
    };
    // G^T as B of GF (k = channel 4 ks + g4, j = pixel 16 pb + l16)
    float g1[4][KP / 4];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb)
#pragma unroll
      for (int ks = 0; ks < KP / 4; ++ks) g1[pb][ks] = gval(16 * pb + l16, 4 * ks + g4);
    // G as B of dF (k = pixel 32 ks + 8 g4 + e, j = channel 16 cb + l16)
    v8bf g2h[2][SUMMARY ? 1 : CB], g2l[2][SUMMARY ? 1 : CB];
    if constexpr (!SUMMARY) {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          float x[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = gval(32 * ks + 8 * g4 + e, 16 * cb + l16);
          split8(x, g2h[ks][cb], g2l[ks][cb]);
        }
    }

    // per-pixel state at the segment's back end (main pass) or front end (summary pass)
    float T = 1.0f, acc = 0.0f;   // acc: suffix (main) or GC (summary)
    if constexpr (!SUMMARY) {
      const float tf = inside ? Tfin[pix] : 1.0f;
      if (nseg == 1 || seg == nseg - 1) T = tf;
      if (nseg > 1) {
        const int64_t w0 = (int64_t)wi - seg;
        float tb = 1.0f;   // transmittance in front of segment s
        for (int s = 0; s < nseg; ++s) {
          const float P = segP[(w0 + s) * kTilePx + tid], GC = segGC[(w0 + s) * kTilePx + tid];
          if (s > seg) acc = __builtin_fmaf(tb, GC, acc);
          tb *= P;
          if (s == seg && seg < nseg - 1) T = tb;
        }
      }
    }

    SStage<NS> st;
    if (b0 > a0) {
      const int f0 = SUMMARY ? a0 : max(a0, b0 - kB);
      const int f1 = SUMMARY ? min(b0, a0 + kB) : b0;
      st.fetch(vals, c.start + f0, f1 - f0, c.item, n, rec, depth, rgb, sem, emb, n_sem);
    }
    const int n_batches = (b0 - a0 + kB - 1) / kB;
    for (int bi = 0; bi < n_batches; ++bi) {
      // main pass: batches from the back; summary pass: from the front
      const int lo = SUMMARY ? a0 + bi * kB : max(a0, b0 - (bi + 1) * kB);
      const int hi = SUMMARY ? min(b0, lo + kB) : b0 - bi * kB;
      const int cnt = hi - lo;
      lds_barrier();
      st.commit_rows(s_rec, s_f, s_gid, ox, oy);
      if constexpr (!SUMMARY) {
        for (int i = tid; i < kB * KP; i += 256) s_df[i] = 0.0f;
        for (int i = tid; i < kB * 6 * 16; i += 256) s_geo[i] = 0.0f;
      }
      lds_barrier();
      if (bi + 1 < n_batches) {
        const int nlo = SUMMARY ? hi : max(a0, lo - kB);
        const int nhi = SUMMARY ? min(b0, hi + kB) : lo;
        st.fetch(vals, c.start + nlo, nhi - nlo, c.item, n, rec, depth, rgb, sem, emb, n_sem);
      }
      if (__ballot((uint32_t)lo < last) != 0ull) {
        // GF^T[i][p] in single precision (it decides dL/dalpha, where terms cancel):
        // v_mfma_f32_16x16x4f32, A = F (i = Gaussian 16 bq + l16, k = channel 4 ks + g4), B = G^T
        uint32_t X[4][8];
        {
          v4f gfa[4][2];
#pragma unroll
          for (int pb = 0; pb < 4; ++pb) gfa[pb][0] = gfa[pb][1] = zero4();
#pragma unroll
          for (int bq = 0; bq < 2; ++bq)
#pragma unroll
            for (int ks = 0; ks < KP / 4; ++ks) {
              const float a = s_f[(16 * bq + l16) * FST + 4 * ks + g4];
#pragma unroll
              for (int pb = 0; pb < 4; ++pb)
                gfa[pb][bq] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, g1[pb][ks], gfa[pb][bq], 0, 0, 0);
            }
#pragma unroll
          for (int pb = 0; pb < 4; ++pb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              X[pb][r] = __float_as_uint(gfa[pb][0][r]);
              X[pb][4 + r] = __float_as_uint(gfa[pb][1][r]);
            }
        }
        // lane row g4 held Gaussians {4 g4 + r, 16 + 4 g4 + r} of all four pixel rows; now
        // every lane holds its own pixel's values: X[g][4 bq + r] = gf of Gaussian 16 bq + 4 g + r
        block_transpose(X);
        if constexpr (SUMMARY) {
#pragma unroll
          for (int q = 0; q < kB; ++q) {
            const float4 r0 = s_rec[2 * q], r1 = s_rec[2 * q + 1];
            float dx, dy, t;
            const float araw = r1.w * __builtin_amdgcn_exp2f(local_power2(lx, ly, r0, r1, dx, dy, t));
            const bool act = (q < cnt) & ((uint32_t)(lo + q) < last) & (araw >= amin);
            const float w = fminf(amax, araw) * T;
            const float gf = __uint_as_float(X[(q >> 2) & 3][4 * (q >> 4) + (q & 3)]);
            acc = act ? __builtin_fmaf(w, gf, acc) : acc;
            T = act ? T - w : T;
          }
        } else {
          // reverse recurrence, one 16-Gaussian block at a time (back to front)
#pragma unroll
          for (int bq = 1; bq >= 0; --bq) {
            float* Wp = s_w[wave];
            bool any = false;
#pragma unroll
            for (int gq = 3; gq >= 0; --gq)
#pragma unroll
              for (int r = 3; r >= 0; --r) {
                const int q = 16 * bq + 4 * gq + r;
                const float4 r0 = s_rec[2 * q], r1 = s_rec[2 * q + 1];
                float dx, dy, t;
                const float G = __builtin_amdgcn_exp2f(local_power2(lx, ly, r0, r1, dx, dy, t));
                const float araw = r1.w * G;
                const bool act = (q < cnt) & ((uint32_t)(lo + q) < last) & (araw >= amin);
                const float a = fminf(amax, araw);
                const float rom = __builtin_amdgcn_rcpf(1.0f - a);
                const float Tq = act ? T * rom : T;   // transmittance in front of this Gaussian
                const float w = act ? a * Tq : 0.0f;
                const float gf = __uint_as_float(X[gq][4 * bq + r]);
                const float dalpha = Tq * gf - acc * rom;
                acc = act ? __builtin_fmaf(gf, w, acc) : acc;
                T = Tq;
                const bool unclamped = act & (araw < amax);
                const float dpow = unclamped ? dalpha * araw : 0.0f;
                const float dop = unclamped ? dalpha * G : 0.0f;
                Wp[(4 * gq + r) * kPs + lane] = w;
                if (__ballot(act) != 0ull) {
                  any = true;
                  // d power / d (mean2d, A, B, C) up to the per-component factors of kGeoScale
                  const float pdx = dpow * dx, pdy = dpow * dy;
                  const float s0 = row_sum16(dpow * __builtin_fmaf(r1.x, dx, t));   // 2a dx + b dy
                  const float s1 = row_sum16(dpow * __builtin_fmaf(r1.y, dx, 2.0f * (r1.z * dy)));
                  const float s2 = row_sum16(pdx * dx);
                  const float s3 = row_sum16(pdx * dy);
                  const float s4 = row_sum16(pdy * dy);
                  const float s5 = row_sum16(dop);                                  // d/d opacity
                  if (l16 == 0) {
                    float* dst = s_geo + q * 96 + wave * 4 + g4;
                    dst[0] = s0; dst[16] = s1; dst[32] = s2; dst[48] = s3; dst[64] = s4; dst[80] = s5;
                  }
                }
              }
            wave_sync();
            if (__ballot(any) != 0ull) {
              // A = W^T (i = Gaussian l16 of the block, k = pixel 32 ks + 8 g4 + e)
              v8bf wh[2], wl[2];
#pragma unroll
              for (int ks = 0; ks < 2; ++ks) {
                const float* src = Wp + l16 * kPs + 32 * ks + 8 * g4;
                const float4 w0 = *reinterpret_cast<const float4*>(src), w1 = *reinterpret_cast<const float4*>(src + 4);
                const float x[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
                split8(x, wh[ks], wl[ks]);
              }
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) {
                v4f d = zero4();
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) d = mma3(wh[ks], wl[ks], g2h[ks][cb], g2l[ks][cb], d);
                // D[i][c]: Gaussian 16 bq + 4 g4 + r, channel 16 cb + l16
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  if (d[r] != 0.0f) atomicAdd(&s_df[(16 * bq + 4 * g4 + r) * KP + 16 * cb + l16], d[r]);
              }
            }
            wave_sync();   // the block's W is consumed before the next block overwrites it
          }
        }
      }
      if constexpr (!SUMMARY) {
        lds_barrier();
        for (int idx = tid; idx < cnt * KP; idx += 256) {
          const int q = idx / KP, k = idx - q * KP;
          const float val = s_df[idx];
          if (val == 0.0f || k >= Kr) continue;
          const uint32_t g = s_gid[q];
          if (k < 3) atomicAdd(&grgb[3 * (int64_t)g + k], val);
          else if (k == 3) atomicAdd(&g2d[8 * ((int64_t)c.item * n + g) + 6], val);
          else atomicAdd(&gsem[(int64_t)n_sem * g + (k - 4)], val);
        }
        for (int idx = tid; idx < cnt * 6; idx += 256) {
          const int q = idx / 6, comp = idx - q * 6;
          const float* src = s_geo + q * 96 + comp * 16;
          float sum = 0.0f;
#pragma unroll
          for (int r = 0; r < 16; ++r) sum += src[r];
          if (sum != 0.0f) {
            const uint32_t g = s_gid[q];
            atomicAdd(&g2d[8 * ((int64_t)c.item * n + g) + comp], sum * kGeoScale[comp]);
          }
        }
      }
    }
    if constexpr (SUMMARY) {
      segP[(int64_t)wi * kTilePx + tid] = T;
      segGC[(int64_t)wi * kTilePx + tid] = acc;
    }
  }
}

template <int NS>
int launch_fwd_s(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items, int n_items,
                 int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& out, hipStream_t s) {
  hipLaunchKernelGGL(k_render_fwd_split<NS>, dim3(n_tiles), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb, cfg.n_sem,
                     p.rec, p.depth, g.n, items, n_items, vals, ranges, out.color, out.T, out.n_contrib);
  return launch_status();
}

// Caller workspace of the reverse pass: the segment work list, sized for `cap` duplicates.
struct SegWs {
  uint32_t *lmax, *cnt, *base, *partial, *ctl;
  uint64_t* total;
  uint2* work;
  float *P, *GC;
  int64_t max_segs;
};

size_t seg_layout(int n_tiles, int64_t cap, char* base, SegWs* w) {
  const int64_t max_segs = (int64_t)n_tiles + ceil_div(cap, kSeg) + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return base ? base + o : nullptr;
  };
  char* p_lmax = take(4 * (size_t)n_tiles);
  char* p_cnt = take(4 * (size_t)n_tiles);
  char* p_base = take(4 * (size_t)n_tiles);
  char* p_part = take(4 * (size_t)scan_partials_needed(n_tiles));
  char* p_tot = take(8);
  char* p_ctl = take(16);
  char* p_work = take(8 * (size_t)max_segs);
  char* p_P = take(4 * (size_t)kTilePx * max_segs);
  char* p_GC = take(4 * (size_t)kTilePx * max_segs);
  if (w) {
    w->lmax = (uint32_t*)p_lmax;
    w->cnt = (uint32_t*)p_cnt;
    w->base = (uint32_t*)p_base;
    w->partial = (uint32_t*)p_part;
    w->total = (uint64_t*)p_tot;
    w->ctl = (uint32_t*)p_ctl;
    w->work = (uint2*)p_work;
    w->P = (float*)p_P;
    w->GC = (float*)p_GC;
    w->max_segs = max_segs;
  }
  return off;
}

// Blocks of a persistent launch: resident blocks per CU times CUs, per device and kernel.
template <class F>
int persistent_grid(F kernel) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess) return 0;
  return std::max(1, cus * std::max(1, per));
}

template <int NS>
int launch_bwd_s(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items, int n_items,
                 int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& fwd,
                 const gs_images& gin, float* g2d, const gs_grads& gr, void* seg_ws, int64_t cap, hipStream_t s) {
  SegWs w;
  seg_layout(n_tiles, cap, (char*)seg_ws, &w);
  hipLaunchKernelGGL(k_seg_count, dim3(n_tiles), dim3(256), 0, s, items, n_items, ranges, fwd.n_contrib, n_tiles,
                     cfg.tile_order, w.lmax, w.cnt);
  int st = launch_status();
  st = st ? st : scan_u32(w.cnt, w.base, n_tiles, w.partial, w.total, s);
  if (st) return st;
  hipLaunchKernelGGL(k_seg_list, dim3((unsigned)ceil_div(n_tiles, 256)), dim3(256), 0, s, w.cnt, w.base, w.total,
                     n_tiles, cfg.tile_order, w.max_segs, w.work, w.ctl);
  static int grid_sum = 0, grid_main = 0;
  if (!grid_sum) grid_sum = persistent_grid(k_render_bwd_split<NS, true>);
  if (!grid_main) grid_main = persistent_grid(k_render_bwd_split<NS, false>);
  if (!grid_sum || !grid_main) return GS_ERR_HIP;
  hipLaunchKernelGGL((k_render_bwd_split<NS, true>), dim3(grid_sum), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb, cfg.n_sem,
                     p.rec, p.depth, g.n, items, n_items, vals, ranges, fwd.T, fwd.n_contrib, gin.color, g2d, gr.rgb,
                     gr.sem, w.work, w.ctl, w.lmax, w.P, w.GC);
  hipLaunchKernelGGL((k_render_bwd_split<NS, false>), dim3(grid_main), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb,
                     cfg.n_sem, p.rec, p.depth, g.n, items, n_items, vals, ranges, fwd.T, fwd.n_contrib, gin.color, g2d,
                     gr.rgb, gr.sem, w.work, w.ctl, w.lmax, w.P, w.GC);
  return launch_status();
}

}  // namespace

size_t render_seg_workspace(int n_tiles, int64_t dup_capacity) {
  return seg_layout(n_tiles, std::max<int64_t>(dup_capacity, 0), nullptr, nullptr);
}

// Largest duplicate capacity whose segment workspace fits in `bytes` (-1 if none does).
int64_t render_seg_capacity(int n_tiles, size_t bytes) {
  if (render_seg_workspace(n_tiles, 0) > bytes) return -1;
  int64_t lo = 0, hi = 1;
  while (hi < ((int64_t)1 << 40) && render_seg_workspace(n_tiles, hi) <= bytes) hi *= 2;
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (render_seg_workspace(n_tiles, mid) <= bytes) lo = mid; else hi = mid;
  }
  return lo;
}

int launch_render_fwd_split(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items,
                            int n_items, int n_tiles, const uint32_t* vals, const uint32_t* ranges,
                            const gs_images& out, hipStream_t s) {
  const int ns = cfg.n_sem;
  if (ns <= 28) return launch_fwd_s<28>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  if (ns <= 60) return launch_fwd_s<60>(cfg, g, p, items, n_items, n_tiles, vals, ranges, out, s);
  return GS_ERR_UNSUPPORTED;
}

int launch_render_bwd_split(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items,
                            int n_items, int n_tiles, const uint32_t* vals, const uint32_t* ranges,
                            const gs_images& fwd, const gs_images& gin, float* g2d, const gs_grads& gr, void* seg_ws,
                            int64_t cap, hipStream_t s) {
  const int ns = cfg.n_sem;
  if (cap < 0) return GS_ERR_WORKSPACE;
  if (ns <= 28)
    return launch_bwd_s<28>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, seg_ws, cap, s);
  if (ns <= 60)
    return launch_bwd_s<60>(cfg, g, p, items, n_items, n_tiles, vals, ranges, fwd, gin, g2d, gr, seg_ws, cap, s);
  return GS_ERR_UNSUPPORTED;
}

}  // namespace gs
