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

// Splits eight floats into three bfloat16 parts, x = hi + mid + lo to about 2^-24 of x
// (each part the rounding of what the previous ones leave, every remainder exact).
__device__ __forceinline__ void split8x3(const float* x, v8bf& hi, v8bf& mid, v8bf& lo) {
  split8(x, hi, mid);
  const uint4 h = __builtin_bit_cast(uint4, hi), m = __builtin_bit_cast(uint4, mid);
  const uint32_t hw[4] = {h.x, h.y, h.z, h.w}, mw[4] = {m.x, m.y, m.z, m.w};
  uint32_t l[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float r0 = (x[2 * k] - __uint_as_float(hw[k] << 16)) - __uint_as_float(mw[k] << 16);
    const float r1 = (x[2 * k + 1] - __uint_as_float(hw[k] & 0xffff0000u)) - __uint_as_float(mw[k] & 0xffff0000u);
    l[k] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){r0, r1}, bf2));
  }
  lo = __builtin_bit_cast(v8bf, make_uint4(l[0], l[1], l[2], l[3]));
}


// The render record as the compositing loops read it from LDS, 8 floats per Gaussian:
//   mx, my   mean2d relative to the tile's middle (the centre of its pixel (tw / 2, th / 2)),
//            so that a pixel's offset is its integer position relative to that pixel minus
//            (mx, my); a middle origin keeps |mx|, |my| (and their rounding) small for every
//            tile shape;
//   a, b, c  the conic scaled so that a dx^2 + b dx dy + c dy^2 is the exponent of eq. 4
//            in base 2: a = -A log2(e) / 2, b = -B log2(e), c = -C log2(e) / 2;
//   o        opacity (two floats of padding).
// The mean's hi + lo sum is rounded once, after the exact subtraction of the tile origin.
constexpr float kLog2e = 1.4426950408889634f;
struct LRec {
  float4 m;   // mx, my, a, b
  float2 c;   // c, o
};
// Stages half of a render record (part 0: mean hi, lo; part 1: conic, opacity).
__device__ __forceinline__ void stage_rec(float* s_rec, int q, const float4 r, int part, float ox, float oy) {
  float* d = s_rec + 8 * q;
  if (part == 0) {
    *reinterpret_cast<float2*>(d) = make_float2((r.x - ox) + r.z, (r.y - oy) + r.w);
  } else {
    *reinterpret_cast<float2*>(d + 2) = make_float2(-0.5f * kLog2e * r.x, -kLog2e * r.y);
    *reinterpret_cast<float2*>(d + 4) = make_float2(-0.5f * kLog2e * r.z, r.w);
  }
}
__device__ __forceinline__ LRec load_rec(const float* s_rec, int q) {
  LRec r;
  r.m = *reinterpret_cast<const float4*>(s_rec + 8 * q);
  r.c = *reinterpret_cast<const float2*>(s_rec + 8 * q + 4);
  return r;
}

// Base-2 footprint exponent at tile-local pixel (lx, ly), clamped at zero; dx, dy are the
// pixel's offsets from the mean and t = a dx + b dy.
__device__ __forceinline__ float local_power2(float lx, float ly, const LRec& r, float& dx, float& dy, float& t) {
  dx = lx - r.m.x;
  dy = ly - r.m.y;
  t = __builtin_fmaf(r.m.z, dx, r.m.w * dy);
  return fminf(__builtin_fmaf(t, dx, (r.c.x * dy) * dy), 0.0f);
}

// Whether the footprint can reach alpha_min anywhere in the rectangle [x0, x1] x [y0, y1]
// of tile-local positions (a wave's band of pixel centres): false only if the largest
// base-2 exponent over the continuous rectangle lies below log2(alpha_min / o) by a margin
// (0.1, far above the exponent's single-precision rounding), so a pixel of the band never
// takes the Gaussian. The exponent is concave; its maximum is 0 at the mean if the mean
// lies in the rectangle, else on an edge, at the edge's own vertex clamped to the edge.
// A degenerate record (a non-finite maximum) is never skipped.
__device__ __forceinline__ bool band_reaches(const LRec& r, float x0, float x1, float y0, float y1, float amin) {
  const float a = r.m.z, b = r.m.w, c = r.c.x;
  const float X0 = x0 - r.m.x, X1 = x1 - r.m.x, Y0 = y0 - r.m.y, Y1 = y1 - r.m.y;
  if (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) return true;
  // the vertices from approximate reciprocals: the exponent is flat there, so the value at
  // a slightly moved point differs from the maximum by far less than the margin
  const float ia = -0.5f * __builtin_amdgcn_rcpf(a), ic = -0.5f * __builtin_amdgcn_rcpf(c);
  auto along_x = [&](float Y) {   // dy = Y, dx over [X0, X1]
    const float dx = fminf(X1, fmaxf(X0, b * Y * ia));
    return (a * dx + b * Y) * dx + c * Y * Y;
  };
  auto along_y = [&](float X) {   // dx = X, dy over [Y0, Y1]
    const float dy = fminf(Y1, fmaxf(Y0, b * X * ic));
    return (c * dy + b * X) * dy + a * X * X;
  };
  const float m = fmaxf(fmaxf(along_x(Y0), along_x(Y1)), fmaxf(along_y(X0), along_y(X1)));
  return !(m < __log2f(amin) - __log2f(r.c.y) - 0.1f);
}

__device__ __forceinline__ v4f mma(v8bf a, v8bf b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
__device__ __forceinline__ v4f mma3(v8bf ah, v8bf al, v8bf bh, v8bf bl, v4f c) {
  c = mma(ah, bh, c);
  c = mma(ah, bl, c);
  c = mma(al, bh, c);
  return c;
}
// Six products of three-part operands: a b to about 2^-24 relative per product term.
__device__ __forceinline__ v4f mma6(const v8bf (&a)[3], const v8bf (&b)[3], v4f c) {
  c = mma(a[0], b[0], c);
  c = mma(a[0], b[1], c);
  c = mma(a[1], b[0], c);
  c = mma(a[0], b[2], c);
  c = mma(a[1], b[1], c);
  c = mma(a[2], b[0], c);
  return c;
}
__device__ __forceinline__ v4f zero4() { return (v4f){0.0f, 0.0f, 0.0f, 0.0f}; }

// The next (up to) four set bits of a wave-uniform mask, lowest first (-1 past the last).
__device__ __forceinline__ void pop4(uint32_t& m, int (&q)[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    q[e] = m ? __builtin_ctz(m) : -1;
    m &= m - 1u;
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Batch staging, double-buffered through registers: thread t stages Gaussian q = t / 8
// of the batch, channels [(t % 8) CPT, +CPT) of its features and, for t % 8 < 2, half of
// its 8-float record. The batch's Gaussian ids are loaded a batch earlier than its data
// (load_ids, then fetch_data), so that the gathers that depend on them issue without
// waiting for a load.
template <int NS>
struct SStage {
  static constexpr int CPT = SShape<NS>::CPT;
  float4 r;
  uint32_t gid, gpre;
  float f[CPT];

  __device__ __forceinline__ void load_ids(const uint32_t* __restrict__ vals, uint32_t b, int cnt) {
    const int q = threadIdx.x >> 3;
    gpre = q < cnt ? vals[b + q] : 0u;
  }
  __device__ __forceinline__ void fetch(const uint32_t* __restrict__ vals, uint32_t b, int cnt, int item, int64_t n,
                                        const float* __restrict__ rec, const float* __restrict__ depth,
                                        const float* __restrict__ rgb, const float* __restrict__ sem,
                                        const uint16_t* __restrict__ emb, int n_sem, int64_t foff) {
    load_ids(vals, b, cnt);
    fetch_data(cnt, item, n, rec, depth, rgb, sem, emb, n_sem, foff);
  }
  // gathers the data of the batch whose ids load_ids loaded (cnt Gaussians)
  __device__ __forceinline__ void fetch_data(int cnt, int item, int64_t n, const float* __restrict__ rec,
                                             const float* __restrict__ depth, const float* __restrict__ rgb,
                                             const float* __restrict__ sem, const uint16_t* __restrict__ emb,
                                             int n_sem, int64_t foff) {
    const int q = threadIdx.x >> 3, part = threadIdx.x & 7;
    const bool live = q < cnt;
    const uint32_t g = gpre;
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
        if (k < 3) v = rgb[3 * ((int64_t)g + foff) + k];
        else if (k == 3) v = depth[e];
        else if (emb) v = __uint_as_float((uint32_t)emb[(int64_t)n_sem * ((int64_t)g + foff) + (k - 4)] << 16);
        else v = sem[(int64_t)n_sem * ((int64_t)g + foff) + (k - 4)];
      }
      f[j] = v;
    }
  }
  // features Gaussian-major, single precision: s_f[q][c]; Gaussian ids to s_gid[q]
  __device__ __forceinline__ void commit_rows(float* s_rec, float* s_f, uint32_t* s_gid, float ox, float oy) const {
    const int q = threadIdx.x >> 3, part = threadIdx.x & 7;
    if (part < 2) stage_rec(s_rec, q, r, part, ox, oy);
    if (part == 0) s_gid[q] = gid;
    float* dst = s_f + q * SShape<NS>::FST + part * CPT;
#pragma unroll
    for (int j = 0; j < CPT; j += 4) *reinterpret_cast<float4*>(dst + j) = make_float4(f[j], f[j + 1], f[j + 2], f[j + 3]);
  }
  // features channel-major: s_f[c][q]
  __device__ __forceinline__ void commit_cols(float* s_rec, uint32_t* s_f, float ox, float oy) const {
    const int q = threadIdx.x >> 3, part = threadIdx.x & 7;
    if (part < 2) stage_rec(s_rec, q, r, part, ox, oy);
#pragma unroll
    for (int j = 0; j < CPT; ++j) s_f[(part * CPT + j) * kWs + q] = pack_hl(f[j]);
  }
};

// ------------------------------------------------------------------------- forward
// Long tile lists are cut into segments of seg_len(cfg) list positions. The reverse pass
// takes every segment as a work item of its own; the forward walks up to `chunk`
// consecutive segments of a list in one work item (one sequential transmittance chain),
// so that only lists longer than a chunk need a starting transmittance from a pre-pass.
// The forward state and the reverse pass's segment list are sized for the configured length
// (at most one segment per tile more than the duplicates over it); seg_len = 0 selects
// kSegDefault.
constexpr int kSegDefault = 1024;
__host__ __device__ inline int seg_len(const gs_config& cfg) { return cfg.seg_len > 0 ? cfg.seg_len : kSegDefault; }

// Segments per forward work item (cfg.fwd_chunk; 0 = the whole list).
__host__ __device__ inline int fwd_chunk(const gs_config& cfg) { return cfg.fwd_chunk > 0 ? cfg.fwd_chunk : 1 << 16; }

// Saved state of a forward that split its long lists, one slot per segment (a tile's
// slots are consecutive from tbase[tile]; the work list has an entry per slot):
//   P[slot][px]     at the first slot of a chunk: product of (1 - alpha) over the chunk's
//                   Gaussians with alpha >= alpha_min, the stop rule ignored
//                   (transmittance pre-pass; not for a list's last chunk);
//   Te[slot][px]    T at the segment's end, for pixels active in it;
//   info[slot][px]  1 + list position of the last blend in it (0 if none) | active at its
//                   start << 30 | stopped inside it << 31;
//   CS[slot][k][px] the segment's colour, then the sum of the colours of all later
//                   segments of the list, which the reverse pass turns into its starting
//                   sum of w (g . f) with one dot product.
struct FState {
  uint32_t* tcnt;    // [n_tiles] segments of the tile: 1 = whole list, no slot data
  uint32_t* tbase;   // [n_tiles] first slot of the tile
  float* P;
  float* Te;
  uint32_t* info;
  float* CS;
};
constexpr uint32_t kInfoActive = 1u << 30, kInfoStopped = 1u << 31, kInfoLast = kInfoActive - 1;

// Segments per tile: every tile is at least one item (it writes the tile's output).
__global__ __launch_bounds__(256) void k_fseg_count(const uint32_t* __restrict__ ranges, int n_tiles, int order,
                                                    uint32_t seg, uint32_t* __restrict__ cnt_ord) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const uint32_t len = ranges[2 * (int64_t)t + 1] - ranges[2 * (int64_t)t];
  cnt_ord[order ? t : n_tiles - 1 - t] = len <= seg ? 1u : (len + seg - 1) / seg;
}

// Transmittance pre-pass: P of every chunk of a list but the last. Persistent blocks
// take work items from ctl[2].
__global__ __launch_bounds__(256) void k_fwd_trans(gs_config cfg, const float* __restrict__ rec, int64_t n,
                                                   const gs_item* __restrict__ items, int n_items,
                                                   const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ ranges, const uint2* __restrict__ work,
                                                   uint32_t* __restrict__ ctl, float* __restrict__ P) {
  __shared__ __align__(16) float s_rec[8 * kB];
  __shared__ uint32_t s_wi;
  const int tid = threadIdx.x;
  const int tws = tile_shift(cfg);
  const float lx = (float)((tid & ((1 << tws) - 1)) - (1 << (tws - 1))), ly = (float)((tid >> tws) - (128 >> tws));
  const float amin = cfg.alpha_min, amax = cfg.alpha_max, tmin = cfg.t_min;
  const uint32_t n_work = ctl[0];
  for (;;) {
    if (tid == 0) s_wi = atomicAdd(&ctl[2], 1u);
    lds_barrier();
    const uint32_t wi = s_wi;
    lds_barrier();
    if (wi >= n_work) break;
    const uint2 wk = work[wi];
    const int seg = (int)(wk.y & 0xffffu), nseg = (int)(wk.y >> 16);
    const int chunk = fwd_chunk(cfg);
    if (seg % chunk != 0 || seg + chunk >= nseg) continue;
    const Ctx c = make_ctx_of(items, n_items, ranges, (int)wk.x, tws);
    int u, v;
    tile_pixel(c, tid, u, v);
    const bool inside = u < c.W && v < c.H;
    const float ox = (float)tile_mid_x(c) + 0.5f, oy = (float)tile_mid_y(c) + 0.5f;
    const int seglen = seg_len(cfg);
    const uint32_t a0 = c.start + seg * seglen;
    const uint32_t b0 = (uint32_t)min((int64_t)c.end, (int64_t)a0 + (int64_t)chunk * seglen);
    // thread t < 64 stages half (t % 2) of the record of Gaussian t / 2
    const int q = tid >> 1, part = tid & 1;
    auto fetch = [&](uint32_t b) -> float4 {
      if (tid >= 2 * kB || b + q >= b0) return make_float4(0.f, 0.f, 0.f, 0.f);
      const int64_t e = (int64_t)c.item * n + vals[b + q];
      return reinterpret_cast<const float4*>(rec + kRecFloats * e)[part];
    };
    float p = 1.0f;
    float4 r = fetch(a0);
    for (uint32_t b = a0; b < b0; b += kB) {
      // below t_min the product's exact value no longer matters
      if (__syncthreads_count(inside & (p >= tmin)) == 0) break;
      if (tid < 2 * kB) stage_rec(s_rec, q, r, part, ox, oy);
      lds_barrier();
      const int cnt = (int)min((uint32_t)kB, b0 - b);
      r = fetch(b + kB);
      // records of the next four Gaussians are read while the current four are used
      LRec R[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) R[e] = load_rec(s_rec, e);
#pragma unroll
      for (int k4 = 0; k4 < kB; k4 += 4) {
        LRec N[4];
        if (k4 + 4 < kB)
#pragma unroll
          for (int e = 0; e < 4; ++e) N[e] = load_rec(s_rec, k4 + 4 + e);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float dx, dy, t;
          const float araw = R[e].c.y * __builtin_amdgcn_exp2f(local_power2(lx, ly, R[e], dx, dy, t));
          const bool ok = (k4 + e < cnt) & (araw >= amin);
          p = ok ? p - fminf(amax, araw) * p : p;
        }
        if (k4 + 4 < kB)
#pragma unroll
          for (int e = 0; e < 4; ++e) R[e] = N[e];
      }
    }
    P[(int64_t)wi * kTilePx + tid] = p;
  }
}

// Compositing of one work item per block: a whole tile list (SEG = false, one block per
// tile) or, SEG = true, a chunk of up to cfg.fwd_chunk segments of a list taken by persistent
// blocks from ctl[1], starting from the product of the earlier chunks' P. A split list
// leaves each segment's colour, end T and blend record in its slot; when the list is one
// chunk, the block also joins its segments (image, T, n_contrib, suffix colours).
template <int NS, bool SEG>
__global__ __launch_bounds__(256, 3) void k_render_fwd_split(gs_config cfg, const float* __restrict__ rgb,
                                                          const float* __restrict__ sem,
                                                          const uint16_t* __restrict__ emb, int n_sem,
                                                          const float* __restrict__ rec,
                                                          const float* __restrict__ depth, int64_t n,
                                                          const gs_item* __restrict__ items, int n_items,
                                                          const uint32_t* __restrict__ vals,
                                                          const uint32_t* __restrict__ ranges, float* __restrict__ color,
                                                          float* __restrict__ Tout, uint32_t* __restrict__ ncout,
                                                          const uint2* __restrict__ work, uint32_t* __restrict__ ctl,
                                                          FState fs) {
  using S = SShape<NS>;
  constexpr int CB = S::CB, KP = S::KP;
  __shared__ __align__(16) float s_rec[8 * kB];
  __shared__ __align__(16) uint32_t s_f[KP * kWs];          // F^T, packed hi|lo, [channel][Gaussian]
  __shared__ __align__(16) float s_w[4][64 * kWs];          // per wave W, [pixel][Gaussian]
  __shared__ uint32_t s_wi;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int Kr = 4 + n_sem;
  const int tws = tile_shift(cfg);
  const float lx = (float)((tid & ((1 << tws) - 1)) - (1 << (tws - 1))), ly = (float)((tid >> tws) - (128 >> tws));
  const float amin = cfg.alpha_min, amax = cfg.alpha_max, tmin = cfg.t_min;
  const uint32_t n_work = SEG ? ctl[0] : 1u;
  float* W = s_w[wave];
  // this wave's band of tile-local pixel positions
  const float bx0 = (float)(-(1 << (tws - 1))), bx1 = (float)((1 << (tws - 1)) - 1);
  const float by0 = (float)(((64 * wave) >> tws) - (128 >> tws)), by1 = (float)(((64 * wave + 63) >> tws) - (128 >> tws));
  for (uint32_t round = 0;; ++round) {
    uint32_t wi = 0;
    int tile, seg = 0, nseg = 1;
    if constexpr (SEG) {
      if (tid == 0) s_wi = atomicAdd(&ctl[1], 1u);
      lds_barrier();
      wi = s_wi;
      lds_barrier();
      if (wi >= n_work) break;
      const uint2 wk = work[wi];
      tile = (int)wk.x;
      seg = (int)(wk.y & 0xffffu);
      nseg = (int)(wk.y >> 16);
      if (seg % fwd_chunk(cfg) != 0) continue;   // inside a chunk walked by another item
    } else {
      if (round > 0) break;
      tile = cfg.tile_order ? (int)blockIdx.x : (int)gridDim.x - 1 - (int)blockIdx.x;
    }
    const Ctx c = make_ctx_of(items, n_items, ranges, tile, tws);
    const int64_t foff = feature_offset(cfg, c.view, n);
    int u, v;
    tile_pixel(c, tid, u, v);
    const bool inside = u < c.W && v < c.H;
    const float ox = (float)tile_mid_x(c) + 0.5f, oy = (float)tile_mid_y(c) + 0.5f;
    const bool split = SEG && nseg > 1;
    const int chunk = fwd_chunk(cfg), seglen = seg_len(cfg);
    const int s_hi = split ? min(nseg, seg + chunk) : 1;   // segments [seg, s_hi) of this item
    const int64_t slot0 = (int64_t)wi - seg;                  // the tile's first slot
    v4f acc[CB][4];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int pb = 0; pb < 4; ++pb) acc[cb][pb] = zero4();
    float T = 1.0f;
    if (split)
      for (int s2 = 0; s2 < seg; s2 += chunk) T *= fs.P[(slot0 + s2) * kTilePx + tid];
    // a pixel whose transmittance in front of the chunk is below t_min stopped earlier
    bool done = !(inside & (T >= tmin));
    uint32_t last = 0;
    SStage<NS> st;
    for (int sg = seg; sg < s_hi; ++sg) {
      const uint32_t a0 = split ? c.start + sg * seglen : c.start;
      const uint32_t b0 = split ? min(c.end, a0 + seglen) : c.end;
      const bool active = !done;
      if (a0 < b0) {
        st.fetch(vals, a0, (int)min((uint32_t)kB, b0 - a0), c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
        if (a0 + kB < b0) st.load_ids(vals, a0 + kB, (int)min((uint32_t)kB, b0 - a0 - kB));
      }
      for (uint32_t b = a0; b < b0; b += kB) {
        // every wave is past the previous batch's LDS reads; stop once every pixel has
        if (__syncthreads_count(!done) == 0) break;
        st.commit_cols(s_rec, s_f, ox, oy);
        __syncthreads();
        const int cnt = (int)min((uint32_t)kB, b0 - b);
        if (b + kB < b0) {
          st.fetch_data((int)min((uint32_t)kB, b0 - b - kB), c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
          if (b + 2 * kB < b0) st.load_ids(vals, b + 2 * kB, (int)min((uint32_t)kB, b0 - b - 2 * kB));
        }
        // front-to-back recurrence, branch-free; only T carries from one Gaussian to the next.
        // A wave whose pixels have all stopped skips it (and the products), leaving its
        // SIMD's issue slots to the other waves there while the block's other waves go on.
        bool took = false;
        const uint32_t base = b - c.start;
        // with 32 channels, only the Gaussians that can reach a pixel of the wave's band;
        // with 64 (whose registers are full) every Gaussian of the batch
        if constexpr (KP <= 32) {
          if (__ballot(!done) != 0ull) {
            // the batch's Gaussians that can reach alpha_min somewhere in this wave's band of
            // pixels (lane q < 32 tests Gaussian q); the others take no pixel of the band
            bool hit = false;
            if (lane < kB && lane < cnt) hit = band_reaches(load_rec(s_rec, lane), bx0, bx1, by0, by1, amin);
            uint32_t m = (uint32_t)__ballot(hit);
            // their weights only; the rest of the row is zero
  #pragma unroll
            for (int q4 = 0; q4 < kB; q4 += 4)
              *reinterpret_cast<float4*>(W + lane * kWs + q4) = make_float4(0.f, 0.f, 0.f, 0.f);
            // four at a time in list order, the next four's records read while these are used
            // (two register sets taking turns)
            auto load4 = [&](const int (&q)[4], LRec (&R)[4]) {
  #pragma unroll
              for (int e = 0; e < 4; ++e) R[e] = load_rec(s_rec, q[e] < 0 ? 0 : q[e]);
            };
            auto run4 = [&](const int (&q)[4], const LRec (&R)[4]) {
  #pragma unroll
              for (int e = 0; e < 4; ++e) {
                if (q[e] < 0) break;   // uniform: the last group's missing entries
                float dx, dy, t;
                const float araw = R[e].c.y * __builtin_amdgcn_exp2f(local_power2(lx, ly, R[e], dx, dy, t));
                const bool ok = !done & (araw >= amin);
                const float w = fminf(amax, araw) * T;
                const float Tn = T - w;
                const bool stop = ok & (Tn < tmin);
                const bool take = ok & !stop;
                W[lane * kWs + q[e]] = take ? w : 0.0f;
                T = take ? Tn : T;
                done = done | stop;
                last = take ? base + q[e] + 1 : last;
                took |= take;
              }
            };
            int qa[4], qb[4];
            LRec RA[4], RB[4];
            pop4(m, qa);
            load4(qa, RA);
            for (;;) {
              if (qa[0] < 0) break;
              pop4(m, qb);
              if (qb[0] >= 0) load4(qb, RB);
              run4(qa, RA);
              if (qb[0] < 0) break;
              pop4(m, qa);
              if (qa[0] >= 0) load4(qa, RA);
              run4(qb, RB);
            }
          }
        } else {
          if (__ballot(!done) != 0ull) {
            // records of the next four Gaussians are read while the current four are used
            LRec R[4];
  #pragma unroll
            for (int e = 0; e < 4; ++e) R[e] = load_rec(s_rec, e);
  #pragma unroll
            for (int q4 = 0; q4 < kB; q4 += 4) {
              LRec N[4];
              if (q4 + 4 < kB)
  #pragma unroll
                for (int e = 0; e < 4; ++e) N[e] = load_rec(s_rec, q4 + 4 + e);
              __builtin_amdgcn_sched_barrier(0);
              float wq[4];
  #pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int q = q4 + e;
                float dx, dy, t;
                const float araw = R[e].c.y * __builtin_amdgcn_exp2f(local_power2(lx, ly, R[e], dx, dy, t));
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
              if (q4 + 4 < kB)
  #pragma unroll
                for (int e = 0; e < 4; ++e) R[e] = N[e];
            }
          }
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
      if (split) {
        // the segment's slot; D[c][p]: lane holds pixel 16 pb + l16 of this wave, channels
        // 16 cb + 4 g4 + r
        const int64_t sl = slot0 + sg;
        float* dst = fs.CS + sl * Kr * kTilePx + wave * 64 + l16;
#pragma unroll
        for (int pb = 0; pb < 4; ++pb)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ch = 16 * cb + 4 * g4 + r;
              if (ch < Kr) dst[ch * kTilePx + 16 * pb] = acc[cb][pb][r];
              acc[cb][pb][r] = 0.0f;
            }
        const int64_t o = sl * kTilePx + tid;
        fs.Te[o] = T;
        const uint32_t lseg = last > (uint32_t)(sg * seglen) ? last : 0u;
        fs.info[o] = lseg | (active ? kInfoActive : 0u) | ((active && done) ? kInfoStopped : 0u);
      }
    }
    if (split && nseg > chunk) continue;   // joined by k_fwd_combine
    const int64_t pix = c.pixel_base + (int64_t)v * c.W + u;
    if (inside) {
      Tout[pix] = T;
      ncout[pix] = last;
    }
    // D[c][p] (the image), or for a split list the sum of its segments' colours taken back
    // to front, each slot left holding the sum of the ones after it (acc, zero after the
    // last flush, carries the running sum; every value read here was written by this lane)
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) {
      if (split) {
        float* p = fs.CS + slot0 * Kr * kTilePx + wave * 64 + 16 * pb + l16;
        for (int s2 = nseg - 1; s2 >= 0; --s2) {
          float* ps = p + (int64_t)s2 * Kr * kTilePx;
          float cs[CB][4];
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ch = 16 * cb + 4 * g4 + r;
              cs[cb][r] = ch < Kr ? ps[ch * kTilePx] : 0.0f;
            }
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ch = 16 * cb + 4 * g4 + r;
              if (ch < Kr) ps[ch * kTilePx] = acc[cb][pb][r];
              acc[cb][pb][r] += cs[cb][r];
            }
        }
      }
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
  }
}

// Joins the segments of every list longer than one chunk: a pixel takes its segments in
// order up to the one in which it stopped (a later chunk that still found it active, its
// starting product being rounded differently from the stopping chain, is dropped); the
// image gets their colour sum, T and n_contrib, and each segment's colour is replaced by
// the sum of the colours of the kept segments after it. Segments are walked back to
// front with all channels of a segment loaded at once.
template <int NS>
__global__ __launch_bounds__(256) void k_fwd_combine(const gs_item* __restrict__ items, int n_items,
                                                     const uint32_t* __restrict__ ranges, int Kr, int chunk, int tws,
                                                     FState fs, float* __restrict__ color, float* __restrict__ Tout,
                                                     uint32_t* __restrict__ ncout) {
  constexpr int KP = SShape<NS>::KP;
  const int tile = blockIdx.x, tid = threadIdx.x;
  const int nseg = (int)fs.tcnt[tile];
  if (nseg <= chunk) return;
  const Ctx c = make_ctx_of(items, n_items, ranges, tile, tws);
  int u, v;
  tile_pixel(c, tid, u, v);
  if (u >= c.W || v >= c.H) return;
  const int64_t b = fs.tbase[tile];
  float T = 1.0f;
  uint32_t last = 0;
  int s_end = nseg;
  for (int s = 0; s < nseg; ++s) {
    const int64_t o = (b + s) * kTilePx + tid;
    const uint32_t inf = fs.info[o];
    if (!(inf & kInfoActive)) break;
    T = fs.Te[o];
    if (inf & kInfoLast) last = inf & kInfoLast;
    if (inf & kInfoStopped) {
      s_end = s + 1;
      break;
    }
  }
  const int64_t pix = c.pixel_base + (int64_t)v * c.W + u;
  Tout[pix] = T;
  ncout[pix] = last;
  float sum[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) sum[k] = 0.0f;
  for (int s = nseg - 1; s >= 0; --s) {
    float* p = fs.CS + (b + s) * Kr * kTilePx + tid;
    float cs[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) cs[k] = (k < Kr && s < s_end) ? p[k * kTilePx] : 0.0f;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      if (k < Kr) p[k * kTilePx] = sum[k];
      sum[k] += cs[k];
    }
  }
  float* out = color + c.pixel_base * Kr + (int64_t)v * c.W + u;
#pragma unroll
  for (int k = 0; k < KP; ++k)
    if (k < Kr) out[k * c.HW] = sum[k];
}

// ------------------------------------------------------------------------- backward
// Swaps the 4x4 blocks (lane row R, register group X[pb]) -> (lane row pb, group R):
// permlane32 exchanges rows 0,1 with 2,3, permlane16 rows 0 with 1 and 2 with 3.
template <int NK>
__device__ __forceinline__ void block_transpose(uint32_t (&X)[4][NK]) {
#pragma unroll
  for (int k = 0; k < NK; ++k) {
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

// Walking a segment of a split list backwards needs, per pixel, the transmittance after
// it and the suffix sum over every later Gaussian of w (g . f). Without the forward's
// saved state, a summary pass gives every segment s of a long list, per pixel,
//   P_s  = prod over its blended Gaussians of (1 - alpha)            (front to back)
//   GC_s = sum over its blended Gaussians of alpha T_loc (g . f),     T_loc from 1
// and then T_after(s) = prod_{s' <= s} P_s' and suffix(s) = sum_{s' > s} T_before(s') GC_s'.
// With the exponent E = a dx^2 + b dx dy + c dy^2 of the local record (E = log2(e) power),
// d power/d mean2d = -(dE/d dx, dE/d dy) / log2(e) and d power/d(A, B, C) =
// -(dx^2 / 2, dx dy, dy^2 / 2); the reverse pass sums dE/d dx, dE/d dy, dx^2, dx dy, dy^2
// (times dL/d power) and applies these factors once per Gaussian.
// Partial sums per (Gaussian, component) left in LDS by a batch: 4 per wave.
constexpr int kGeoSlots = 16;

// Sums the geometric terms of GG Gaussians (6 GG values per lane) over the wave's four
// lane rows and over the lane pairs (l16, l16 ^ 8) of a row, halving the values held at each
// step instead of reducing each value separately: a permlane32 swap pairs rows (0, 2) and
// (1, 3), a permlane16 swap rows (0, 1) and (2, 3), a row rotation by 8 the halves of a row.
// A last mirror within each half row pairs lanes i and 7 - i. Lane (row R, l16) returns
// Y[j] = sum of V[f + j] over the 16 lanes (l16 % 4, 7 - l16 % 4) + {0, 8}, times the four
// rows, with f = 6 R + 3 (l16 / 8) for GG = 4 and f = 3 R for GG = 2. Lanes with l16 % 8 < 4
// hold the distinct sums (for GG = 2 the two half rows hold the same ones).
template <int GG>
__device__ __forceinline__ void geo_reduce(const float (&V)[6 * GG], float (&Y)[3]) {
  constexpr int H1 = 3 * GG, H2 = 3 * GG / 2;
  float W[H1], X[H2];
#pragma unroll
  for (int j = 0; j < H1; ++j) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(V[j]), __float_as_uint(V[j + H1]), false, false);
    W[j] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
  }
#pragma unroll
  for (int j = 0; j < H2; ++j) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(W[j]), __float_as_uint(W[j + H2]), false, false);
    X[j] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
  }
  if constexpr (GG == 4) {
    const bool upper = (threadIdx.x & 8) != 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float keep = upper ? X[j + 3] : X[j], send = upper ? X[j] : X[j + 3];
      Y[j] = keep + dpp_ror8(send);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 3; ++j) Y[j] = X[j] + dpp_ror8(X[j]);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) Y[j] += dpp_half_mirror(Y[j]);
}

__constant__ float kGeoScale[6] = {-1.0f / kLog2e, -1.0f / kLog2e, -0.5f, -1.0f, -0.5f, 1.0f};

// One block per tile: the tile's list length in use (largest n_contrib) and its segment
// count, stored in work order (coarse pyramid levels first unless tile_order = 1).
// With a forward state, a tile that the forward did not split stays one item.
__global__ __launch_bounds__(256) void k_seg_count(const gs_item* __restrict__ items, int n_items,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ ncin, int n_tiles, int order, int tws,
                                                   uint32_t seg, const uint32_t* __restrict__ ftcnt,
                                                   uint32_t* __restrict__ tile_lmax, uint32_t* __restrict__ cnt_ord) {
  __shared__ uint32_t s_m;
  const int tile = blockIdx.x;
  const int item = item_of_tile(items, n_items, tile);
  const gs_item it = items[item];
  const int lt = tile - it.tile_base;
  const int u = ((lt % it.tiles_x) << tws) + (threadIdx.x & ((1 << tws) - 1));
  const int v = (lt / it.tiles_x) * (kTilePx >> tws) + (threadIdx.x >> tws);
  const uint32_t len = ranges[2 * (int64_t)tile + 1] - ranges[2 * (int64_t)tile];
  const uint32_t last = (u < it.W && v < it.H) ? min(ncin[it.pixel_base + (int64_t)v * it.W + u], len) : 0u;
  if (threadIdx.x == 0) s_m = 0;
  __syncthreads();
  atomicMax(&s_m, last);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t m = s_m;
    tile_lmax[tile] = m;
    const bool one = m <= seg || (ftcnt && ftcnt[tile] < 2);
    cnt_ord[order ? tile : n_tiles - 1 - tile] = m == 0 ? 0u : (one ? 1u : (m + seg - 1) / seg);
  }
}

// Work list: (tile, segment | segment count << 16). If the segments do not fit the
// workspace, every tile becomes a single item. Also resets the two work counters and,
// if tcnt is given, records per tile its item count and first item.
__global__ void k_seg_list(const uint32_t* __restrict__ cnt_ord, const uint32_t* __restrict__ base_ord,
                           const uint64_t* __restrict__ total, int n_tiles, int order, int64_t max_segs,
                           uint2* __restrict__ work, uint32_t* __restrict__ ctl, uint32_t* __restrict__ tcnt,
                           uint32_t* __restrict__ tbase) {
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
    if (tcnt) {
      tcnt[tile] = c;
      tbase[tile] = b;
    }
  } else {
    work[o] = make_uint2(tile, 1u << 16);
    if (tcnt) {
      tcnt[tile] = 1;
      tbase[tile] = o;
    }
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
                                                          float* __restrict__ segP, float* __restrict__ segGC,
                                                          FState fs) {
  using S = SShape<NS>;
  constexpr int KP = S::KP, CB = S::CB, FST = S::FST;
  constexpr int GG = NS > 28 ? 2 : 4;         // Gaussians per geometric-term reduction (register budget)
  __shared__ __align__(16) float s_rec[8 * kB];
  __shared__ __align__(16) float s_f[kB * FST];             // F, [Gaussian][channel]
  constexpr int DFS = KP + 4;                 // row stride of s_df: lane rows land on other banks
  // One pool for the batch loop's W (per wave, 16 Gaussians, [Gaussian][pixel]) and two
  // buffers each of dF ([Gaussian][channel]) and geometric partial sums
  // ([Gaussian][component][slot]): a batch's sums are flushed to global memory during the
  // next batch. At the start of a work item each wave stages its pixels' upstream gradient
  // in the pool instead (32 channels at a time, [channel][pixel], rows of kGst floats).
  constexpr int kWsz = 4 * 16 * kPs, kDsz = kB * DFS, kGsz = kB * 6 * kGeoSlots, kGst = 64 + 4;
  static_assert(4 * 32 * kGst <= kWsz + 2 * kDsz + 2 * kGsz, "staging fits the pool");
  __shared__ __align__(16) float s_pool[SUMMARY ? 1 : kWsz + 2 * kDsz + 2 * kGsz];
  __shared__ uint32_t s_wi;
  __shared__ uint32_t s_gid[2][kB];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int Kr = 4 + n_sem;
  const float amin = cfg.alpha_min, amax = cfg.alpha_max;
  const uint32_t n_work = ctl[0];
  // this wave's band of tile-local pixel positions
  const int tws0 = tile_shift(cfg);
  const float bx0 = (float)(-(1 << (tws0 - 1))), bx1 = (float)((1 << (tws0 - 1)) - 1);
  const float by0 = (float)(((64 * wave) >> tws0) - (128 >> tws0)), by1 = (float)(((64 * wave + 63) >> tws0) - (128 >> tws0));
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
    const Ctx c = make_ctx_of(items, n_items, ranges, tile, tile_shift(cfg));
    const int64_t foff = feature_offset(cfg, c.view, n);
    int u, v;
    tile_pixel(c, tid, u, v);
    const bool inside = u < c.W && v < c.H;
    const float lx = (float)((tid & ((1 << c.tws) - 1)) - (1 << (c.tws - 1))), ly = (float)((tid >> c.tws) - (128 >> c.tws));
    const float ox = (float)tile_mid_x(c) + 0.5f, oy = (float)tile_mid_y(c) + 0.5f;
    const int64_t pix = c.pixel_base + (int64_t)v * c.W + u;
    // n_contrib comes from the matching forward; clamp so that a mismatched call stays in range
    const uint32_t len = c.end - c.start;
    const uint32_t last = inside ? min(ncin[pix], len) : 0u;
    const int lmax = (int)tile_lmax[tile];
    const int seglen = seg_len(cfg);
    const int a0 = nseg == 1 ? 0 : seg * seglen;
    const int b0 = nseg == 1 ? lmax : min(lmax, a0 + seglen);

    // upstream gradient of a wave pixel (0..63) and channel, zero outside the image
    auto gval = [&](int wp, int ch) -> float {
      int pu, pv;
      tile_pixel(c, wave * 64 + wp, pu, pv);
      if (pu >= c.W || pv >= c.H || ch >= Kr) return 0.0f;
      return gcolor[c.pixel_base * Kr + (int64_t)pv * c.W + pu + ch * c.HW];
    };
    // G^T as B of GF (k = channel 4 ks + g4, j = pixel 16 pb + l16); with 32 padded channels
    // the main pass takes GF on bfloat16 matrix cores instead, each operand in three parts
    // (single-precision products at a sixth of the 16x16x4 products' matrix-core time):
    // g3[part][pb], B of 16x16x32 (k = channel 8 g4 + e, j = pixel 16 pb + l16)
    constexpr bool kGF3 = !SUMMARY && KP == 32;
    float g1[4][kGF3 ? 1 : KP / 4];
    v8bf g3[kGF3 ? 4 : 1][3];
    if constexpr (SUMMARY) {
#pragma unroll
      for (int pb = 0; pb < 4; ++pb)
#pragma unroll
        for (int ks = 0; ks < KP / 4; ++ks) g1[pb][ks] = gval(16 * pb + l16, 4 * ks + g4);
    }
    // G as B of dF (k = pixel 32 ks + 8 g4 + e, j = channel 16 cb + l16). Main pass: each
    // wave stages its 64 pixels' upstream gradient, 32 channels at a time, with one
    // coalesced load per channel and lane, and builds both operand layouts from LDS; the
    // lane's own pixel's values also give the state's dot product.
    v8bf g2h[2][SUMMARY ? 1 : CB], g2l[2][SUMMARY ? 1 : CB];
    float gdot = 0.0f;          // sum_k g_k S_k of the lane's pixel (forward state)
    if constexpr (!SUMMARY) {
      const bool use_state = nseg > 1 && fs.tcnt != nullptr && inside;
      const float* sc = use_state ? fs.CS + ((int64_t)fs.tbase[tile] + seg) * Kr * kTilePx + tid : nullptr;
      const float* gp = gcolor + c.pixel_base * Kr + (int64_t)v * c.W + u;   // this lane's pixel (tid)
      float* stg = s_pool + wave * 32 * kGst;
#pragma unroll
      for (int h = 0; h < KP / 32; ++h) {
        float gl[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) gl[j] = (inside && 32 * h + j < Kr) ? gp[(int64_t)(32 * h + j) * c.HW] : 0.0f;
        if (use_state) {
          // all 32 loads in flight where the registers allow it, else 8 at a time
          constexpr int kSv = KP <= 32 ? 32 : 8;
#pragma unroll
          for (int j0 = 0; j0 < 32; j0 += kSv) {
            float sv[kSv];
#pragma unroll
            for (int j = 0; j < kSv; ++j) sv[j] = 32 * h + j0 + j < Kr ? sc[(32 * h + j0 + j) * kTilePx] : 0.0f;
#pragma unroll
            for (int j = 0; j < kSv; ++j) gdot = __builtin_fmaf(gl[j0 + j], sv[j], gdot);
          }
        }
#pragma unroll
        for (int j = 0; j < 32; ++j) stg[j * kGst + lane] = gl[j];
        wave_sync();
        if constexpr (kGF3) {
#pragma unroll
          for (int pb = 0; pb < 4; ++pb) {
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = stg[(8 * g4 + e) * kGst + 16 * pb + l16];
            split8x3(x, g3[pb][0], g3[pb][1], g3[pb][2]);
          }
        } else {
#pragma unroll
          for (int ks = 8 * h; ks < 8 * h + 8; ++ks)
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) g1[pb][ks] = stg[(4 * ks + g4 - 32 * h) * kGst + 16 * pb + l16];
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
          for (int cb = 2 * h; cb < 2 * h + 2; ++cb) {
            const float* src = stg + (16 * cb + l16 - 32 * h) * kGst + 32 * ks + 8 * g4;
            const float4 x0 = *reinterpret_cast<const float4*>(src), x1 = *reinterpret_cast<const float4*>(src + 4);
            const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
            split8(x, g2h[ks][cb], g2l[ks][cb]);
          }
        wave_sync();   // every lane has read the stage before the next half overwrites it
      }
    }

    // per-pixel state at the segment's back end (main pass) or front end (summary pass)
    float T = 1.0f, acc = 0.0f;   // acc: suffix (main) or GC (summary)
    if constexpr (!SUMMARY) {
      const float tf = inside ? Tfin[pix] : 1.0f;
      if (nseg == 1 || seg == nseg - 1) T = tf;
      if (nseg > 1 && fs.tcnt) {
        // the forward's state: T at the segment's end and the suffix colour sum
        const int64_t slot = (int64_t)fs.tbase[tile] + seg, o = slot * kTilePx + tid;
        if (fs.info[o] & kInfoActive) T = fs.Te[o];
        acc = gdot;
      } else if (nseg > 1) {
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
    const int n_batches = (b0 - a0 + kB - 1) / kB;
    // list range [lo, hi) of batch bi: the main pass from the back, the summary pass from the front
    auto batch_lo = [&](int bi) { return SUMMARY ? a0 + bi * kB : max(a0, b0 - (bi + 1) * kB); };
    auto batch_hi = [&](int bi) { return SUMMARY ? min(b0, a0 + (bi + 1) * kB) : b0 - bi * kB; };
    if (n_batches > 0) {
      st.fetch(vals, c.start + batch_lo(0), batch_hi(0) - batch_lo(0), c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
      if (n_batches > 1) st.load_ids(vals, c.start + batch_lo(1), batch_hi(1) - batch_lo(1));
    }
    // one FP32 atomic per (Gaussian, channel) and (Gaussian, component) of a finished batch
    auto flush = [&](int fb, int fcnt) {
      const float* fdf = s_pool + kWsz + fb * kDsz;
      const float* fgeo = s_pool + kWsz + 2 * kDsz + fb * kGsz;
      const uint32_t* fgid = s_gid[fb];
      if constexpr (KP <= 32) {
        // feature gradients: Gaussian q = idx / KP, channel k = idx % KP, all LDS reads first
        constexpr int kFl = kB * KP / 256;
        float fv[kFl];
        uint32_t fg[kFl];
#pragma unroll
        for (int j = 0; j < kFl; ++j) {
          const int idx = tid + 256 * j, q = idx / KP;
          fv[j] = fdf[q * DFS + (idx - q * KP)];
          fg[j] = fgid[q];
        }
#pragma unroll
        for (int j = 0; j < kFl; ++j) {
          const int idx = tid + 256 * j, q = idx / KP, k = idx - q * KP;
          const float val = fv[j];
          if (q >= fcnt || val == 0.0f || k >= Kr) continue;
          const uint32_t g = fg[j];
          if (k < 3) atomicAdd(&grgb[3 * ((int64_t)g + foff) + k], val);
          else if (k == 3) atomicAdd(&g2d[8 * ((int64_t)c.item * n + g) + 6], val);
          else atomicAdd(&gsem[(int64_t)n_sem * ((int64_t)g + foff) + (k - 4)], val);
        }
      } else {
        // (a register budget without room for the unrolled form)
        for (int idx = tid; idx < fcnt * KP; idx += 256) {
          const int q = idx / KP, k = idx - q * KP;
          const float val = fdf[q * DFS + k];
          if (val == 0.0f || k >= Kr) continue;
          const uint32_t g = fgid[q];
          if (k < 3) atomicAdd(&grgb[3 * ((int64_t)g + foff) + k], val);
          else if (k == 3) atomicAdd(&g2d[8 * ((int64_t)c.item * n + g) + 6], val);
          else atomicAdd(&gsem[(int64_t)n_sem * ((int64_t)g + foff) + (k - 4)], val);
        }
      }
      for (int idx = tid; idx < fcnt * 6; idx += 256) {
        const int q = idx / 6, comp = idx - q * 6;
        const float4* src = reinterpret_cast<const float4*>(fgeo + idx * kGeoSlots);
        float sum = 0.0f;
#pragma unroll
        for (int r = 0; r < kGeoSlots / 4; ++r) {
          const float4 x = src[r];
          sum += (x.x + x.y) + (x.z + x.w);
        }
        if (sum != 0.0f) {
          const uint32_t g = fgid[q];
          atomicAdd(&g2d[8 * ((int64_t)c.item * n + g) + comp], sum * kGeoScale[comp]);
        }
      }
    };
    int prev_cnt = 0;
    for (int bi = 0; bi < n_batches; ++bi) {
      const int lo = batch_lo(bi), hi = batch_hi(bi);
      const int cnt = hi - lo;
      const int buf = bi & 1;
      float* const s_df = s_pool + kWsz + buf * kDsz;
      float* const s_geo = s_pool + kWsz + 2 * kDsz + buf * kGsz;
      lds_barrier();
      st.commit_rows(s_rec, s_f, s_gid[buf], ox, oy);
      if constexpr (!SUMMARY) {
        for (int i = tid; i < kB * DFS; i += 256) s_df[i] = 0.0f;
        for (int i = tid; i < kB * 6 * kGeoSlots / 4; i += 256) reinterpret_cast<float4*>(s_geo)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      lds_barrier();
      // every wave is done with the previous batch: its sums go out while this one runs
      if constexpr (!SUMMARY)
        if (bi > 0) flush(buf ^ 1, prev_cnt);
      prev_cnt = cnt;
      // the next batch's gather: the summary pass issues it here; the main pass after its
      // recurrence, whose register peak it would otherwise add to
      auto fetch_next = [&]() {
        if (bi + 1 < n_batches) {
          st.fetch_data(batch_hi(bi + 1) - batch_lo(bi + 1), c.item, n, rec, depth, rgb, sem, emb, n_sem, foff);
          if (bi + 2 < n_batches) st.load_ids(vals, c.start + batch_lo(bi + 2), batch_hi(bi + 2) - batch_lo(bi + 2));
        }
      };
      if constexpr (SUMMARY) fetch_next();
      const bool wave_live = __ballot((uint32_t)lo < last) != 0ull;
      // the batch's Gaussians that can reach alpha_min in this wave's band of pixels (lane
      // q < 32 tests Gaussian q)
      uint32_t bmask = 0xffffffffu;
      if constexpr (!SUMMARY) {
        bool hit = false;
        if (wave_live && lane < kB && lane < cnt) hit = band_reaches(load_rec(s_rec, lane), bx0, bx1, by0, by1, amin);
        bmask = (uint32_t)__ballot(hit);
      }
      if (!SUMMARY && !wave_live) fetch_next();
      if (wave_live) {
        // GF^T[i][p] in single precision (it decides dL/dalpha, where terms cancel):
        // v_mfma_f32_16x16x4f32, A = F (i = Gaussian 16 bq + l16, k = channel 4 ks + g4), B = G^T
        uint32_t X[4][8];
        if constexpr (SUMMARY) {
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
        if constexpr (SUMMARY) block_transpose(X);
        if constexpr (SUMMARY) {
#pragma unroll
          for (int q = 0; q < kB; ++q) {
            const LRec rq = load_rec(s_rec, q);
            float dx, dy, t;
            const float araw = rq.c.y * __builtin_amdgcn_exp2f(local_power2(lx, ly, rq, dx, dy, t));
            const bool act = (q < cnt) & ((uint32_t)(lo + q) < last) & (araw >= amin);
            const float w = fminf(amax, araw) * T;
            const float gf = __uint_as_float(X[(q >> 2) & 3][4 * (q >> 4) + (q & 3)]);
            acc = act ? __builtin_fmaf(w, gf, acc) : acc;
            T = act ? T - w : T;
          }
        } else {
          // reverse recurrence, one 16-Gaussian block at a time (back to front), each with
          // its own GF^T block: Y[g][r] = gf of Gaussian 16 bq + 4 g + r after the transpose
#pragma unroll
          for (int bq = 1; bq >= 0; --bq) {
            uint32_t Y4[4][4];
            {
              v4f gfa[4];
#pragma unroll
              for (int pb = 0; pb < 4; ++pb) gfa[pb] = zero4();
              if constexpr (kGF3) {
                // A = F (i = Gaussian 16 bq + l16, k = channel 8 g4 + e)
                const float* src = s_f + (16 * bq + l16) * FST + 8 * g4;
                const float4 f0 = *reinterpret_cast<const float4*>(src), f1 = *reinterpret_cast<const float4*>(src + 4);
                const float x[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
                v8bf fa[3];
                split8x3(x, fa[0], fa[1], fa[2]);
#pragma unroll
                for (int pb = 0; pb < 4; ++pb) gfa[pb] = mma6(fa, g3[pb], gfa[pb]);
              } else {
#pragma unroll
                for (int ks = 0; ks < KP / 4; ++ks) {
                  const float a = s_f[(16 * bq + l16) * FST + 4 * ks + g4];
#pragma unroll
                  for (int pb = 0; pb < 4; ++pb)
                    gfa[pb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, g1[pb][ks], gfa[pb], 0, 0, 0);
                }
              }
#pragma unroll
              for (int pb = 0; pb < 4; ++pb)
#pragma unroll
                for (int r = 0; r < 4; ++r) Y4[pb][r] = __float_as_uint(gfa[pb][r]);
            }
            block_transpose(Y4);
            float* Wp = s_pool + wave * 16 * kPs;
            bool any = false;
#pragma unroll
            for (int gb = 16 / GG - 1; gb >= 0; --gb) {
              // a group none of whose Gaussians can reach the wave's band takes no pixel of it
              if (((bmask >> (16 * bq + GG * gb)) & ((1u << GG) - 1u)) == 0u) {
#pragma unroll
                for (int r = 0; r < GG; ++r) Wp[(GG * gb + r) * kPs + lane] = 0.0f;
                continue;
              }
              float V[6 * GG];   // V[6 r + k]: component k of the geometric terms of Gaussian GG gb + r
              bool gact = false;
#pragma unroll
              for (int r = GG - 1; r >= 0; --r) {
                const int qq = GG * gb + r, q = 16 * bq + qq;
                const LRec rq = load_rec(s_rec, q);
                float dx, dy, t;
                const float G = __builtin_amdgcn_exp2f(local_power2(lx, ly, rq, dx, dy, t));
                const float araw = rq.c.y * G;
                const bool act = (q < cnt) & ((uint32_t)(lo + q) < last) & (araw >= amin);
                const float a = fminf(amax, araw);
                const float rom = __builtin_amdgcn_rcpf(1.0f - a);
                const float Tq = act ? T * rom : T;   // transmittance in front of this Gaussian
                const float w = act ? a * Tq : 0.0f;
                const float gf = __uint_as_float(Y4[qq >> 2][qq & 3]);
                const float dalpha = Tq * gf - acc * rom;
                acc = act ? __builtin_fmaf(gf, w, acc) : acc;
                T = Tq;
                const bool unclamped = act & (araw < amax);
                const float dpow = unclamped ? dalpha * araw : 0.0f;
                const float dop = unclamped ? dalpha * G : 0.0f;
                Wp[qq * kPs + lane] = w;
                gact |= act;
                // d power / d (mean2d, A, B, C) up to the per-component factors of kGeoScale
                const float pdx = dpow * dx, pdy = dpow * dy;
                V[6 * r + 0] = dpow * __builtin_fmaf(rq.m.z, dx, t);   // 2a dx + b dy
                V[6 * r + 1] = dpow * __builtin_fmaf(rq.m.w, dx, 2.0f * (rq.c.x * dy));
                V[6 * r + 2] = pdx * dx;
                V[6 * r + 3] = pdx * dy;
                V[6 * r + 4] = pdy * dy;
                V[6 * r + 5] = dop;                                  // d/d opacity
              }
              if (__ballot(gact) != 0ull) {
                any = true;
                float Y[3];
                geo_reduce<GG>(V, Y);
                // Gaussian and first component of this lane's three sums
                const int qd = 16 * bq + GG * gb + (GG == 4 ? g4 : g4 >> 1);
                const int k0 = GG == 4 ? 3 * (l16 >> 3) : 3 * (g4 & 1);
                float* dst = s_geo + (qd * 6 + k0) * kGeoSlots + wave * 4 + (l16 & 3);
                if ((l16 & 4) == 0 && (GG == 4 || l16 < 8))
#pragma unroll
                  for (int j = 0; j < 3; ++j) dst[j * kGeoSlots] = Y[j];
              }
            }
            if (bq == 0) fetch_next();
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
                  if (d[r] != 0.0f) atomicAdd(&s_df[(16 * bq + 4 * g4 + r) * DFS + 16 * cb + l16], d[r]);
              }
            }
            wave_sync();   // the block's W is consumed before the next block overwrites it
          }
        }
      }
    }
    // the work item's last batch
    if constexpr (!SUMMARY) {
      if (n_batches > 0) {
        lds_barrier();
        flush((n_batches - 1) & 1, prev_cnt);
      }
    }
    if constexpr (SUMMARY) {
      segP[(int64_t)wi * kTilePx + tid] = T;
      segGC[(int64_t)wi * kTilePx + tid] = acc;
    }
  }
}

// Caller workspace of the reverse pass: the segment work list, sized for `cap` duplicates in
// segments of `seg` list positions (at most one more segment per tile than cap / seg).
struct SegWs {
  uint32_t *lmax, *cnt, *base, *partial, *ctl;
  uint64_t* total;
  uint2* work;
  float *P, *GC;
  int64_t max_segs;
};

size_t seg_layout(int n_tiles, int64_t cap, int seg, char* base, SegWs* w) {
  const int64_t max_segs = (int64_t)n_tiles + ceil_div(cap, seg) + 1;
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

// Caller buffer of a splitting forward (its saved state), sized for `cap` duplicates, K
// channels and segments of `seg` list positions.
struct FLayout {
  FState fs;
  uint32_t *cnt, *base, *partial, *ctl;
  uint64_t* total;
  uint2* work;
  int64_t max_segs;
};

size_t fstate_layout(int n_tiles, int64_t cap, int K, int seg, char* base, FLayout* w) {
  const int64_t max_segs = (int64_t)n_tiles + ceil_div(cap, seg) + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return base ? base + o : nullptr;
  };
  char* p_tcnt = take(4 * (size_t)n_tiles);
  char* p_tbase = take(4 * (size_t)n_tiles);
  char* p_cnt = take(4 * (size_t)n_tiles);
  char* p_base = take(4 * (size_t)n_tiles);
  char* p_part = take(4 * (size_t)scan_partials_needed(n_tiles));
  char* p_tot = take(8);
  char* p_ctl = take(16);
  char* p_work = take(8 * (size_t)max_segs);
  char* p_P = take(4 * (size_t)kTilePx * max_segs);
  char* p_Te = take(4 * (size_t)kTilePx * max_segs);
  char* p_info = take(4 * (size_t)kTilePx * max_segs);
  char* p_CS = take(4 * (size_t)kTilePx * max_segs * (size_t)K);
  if (w) {
    w->fs.tcnt = (uint32_t*)p_tcnt;
    w->fs.tbase = (uint32_t*)p_tbase;
    w->fs.P = (float*)p_P;
    w->fs.Te = (float*)p_Te;
    w->fs.info = (uint32_t*)p_info;
    w->fs.CS = (float*)p_CS;
    w->cnt = (uint32_t*)p_cnt;
    w->base = (uint32_t*)p_base;
    w->partial = (uint32_t*)p_part;
    w->total = (uint64_t*)p_tot;
    w->ctl = (uint32_t*)p_ctl;
    w->work = (uint2*)p_work;
    w->max_segs = max_segs;
  }
  return off;
}

}  // namespace

int render_seg_len(const gs_config& cfg) { return seg_len(cfg); }

size_t render_state_bytes(int n_tiles, int64_t dup_capacity, int K, int seg) {
  return fstate_layout(n_tiles, std::max<int64_t>(dup_capacity, 0), K, seg, nullptr, nullptr);
}

// Largest duplicate capacity whose forward state fits in `bytes` (-1 if none does).
int64_t render_state_capacity(int n_tiles, int K, int seg, size_t bytes) {
  if (render_state_bytes(n_tiles, 0, K, seg) > bytes) return -1;
  int64_t lo = 0, hi = 1;
  while (hi < ((int64_t)1 << 40) && render_state_bytes(n_tiles, hi, K, seg) <= bytes) hi *= 2;
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (render_state_bytes(n_tiles, mid, K, seg) <= bytes) lo = mid; else hi = mid;
  }
  return lo;
}

namespace {

// Forward state of images `im` (fs.tcnt == nullptr if there is none).
FLayout state_of(const gs_images& im, int n_tiles, int K, int seg) {
  FLayout w{};
  if (!im.state) return w;
  const int64_t cap = render_state_capacity(n_tiles, K, seg, im.state_bytes);
  if (cap >= 0) fstate_layout(n_tiles, cap, K, seg, (char*)im.state, &w);
  return w;
}

template <int NS>
int launch_fwd_s(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items, int n_items,
                 int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& out, hipStream_t s) {
  const FLayout w = state_of(out, n_tiles, 4 + cfg.n_sem, seg_len(cfg));
  if (!w.fs.tcnt) {
    hipLaunchKernelGGL((k_render_fwd_split<NS, false>), dim3(n_tiles), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb,
                       cfg.n_sem, p.rec, p.depth, g.n, items, n_items, vals, ranges, out.color, out.T, out.n_contrib,
                       nullptr, nullptr, w.fs);
    return launch_status();
  }
  const unsigned tb = (unsigned)ceil_div(n_tiles, 256);
  hipLaunchKernelGGL(k_fseg_count, dim3(tb), dim3(256), 0, s, ranges, n_tiles, cfg.tile_order,
                     (uint32_t)seg_len(cfg), w.cnt);
  int st = launch_status();
  st = st ? st : scan_u32(w.cnt, w.base, n_tiles, w.partial, w.total, s);
  if (st) return st;
  hipLaunchKernelGGL(k_seg_list, dim3(tb), dim3(256), 0, s, w.cnt, w.base, w.total, n_tiles, cfg.tile_order,
                     w.max_segs, w.work, w.ctl, w.fs.tcnt, w.fs.tbase);
  const int grid_t = resident_blocks(k_fwd_trans, 256, 0);
  const int grid_f = resident_blocks(k_render_fwd_split<NS, true>, 256, 0);
  if (!grid_t || !grid_f) return GS_ERR_HIP;
  if (cfg.fwd_chunk > 0)
    hipLaunchKernelGGL(k_fwd_trans, dim3(grid_t), dim3(256), 0, s, cfg, p.rec, g.n, items, n_items, vals, ranges,
                       w.work, w.ctl, w.fs.P);
  hipLaunchKernelGGL((k_render_fwd_split<NS, true>), dim3(grid_f), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb, cfg.n_sem,
                     p.rec, p.depth, g.n, items, n_items, vals, ranges, out.color, out.T, out.n_contrib, w.work, w.ctl,
                     w.fs);
  if (cfg.fwd_chunk > 0)
    hipLaunchKernelGGL(k_fwd_combine<NS>, dim3(n_tiles), dim3(256), 0, s, items, n_items, ranges, 4 + cfg.n_sem,
                       cfg.fwd_chunk, tile_shift(cfg), w.fs, out.color, out.T, out.n_contrib);
  return launch_status();
}

template <int NS>
int launch_bwd_s(const gs_config& cfg, const gs_gaussians& g, const gs_projected& p, const gs_item* items, int n_items,
                 int n_tiles, const uint32_t* vals, const uint32_t* ranges, const gs_images& fwd,
                 const gs_images& gin, float* g2d, const gs_grads& gr, void* seg_ws, int64_t cap, hipStream_t s) {
  SegWs w;
  seg_layout(n_tiles, cap, seg_len(cfg), (char*)seg_ws, &w);
  // with the forward's saved state the segments start from it: no summary pass
  const FState fs = state_of(fwd, n_tiles, 4 + cfg.n_sem, seg_len(cfg)).fs;
  hipLaunchKernelGGL(k_seg_count, dim3(n_tiles), dim3(256), 0, s, items, n_items, ranges, fwd.n_contrib, n_tiles,
                     cfg.tile_order, tile_shift(cfg), (uint32_t)seg_len(cfg), fs.tcnt, w.lmax, w.cnt);
  int st = launch_status();
  st = st ? st : scan_u32(w.cnt, w.base, n_tiles, w.partial, w.total, s);
  if (st) return st;
  hipLaunchKernelGGL(k_seg_list, dim3((unsigned)ceil_div(n_tiles, 256)), dim3(256), 0, s, w.cnt, w.base, w.total,
                     n_tiles, cfg.tile_order, w.max_segs, w.work, w.ctl, nullptr, nullptr);
  const int grid_sum = resident_blocks(k_render_bwd_split<NS, true>, 256, 0);
  const int grid_main = resident_blocks(k_render_bwd_split<NS, false>, 256, 0);
  if (!grid_sum || !grid_main) return GS_ERR_HIP;
  if (!fs.tcnt)
    hipLaunchKernelGGL((k_render_bwd_split<NS, true>), dim3(grid_sum), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb,
                       cfg.n_sem, p.rec, p.depth, g.n, items, n_items, vals, ranges, fwd.T, fwd.n_contrib, gin.color,
                       g2d, gr.rgb, gr.sem, w.work, w.ctl, w.lmax, w.P, w.GC, fs);
  hipLaunchKernelGGL((k_render_bwd_split<NS, false>), dim3(grid_main), dim3(256), 0, s, cfg, g.rgb, g.sem, g.emb,
                     cfg.n_sem, p.rec, p.depth, g.n, items, n_items, vals, ranges, fwd.T, fwd.n_contrib, gin.color, g2d,
                     gr.rgb, gr.sem, w.work, w.ctl, w.lmax, w.P, w.GC, fs);
  return launch_status();
}

}  // namespace

size_t render_seg_workspace(int n_tiles, int64_t dup_capacity, int seg) {
  return seg_layout(n_tiles, std::max<int64_t>(dup_capacity, 0), seg, nullptr, nullptr);
}

// Largest duplicate capacity whose segment workspace fits in `bytes` (-1 if none does).
int64_t render_seg_capacity(int n_tiles, int seg, size_t bytes) {
  if (render_seg_workspace(n_tiles, 0, seg) > bytes) return -1;
  int64_t lo = 0, hi = 1;
  while (hi < ((int64_t)1 << 40) && render_seg_workspace(n_tiles, hi, seg) <= bytes) hi *= 2;
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (render_seg_workspace(n_tiles, mid, seg) <= bytes) lo = mid; else hi = mid;
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
