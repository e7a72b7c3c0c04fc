// Tile binning and depth ordering of the footprints (the sorted set N of eq. 7-9).
//
// The required order is (global tile, float32 depth, Gaussian index). Instead of
// radix-sorting every duplicate by a 64-bit (tile | depth) key, this path
//   1. compacts the visible (item, Gaussian) entries and radix-sorts them by
//      (item, depth) -- a stable sort, so equal depths keep index order;
//   2. emits each entry's tiles in that order;
//   3. stably radix-sorts the duplicates by tile id alone.
// A stable sort by tile of a sequence already ordered by (depth, index) yields
// exactly the (tile, depth, index) order, with ceil(log2(tiles)) key bits per
// duplicate instead of 32 + ceil(log2(tiles)).
//
// Every kernel reads its element count from device memory, so the sequence has no
// host synchronisation and can be captured in a graph; grids are sized for the
// capacity and blocks past the live count exit early.
#include "common.h"

#include <algorithm>
#include <cmath>

namespace gs {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;   // 4096
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kRadixThreads * kRadixItems;  // 2048
constexpr int kRadixWaveSpan = kRadixTile / 4;            // keys per wave
// Digits of 8 to 11 bits: a sort of b-bit keys takes ceil(b / 11) passes of equal width
// (the (item, depth) keys of the visible entries have 31 + log2(items) bits, the
// duplicates' tile ids log2(tiles)).
constexpr int kDigitMax = 11;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of uint32 (three phases), count from device memory.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t& total, uint32_t* sh /*[4]*/) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wid; ++w) base += sh[w];
  total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return base + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, const uint64_t* count_dev,
                                                               int64_t count_host, uint32_t* __restrict__ partial) {
  const int64_t count = count_dev ? (int64_t)*count_dev : count_host;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  if (base < count) {
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t idx = base + (int64_t)k * kScanThreads + threadIdx.x;
      if (idx < count) s += in[idx];
    }
  }
  __shared__ uint32_t sh[4];
  uint32_t total;
  block_exclusive_scan(s, total, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Single block: exclusive scan of the block partials; total to *total_out (uint64).
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* partial, int64_t n_partial_cap, const uint64_t* count_dev,
                                                        int64_t count_host, uint64_t* total_out) {
  const int64_t count = count_dev ? (int64_t)*count_dev : count_host;
  const int64_t np = min(n_partial_cap, (count + kScanTile - 1) / kScanTile);
  __shared__ uint64_t sh[1024];
  const int t = threadIdx.x;
  const int64_t per = (np + 1023) / 1024;
  const int64_t b0 = t * per, b1 = min(np, b0 + per);
  uint64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += partial[b];
  sh[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint64_t v = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  uint64_t run = sh[t] - s;
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t v = partial[b];
    partial[b] = (uint32_t)run;
    run += v;
  }
  if (t == 1023 && total_out) *total_out = sh[1023];
}

// in and out may be the same array (in-place scans): each thread reads its elements
// before it writes them, and no other thread touches them.
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const uint32_t* in, const uint64_t* count_dev,
                                                              int64_t count_host, const uint32_t* __restrict__ partial,
                                                              uint32_t* out) {
  const int64_t count = count_dev ? (int64_t)*count_dev : count_host;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= count) return;
  // blocked arrangement: thread t owns kScanItems consecutive elements
  uint32_t v[kScanItems];
  uint32_t s = 0;
  const int64_t tb = base + (int64_t)threadIdx.x * kScanItems;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = tb + k;
    v[k] = idx < count ? in[idx] : 0;
    s += v[k];
  }
  __shared__ uint32_t sh[4];
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, total, sh) + partial[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = tb + k;
    if (idx < count) out[idx] = run;
    run += v[k];
  }
}

// Two-kernel form for inputs of up to kDirectTiles tiles: each apply block sums the tile
// totals before it itself (at most kDirectTiles loads over 256 threads), so the single-block
// scan of the partials between the two passes, a launch bound by latency, is not needed.
// Block 0 also sums all of them for the total.
constexpr int64_t kDirectTiles = 2048;

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* sh /*[4]*/) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const uint64_t t = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return t;
}

// (in and out may be the same array, as for k_scan_apply)
__global__ __launch_bounds__(kScanThreads) void k_scan_apply_direct(const uint32_t* in,
                                                                     const uint64_t* count_dev, int64_t count_host,
                                                                     const uint32_t* __restrict__ partial,
                                                                     uint32_t* out, uint64_t* total_out) {
  const int64_t count = count_dev ? (int64_t)*count_dev : count_host;
  const int64_t np = min((int64_t)gridDim.x, (count + kScanTile - 1) / kScanTile);
  const int64_t lim = blockIdx.x == 0 ? np : min((int64_t)blockIdx.x, np);
  uint64_t acc = 0;
  for (int64_t j = threadIdx.x; j < lim; j += kScanThreads) acc += partial[j];
  __shared__ uint64_t sh64[4];
  const uint64_t pre = block_sum_u64(acc, sh64);
  if (blockIdx.x == 0 && threadIdx.x == 0 && total_out) *total_out = pre;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= count) return;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  const int64_t tb = base + (int64_t)threadIdx.x * kScanItems;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = tb + k;
    v[k] = idx < count ? in[idx] : 0;
    s += v[k];
  }
  __shared__ uint32_t sh[4];
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, total, sh) + (blockIdx.x == 0 ? 0u : (uint32_t)pre);
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = tb + k;
    if (idx < count) out[idx] = run;
    run += v[k];
  }
}

// One workgroup scans inputs up to kOneMax elements in tiles of 16K (16 consecutive per
// thread), carrying the running total and loading the next tile while scanning this one:
// one launch instead of three, where launch latency rather than bandwidth sets the time
// (radix histograms, per-tile counts).
constexpr int kOneThreads = 1024;
constexpr int kOneItems = 16;
constexpr int kOneTile = kOneItems * kOneThreads;
constexpr int64_t kOneMax = (int64_t)1 << 15;

__device__ __forceinline__ void one_load(const uint32_t* in, int64_t i0, int64_t count, uint32_t (&v)[kOneItems]) {
  if (i0 + kOneItems <= count && ((reinterpret_cast<uintptr_t>(in + i0) & 15) == 0)) {
#pragma unroll
    for (int k = 0; k < kOneItems; k += 4) {
      const uint4 q = *reinterpret_cast<const uint4*>(in + i0 + k);
      v[k] = q.x; v[k + 1] = q.y; v[k + 2] = q.z; v[k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kOneItems; ++k) v[k] = i0 + k < count ? in[i0 + k] : 0u;
  }
}

__global__ __launch_bounds__(kOneThreads) void k_scan_one(const uint32_t* in, const uint64_t* count_dev,
                                                          int64_t count_host, uint32_t* out, uint64_t* total_out) {
  __shared__ uint32_t sh[kOneThreads / 64];
  const int64_t count = count_dev ? (int64_t)*count_dev : count_host;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  uint64_t carry = 0;
  uint32_t cur[kOneItems], nxt[kOneItems];
  if (count > 0) one_load(in, (int64_t)kOneItems * t, count, cur);
  for (int64_t base = 0; base < count; base += kOneTile) {
    const int64_t i0 = base + (int64_t)kOneItems * t;
    if (base + kOneTile < count) one_load(in, i0 + kOneTile, count, nxt);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kOneItems; ++k) s += cur[k];
    uint32_t inc = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t x = __shfl_up(inc, off, 64);
      if (lane >= off) inc += x;
    }
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kOneThreads / 64; ++w) {
      const uint32_t x = sh[w];
      wbase += w < wid ? x : 0u;
      tot += x;
    }
    __syncthreads();   // sh is rewritten for the next tile
    uint32_t run = (uint32_t)carry + wbase + (inc - s);
#pragma unroll
    for (int k = 0; k < kOneItems; ++k) {
      if (i0 + k < count) out[i0 + k] = run;
      run += cur[k];
    }
    carry += tot;
#pragma unroll
    for (int k = 0; k < kOneItems; ++k) cur[k] = nxt[k];
  }
  if (t == 0 && total_out) *total_out = carry;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort pass (B-bit digit) of (key, value) pairs. A block owns `sub`
// consecutive sub-tiles of kRadixTile keys, so that the per-block digit histogram (and its
// scan) is small against the keys: the histogram kernel counts the block's keys, the scan
// turns the counts into each block's first output slot per digit, and the scatter walks the
// sub-tiles in order, carrying a running slot per digit in LDS. Within a sub-tile each wave
// ranks its keys with B ballots per key against per-wave digit counters.
// ---------------------------------------------------------------------------
template <class Key, int B>
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const Key* __restrict__ keys, const uint64_t* count_dev,
                                                              int shift, int nblk, int sub, uint32_t* __restrict__ hist) {
  constexpr int ND = 1 << B;
  __shared__ uint32_t h[ND];
  for (int d = threadIdx.x; d < ND; d += kRadixThreads) h[d] = 0;
  __syncthreads();
  const int64_t count = (int64_t)*count_dev;
  const int64_t base = (int64_t)blockIdx.x * kRadixTile * sub;
  const int64_t end = min(count, base + (int64_t)kRadixTile * sub);
  // every block writes its counts (zeros past the live keys): the scan reads them all
  for (int64_t i0 = base + (threadIdx.x & ~63); i0 < end; i0 += kRadixThreads) {
    const int64_t idx = i0 + (threadIdx.x & 63);
    const bool ok = idx < end;
    const uint32_t d = ok ? (uint32_t)(keys[idx] >> shift) & (uint32_t)(ND - 1) : 0u;
    // one LDS atomic per key, or one for the whole wave when all its keys share the digit (the
    // top digits of sorted or tied keys); grouping equal digits by ballots cost more than the
    // atomics' bank conflicts save
    const uint64_t act = __ballot(ok);
    const uint32_t d0 = (uint32_t)__shfl((int)d, 0, 64);
    if (__ballot(ok && d == d0) == act && (act & 1ull)) {
      if ((threadIdx.x & 63) == 0) atomicAdd(&h[d0], (uint32_t)__popcll(act));
    } else if (ok) {
      atomicAdd(&h[d], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < ND; d += kRadixThreads) hist[(int64_t)d * nblk + blockIdx.x] = h[d];
}

template <class Key, int B>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const Key* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                                 Key* __restrict__ kout, uint32_t* __restrict__ vout,
                                                                 const uint64_t* count_dev, int shift, int nblk, int sub,
                                                                 const uint32_t* __restrict__ offs) {
  constexpr int ND = 1 << B;
  constexpr int DPT = ND / kRadixThreads;   // digits per thread in the per-digit phase
  __shared__ uint32_t cnt[4][ND];
  __shared__ uint32_t run[ND];
  __shared__ uint32_t delta[ND];            // a digit's output slot minus its staged position
  __shared__ Key s_k[kRadixTile];           // the sub-tile in digit order
  __shared__ uint32_t s_v[kRadixTile];
  __shared__ uint32_t sh[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t count = (int64_t)*count_dev;
  const int64_t block0 = (int64_t)blockIdx.x * kRadixTile * sub;
  if (block0 >= count) return;
  for (int d = threadIdx.x; d < ND; d += kRadixThreads) run[d] = offs[(int64_t)d * nblk + blockIdx.x];
  const uint64_t lt = lanemask_lt();
  for (int st = 0; st < sub; ++st) {
    const int64_t tile0 = block0 + (int64_t)st * kRadixTile;
    if (tile0 >= count) break;                      // uniform over the block
    for (int d = lane; d < ND; d += 64) cnt[wid][d] = 0;
    __syncthreads();
    const int64_t base = tile0 + (int64_t)wid * kRadixWaveSpan;
    Key k[kRadixItems];
    uint32_t v[kRadixItems], pos[kRadixItems], dig[kRadixItems];
    bool ok[kRadixItems];
    for (int r = 0; r < kRadixItems; ++r) {
      const int64_t idx = base + (int64_t)r * 64 + lane;
      ok[r] = idx < count;
      k[r] = ok[r] ? kin[idx] : Key(0);
      v[r] = ok[r] ? vin[idx] : 0u;
    }
    for (int r = 0; r < kRadixItems; ++r) {
      const uint32_t d = (uint32_t)(k[r] >> shift) & (uint32_t)(ND - 1);
      dig[r] = d;
      uint64_t peers = __ballot(ok[r]);
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
      }
      const uint32_t rank = __popcll(peers & lt);
      uint32_t old = 0;
      if (ok[r]) old = cnt[wid][d];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      if (ok[r] && rank == 0) cnt[wid][d] = old + (uint32_t)__popcll(peers);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      pos[r] = old + rank;
    }
    __syncthreads();
    // per digit (thread tid owns DPT consecutive digits): the digit's staged start (a prefix
    // over the digits), each wave's start within it, and the offset to its output slots
    uint32_t tot[DPT], s = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = threadIdx.x * DPT + j;
      tot[j] = cnt[0][d] + cnt[1][d] + cnt[2][d] + cnt[3][d];
      s += tot[j];
    }
    uint32_t all;
    uint32_t ls = block_exclusive_scan(s, all, sh);
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = threadIdx.x * DPT + j;
      const uint32_t c0 = cnt[0][d], c1 = cnt[1][d], c2 = cnt[2][d];
      cnt[0][d] = ls;
      cnt[1][d] = ls + c0;
      cnt[2][d] = ls + c0 + c1;
      cnt[3][d] = ls + c0 + c1 + c2;
      delta[d] = run[d] - ls;
      run[d] += tot[j];
      ls += tot[j];
    }
    __syncthreads();
    // stage in digit order, then write runs of equal digits to consecutive slots
    for (int r = 0; r < kRadixItems; ++r) {
      if (!ok[r]) continue;
      const uint32_t lp = cnt[wid][dig[r]] + pos[r];
      s_k[lp] = k[r];
      s_v[lp] = v[r];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < all; i += kRadixThreads) {
      const Key kk = s_k[i];
      const uint32_t dst = i + delta[(uint32_t)(kk >> shift) & (uint32_t)(ND - 1)];
      kout[dst] = kk;
      vout[dst] = s_v[i];
    }
    __syncthreads();                                  // cnt and the stage are reused by the next sub-tile
  }
}

// Compaction of the visible entries (radius > 0) in entry order: per block of kCpTile
// entries (kCpItems consecutive ones per thread) a count, then, after the counts' scan,
// each block writes its visible entries from its first slot with the in-block prefix.
constexpr int kCpItems = 16;
constexpr int kCpTile = 256 * kCpItems;

__device__ __forceinline__ void load_radii(const int32_t* __restrict__ radius, int64_t E, int64_t base,
                                           int32_t (&r)[kCpItems]) {
  if (base + kCpItems <= E && (reinterpret_cast<uintptr_t>(radius + base) & 15) == 0) {
#pragma unroll
    for (int k = 0; k < kCpItems; k += 4) {
      const int4 q = *reinterpret_cast<const int4*>(radius + base + k);
      r[k] = q.x; r[k + 1] = q.y; r[k + 2] = q.z; r[k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kCpItems; ++k) r[k] = base + k < E ? radius[base + k] : 0;
  }
}

__global__ __launch_bounds__(256) void k_vis_count(const int32_t* __restrict__ radius, int64_t E,
                                                   uint32_t* __restrict__ counts) {
  const int64_t base = (int64_t)blockIdx.x * kCpTile + (int64_t)threadIdx.x * kCpItems;
  int32_t r[kCpItems];
  load_radii(radius, E, base, r);
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kCpItems; ++k) c += r[k] > 0 ? 1u : 0u;
  __shared__ uint32_t sh[4];
  uint32_t total;
  block_exclusive_scan(c, total, sh);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Visible entry e = item * n + g gets the depth-sort key (item << 31) | bits(depth), the low
// kb bits the sort orders by; with cnt_shift > 0 the entry's tile count rides in the bits
// from cnt_shift up (never sorted on, carried with the key), so that the duplication's
// offsets come from the sorted keys in order instead of a gather of every record.
__global__ __launch_bounds__(256) void k_compact(gs_config cfg, const int32_t* __restrict__ radius,
                                                 const float* __restrict__ depth, const float* __restrict__ rec,
                                                 const gs_item* __restrict__ items, int64_t E, int64_t n,
                                                 int cnt_shift, const uint32_t* __restrict__ offs,
                                                 uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  // the block's visible entries are staged in LDS in order, then written out coalesced
  __shared__ uint64_t s_key[kCpTile];
  __shared__ uint32_t s_val[kCpTile];
  const int64_t base = (int64_t)blockIdx.x * kCpTile + (int64_t)threadIdx.x * kCpItems;
  int32_t r[kCpItems];
  load_radii(radius, E, base, r);
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kCpItems; ++k) c += r[k] > 0 ? 1u : 0u;
  __shared__ uint32_t sh[4];
  uint32_t total;
  uint32_t p = block_exclusive_scan(c, total, sh);
  // with n >= kCpItems a thread's consecutive entries span at most two items
  const int64_t item0 = base / n, next0 = (item0 + 1) * n;
  const bool two = n >= kCpItems;
#pragma unroll
  for (int k = 0; k < kCpItems; ++k) {
    if (r[k] <= 0) continue;
    const int64_t e = base + k;
    const uint64_t item = (uint64_t)(two ? (e >= next0 ? item0 + 1 : item0) : e / n);
    // a visible entry's depth is above z_near > 0, so its sign bit is 0 (the mask only keeps
    // an invalid negative depth from reaching the item bits)
    uint64_t key = (item << 31) | (uint64_t)(__float_as_uint(depth[e]) & 0x7fffffffu);
    if (cnt_shift > 0) {
      const gs_item it = items[item];
      const Rect R = tile_rect(cfg, it.tiles_x, it.tiles_y, *reinterpret_cast<const float4*>(rec + (int64_t)kRecFloats * e),
                               r[k]);
      key |= (uint64_t)((R.x1 - R.x0) * (R.y1 - R.y0)) << cnt_shift;
    }
    s_key[p] = key;
    s_val[p] = (uint32_t)e;
    ++p;
  }
  __syncthreads();
  const int64_t out0 = offs[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < total; i += 256) {
    keys[out0 + i] = s_key[i];
    vals[out0 + i] = s_val[i];
  }
}

// Tile counts of the sorted entries from the count carried in their keys.
__global__ void k_touched_keys(const uint64_t* __restrict__ skeys, const uint64_t* count_dev, int cnt_shift,
                               uint32_t* __restrict__ touched) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= (int64_t)*count_dev) return;
  touched[j] = (uint32_t)(skeys[j] >> cnt_shift);
}

__global__ void k_touched(gs_config cfg, const uint32_t* __restrict__ svals, const uint64_t* count_dev,
                          const float* __restrict__ rec, const int32_t* __restrict__ radius,
                          const gs_item* __restrict__ items, int64_t n, uint32_t* __restrict__ touched) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= (int64_t)*count_dev) return;
  const uint32_t e = svals[j];
  const gs_item it = items[e / n];
  const Rect R = tile_rect(cfg, it.tiles_x, it.tiles_y, *reinterpret_cast<const float4*>(rec + (int64_t)kRecFloats * e), radius[e]);
  touched[j] = (uint32_t)((R.x1 - R.x0) * (R.y1 - R.y0));
}

// Each wave takes 64 consecutive depth-ordered entries and writes their duplicates as one
// run (their offsets are consecutive): lane l of round k writes output k * 64 + l of the
// run, finding its entry by a binary search over the wave's inclusive count prefix. A
// footprint with many tiles is spread over the wave instead of one lane, and the stores
// are coalesced.
__global__ __launch_bounds__(256) void k_duplicate(gs_config cfg, const uint32_t* __restrict__ svals,
                                                   const uint64_t* count_dev, const uint32_t* __restrict__ offs,
                                                   const float* __restrict__ rec, const int32_t* __restrict__ radius,
                                                   const gs_item* __restrict__ items, int64_t n, int64_t cap,
                                                   uint32_t* __restrict__ tkeys, uint32_t* __restrict__ tvals,
                                                   const uint64_t* __restrict__ dtotal, uint64_t* __restrict__ live,
                                                   int64_t* __restrict__ n_dup_out, int32_t* __restrict__ status,
                                                   uint32_t* __restrict__ ranges, int64_t rn) {
  // (also: the duplicate count clamped to the capacity, with its status, and the tile ranges
  // cleared for the range pass after the tile sort)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint64_t D = *dtotal;
    *live = D > (uint64_t)cap ? (uint64_t)cap : D;
    if (n_dup_out) *n_dup_out = (int64_t)D;
    if (status) *status = D > (uint64_t)cap ? GS_ERR_CAPACITY : GS_OK;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rn; i += (int64_t)gridDim.x * blockDim.x)
    ranges[i] = 0u;
  __shared__ uint32_t s_pre[4][64];   // inclusive prefix of the wave's tile counts
  __shared__ int4 s_rect[4][64];      // x0, width, tiles_x, id of tile (0, y0) of the item
  __shared__ uint32_t s_g[4][64];     // Gaussian index
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t count = (int64_t)*count_dev;
  const int64_t j0 = ((int64_t)blockIdx.x * 4 + wid) * 64;
  if (j0 >= count) return;
  const int64_t j = j0 + lane;
  uint32_t c = 0;
  if (j < count) {
    const uint32_t e = svals[j];
    const int64_t item = (int64_t)(e / (uint32_t)n);   // entries and n fit 32 bits
    const gs_item it = items[item];
    const Rect R = tile_rect(cfg, it.tiles_x, it.tiles_y, *reinterpret_cast<const float4*>(rec + (int64_t)kRecFloats * e),
                             radius[e]);
    const int w = R.x1 - R.x0;
    c = (uint32_t)(w * (R.y1 - R.y0));
    s_rect[wid][lane] = make_int4(R.x0, w, it.tiles_x, it.tile_base + R.y0 * it.tiles_x);
    s_g[wid][lane] = (uint32_t)(e - item * n);
  }
  uint32_t inc = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  s_pre[wid][lane] = inc;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint32_t total = __shfl(inc, 63, 64);
  const int64_t base = offs[j0];
  for (uint32_t k = lane; k < total; k += 64) {
    const int64_t pos = base + k;
    if (pos >= cap) break;
    int lo = 0, hi = 63;   // first entry whose inclusive prefix exceeds k
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_pre[wid][mid] > k) hi = mid; else lo = mid + 1;
    }
    const uint32_t m = k - (lo > 0 ? s_pre[wid][lo - 1] : 0u);   // index within the entry's rect
    const int4 r = s_rect[wid][lo];
    const int row = (int)(m / (uint32_t)r.y), col = (int)m - row * r.y;
    tkeys[pos] = (uint32_t)(r.w + row * r.z + r.x + col);
    tvals[pos] = s_g[wid][lo];
  }
}

__global__ void k_ranges(const uint32_t* __restrict__ tkeys, const uint64_t* count_dev, uint32_t* __restrict__ ranges) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t D = (int64_t)*count_dev;
  if (j >= D) return;
  const uint32_t t = tkeys[j];
  if (j == 0 || tkeys[j - 1] != t) ranges[2 * (int64_t)t] = (uint32_t)j;
  if (j == D - 1 || tkeys[j + 1] != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(j + 1);
}

__global__ void k_full_keys(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ tvals,
                            const uint64_t* count_dev, const float* __restrict__ depth,
                            const gs_item* __restrict__ items, int n_items, int64_t n, uint64_t* __restrict__ keys) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= (int64_t)*count_dev) return;
  const uint32_t t = tkeys[j];
  const int item = item_of_tile(items, n_items, (int)t);
  keys[j] = ((uint64_t)t << 32) | (uint64_t)__float_as_uint(depth[(int64_t)item * n + tvals[j]]);
}

// ---------------------------------------------------------------------------
// Bucket path (short tile lists): a counting sort of the duplicates by tile in one pass,
// then every tile's list sorted by its (depth bits, Gaussian index) keys in LDS.
//
// Block b of the two pair kernels takes the same entries. The first counts the block's
// duplicates per tile with LDS atomics and writes the counts tile-major; their exclusive scan
// gives every (tile, block) its first slot, tile t's list starting at the slot of (t, 0). The
// second kernel hands each duplicate the next slot of its (tile, block) from an LDS counter,
// in whatever order the LDS atomics serve the lanes, and stores its key there. The per-tile
// sort then puts every list in (depth, index) order: the key is unique within a tile (a
// Gaussian meets a tile of its item once), so the order in which slots were taken does not
// show in the result, which is the (tile, depth, index) order of the radix path exactly.
// ---------------------------------------------------------------------------
constexpr int kBkThreads = 1024;
constexpr int kBkWaves = kBkThreads / 64;
constexpr int kBkMaxTiles = 12288;   // tile counters a block keeps in LDS (48 KB)

template <bool COUNT>
__global__ __launch_bounds__(kBkThreads) void k_bucket_pairs(gs_config cfg, const int32_t* __restrict__ radius,
                                                             const float* __restrict__ depth,
                                                             const float* __restrict__ rec,
                                                             const gs_item* __restrict__ items, int64_t E, int64_t n,
                                                             int n_tiles, int nblk, uint32_t* __restrict__ hist,
                                                             int64_t cap, uint64_t* __restrict__ tmp,
                                                             const uint64_t* __restrict__ dtotal,
                                                             int64_t* __restrict__ n_dup_out,
                                                             int32_t* __restrict__ status) {
  __shared__ uint32_t s_cnt[kBkMaxTiles];      // per tile: the block's count, or its next slot
  __shared__ uint32_t s_pre[kBkWaves][64];     // inclusive prefix of the wave's tile counts
  __shared__ int4 s_rect[kBkWaves][64];        // x0, width, tiles_x, id of tile (0, y0) of the item
  __shared__ uint64_t s_key[kBkWaves][64];     // the entry's key within its tiles (scatter)
  const int b = blockIdx.x;
  for (int t = threadIdx.x; t < n_tiles; t += kBkThreads) s_cnt[t] = COUNT ? 0u : hist[(int64_t)t * nblk + b];
  if (!COUNT && b == 0 && threadIdx.x == 0) {
    const uint64_t D = *dtotal;
    if (n_dup_out) *n_dup_out = (int64_t)D;
    if (status) *status = D > (uint64_t)cap ? GS_ERR_CAPACITY : GS_OK;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t n_groups = (E + 63) >> 6, stride = (int64_t)nblk * kBkWaves;
  // groups of 64 consecutive entries, the block's waves on consecutive groups in each round.
  // Loads run ahead of use: a group's records (and depths) are loaded one group ahead, from
  // radii loaded two groups ahead, so that a group's work waits on no memory round trip.
  int64_t grp = (int64_t)b * kBkWaves + wid;
  auto radius_of = [&](int64_t gq) { return gq * 64 + lane < E ? radius[gq * 64 + lane] : 0; };
  auto rec_of = [&](int64_t gq, int r) {
    return r > 0 ? *reinterpret_cast<const float4*>(rec + (int64_t)kRecFloats * (gq * 64 + lane))
                 : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  auto depth_of = [&](int64_t gq, int r) { return (!COUNT && r > 0) ? depth[gq * 64 + lane] : 0.f; };
  int r1 = radius_of(grp), r2 = radius_of(grp + stride);
  float4 m1 = rec_of(grp, r1);
  float d1 = depth_of(grp, r1);
  for (; grp < n_groups; grp += stride) {
    const int64_t e = grp * 64 + lane;
    const int r = r1;
    const float4 mr = m1;
    const float dr = d1;
    r1 = r2;
    m1 = rec_of(grp + stride, r1);
    d1 = depth_of(grp + stride, r1);
    r2 = radius_of(grp + 2 * stride);
    uint32_t c = 0;
    int4 rc = make_int4(0, 1, 0, 0);
    uint64_t key = 0;
    if (r > 0) {   // (r is 0 past the entries)
      const uint32_t item = (uint32_t)e / (uint32_t)n;   // entries fit 32 bits
      const gs_item it = items[item];
      const Rect R = tile_rect(cfg, it.tiles_x, it.tiles_y, mr, r);
      const int w = R.x1 - R.x0;
      c = (uint32_t)(w * (R.y1 - R.y0));
      rc = make_int4(R.x0, w, it.tiles_x, it.tile_base + R.y0 * it.tiles_x);
      // a visible depth is above z_near > 0 (the mask keeps the sign bit out of the order)
      if (!COUNT)
        key = ((uint64_t)(__float_as_uint(dr) & 0x7fffffffu) << 32) | (uint64_t)((uint32_t)e - item * (uint32_t)n);
    }
    uint32_t inc = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t t = __shfl_up(inc, off, 64);
      if (lane >= off) inc += t;
    }
    // (the previous group's reads of the wave's slots are done: a wave's LDS operations
    // complete in order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    s_pre[wid][lane] = inc;
    s_rect[wid][lane] = rc;
    if (!COUNT) s_key[wid][lane] = key;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t total = __shfl(inc, 63, 64);
    for (uint32_t k = lane; k < total; k += 64) {
      int lo = 0, hi = 63;   // first entry whose inclusive prefix exceeds k
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_pre[wid][mid] > k) hi = mid; else lo = mid + 1;
      }
      const uint32_t m = k - (lo > 0 ? s_pre[wid][lo - 1] : 0u);
      const int4 rr = s_rect[wid][lo];
      const int row = (int)(m / (uint32_t)rr.y), col = (int)m - row * rr.y;
      const int tile = rr.w + row * rr.z + rr.x + col;
      const uint32_t pos = atomicAdd(&s_cnt[tile], 1u);
      if (!COUNT && (int64_t)pos < cap) tmp[pos] = s_key[wid][lo];
    }
  }
  if (COUNT) {
    __syncthreads();
    for (int t = threadIdx.x; t < n_tiles; t += kBkThreads) hist[(int64_t)t * nblk + b] = s_cnt[t];
  }
}

// Tile t's list: [offs[t * nblk], offs[(t + 1) * nblk]) (the duplicate total past the last
// tile), clamped to the capacity; a negative length (wrapped 32-bit slots past the capacity)
// reads as empty.
__device__ __forceinline__ void tile_span(const uint32_t* offs, int nblk, int n_tiles, const uint64_t* dtotal,
                                          int64_t cap, int t, int64_t& start, int64_t& len) {
  const int64_t a = offs[(int64_t)t * nblk];
  const int64_t b = t + 1 < n_tiles ? (int64_t)offs[(int64_t)(t + 1) * nblk] : (int64_t)*dtotal;
  start = min(a, cap);
  len = min(b, cap) - start;
}

// Per-tile sort. The list is cut into sub-lists of 256 keys; a wave owns whole sub-lists
// (sub-list c: wave c mod W), which it sorts in registers with Batcher's bitonic network,
// four keys per lane (lane l ends with sorted positions 4 l .. 4 l + 3; steps between lanes
// exchange keys by shuffles). A list of one sub-list is then written out directly. Otherwise
// the sorted sub-lists go to LDS, and the rank of the key at sorted position j in the whole
// list is j plus, for every other sub-list, the number of its keys below the key (a binary
// search). Lists of up to CH keys; T threads (W = T / 64).
constexpr int kSub = 256;

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic sort of the wave's 256 keys, lane l holding positions 4 l + r in v[r].
// Stage (k, j) pairs position i with i ^ j; the pair's lower position takes the smaller key
// when i & k is 0 (an ascending run), the larger one otherwise.
__device__ __forceinline__ void wave_sort256(uint64_t (&v)[4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 2; k <= 256; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j >= 1; j >>= 1) {
      if (j >= 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * lane + r;
          const uint64_t o = shfl_xor64(v[r], j >> 2);   // position i ^ j: lane ^ (j / 4), same r
          const bool lt = v[r] < o;
          const bool want_min = ((i & j) == 0) == ((i & k) == 0);
          v[r] = (lt == want_min) ? v[r] : o;
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int p = r ^ j;
          if (p < r) continue;   // each in-lane pair once, at its lower position
          const bool up = ((4 * lane + r) & k) == 0;
          const uint64_t x = v[r], y = v[p];
          const bool sw = up ? (y < x) : (x < y);
          v[r] = sw ? y : x;
          v[p] = sw ? x : y;
        }
      }
    }
  }
}

template <int T, int CH>
__device__ __forceinline__ void sort_tile(uint64_t* s, const uint64_t* __restrict__ g, int L, int t, int64_t start,
                                          const float* __restrict__ depth, const gs_item* __restrict__ items,
                                          int n_items, int64_t n, uint32_t* __restrict__ vals,
                                          uint64_t* __restrict__ keys) {
  constexpr int W = T / 64, NS = CH / (kSub * W), R = kSub / 64;
  static_assert(R == 4, "four keys per lane");
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nsub = (L + kSub - 1) / kSub;
  uint64_t k[NS][R];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int c0 = (wid + q * W) * kSub, cl = min(kSub, L - c0);   // cl <= 0: no sub-list
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = lane * R + r;
      k[q][r] = j < cl ? g[c0 + j] : ~0ull;   // past the list: +inf, sorted to the end
    }
    if (cl > 0) wave_sort256(k[q]);   // uniform over the wave
  }
  const int64_t item = keys ? item_of_tile(items, n_items, t) : 0;
  if (nsub == 1) {
    if (wid == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int j = lane * R + r;
        if (j >= L) continue;
        const uint32_t gi = (uint32_t)k[0][r];
        vals[start + j] = gi;
        if (keys) {
          const uint32_t db = gi < (uint64_t)n ? __float_as_uint(depth[item * n + gi]) : 0u;
          keys[start + j] = ((uint64_t)(uint32_t)t << 32) | (uint64_t)db;
        }
      }
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int c0 = (wid + q * W) * kSub, cl = min(kSub, L - c0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = lane * R + r;
      if (j < cl) s[c0 + j] = k[q][r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int own = wid + q * W, c0 = own * kSub, cl = min(kSub, L - c0);
    if (cl <= 0) continue;   // uniform over the wave
    // lane l holds positions 4 l .. 4 l + 3 of the sorted sub-list: neighbouring lanes search
    // for neighbouring keys, so their LDS reads mostly meet at the same addresses
    uint32_t rank[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rank[r] = (uint32_t)(lane * R + r);
    // the other sub-lists four at a time, the 4 x R searches in lockstep (branch-free lower
    // bound by binary lifting: pos grows by each power of two while the key at pos + step - 1
    // is below the searched key), so that their LDS reads overlap
    for (int cg = 0; cg < nsub; cg += 4) {
      int nn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = cg + u;
        nn[u] = (c < nsub && c != own) ? min(kSub, L - c * kSub) : 0;
      }
      int pos[4][R];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) pos[u][r] = 0;
#pragma unroll
      for (int step = kSub; step >= 1; step >>= 1) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int p = pos[u][r] + step;
            if (p <= nn[u] && s[(cg + u) * kSub + p - 1] < k[q][r]) pos[u][r] = p;
          }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) rank[r] += (uint32_t)pos[u][r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (lane * R + r >= cl) continue;
      const uint32_t gi = (uint32_t)k[q][r];
      vals[start + rank[r]] = gi;
      if (keys) {
        const uint32_t db = gi < (uint64_t)n ? __float_as_uint(depth[item * n + gi]) : 0u;
        keys[start + rank[r]] = ((uint64_t)(uint32_t)t << 32) | (uint64_t)db;
      }
    }
  }
}

// Lists longer than the long kernel's CH: the all-ascending form of Batcher's bitonic network
// (every compare-exchange puts the smaller key at the lower position; a merge of two sorted
// halves of k keys starts by comparing position i with its mirror k - 1 - i), in place in the
// scatter buffer. Positions past the list count as +inf and never move, so a list of L keys
// is sorted as the next power of two with only its first L positions touched. Steps over
// pairs closer than CH / 2 run chunk by chunk in LDS, the others in global memory.
template <int T>
__device__ __forceinline__ void bt_step(uint64_t* s, int m, int h, bool flip) {
  for (int p = threadIdx.x; p < (m >> 1); p += T) {
    const int q = p & (h - 1), b = (p - q) << 1;
    const int lo = b + q, hi = flip ? b + 2 * h - 1 - q : lo + h;
    const uint64_t x = s[lo], y = s[hi];
    if (y < x) {
      s[lo] = y;
      s[hi] = x;
    }
  }
}

// Steps h = h0, h0 / 2, ..., 1 of merge stage k (a step with h == k / 2 is the flip) on an
// LDS chunk of m keys. Thread t takes pairs t + T r, so for h <= 64 wave w only touches keys
// 128 w + 2 T r .. + 127: two such steps in a row need only the wave's own ordering.
template <int T>
__device__ __forceinline__ void bt_stage(uint64_t* s, int m, int64_t k, int h0, bool& wide) {
  for (int h = h0; h >= 1; h >>= 1) {
    const bool w = h >= 128;
    if (w || wide) {
      __syncthreads();
    } else {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    wide = w;
    bt_step<T>(s, m, h, (int64_t)h == (k >> 1));
  }
}

template <int T, int CH>
__device__ void bitonic_tile(uint64_t* s, uint64_t* g, int64_t L) {
  int64_t m = 1;
  while (m < L) m <<= 1;
  auto chunk = [&](int64_t c0, int64_t k, int h0) {
    for (int i = threadIdx.x; i < CH; i += T) s[i] = c0 + i < L ? g[c0 + i] : ~0ull;
    bool wide = true;
    if (h0 == 0) {
      for (int kk = 2; kk <= CH; kk <<= 1) bt_stage<T>(s, CH, kk, kk >> 1, wide);
    } else {
      bt_stage<T>(s, CH, k, h0, wide);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < CH; i += T)
      if (c0 + i < L) g[c0 + i] = s[i];
    __syncthreads();
  };
  for (int64_t c0 = 0; c0 < L; c0 += CH) chunk(c0, 0, 0);   // every chunk sorted
  for (int64_t k = 2 * CH; k <= m; k <<= 1) {
    for (int64_t h = k >> 1; h >= CH; h >>= 1) {
      const bool flip = h == (k >> 1);
      for (int64_t p = threadIdx.x; p < (m >> 1); p += T) {
        const int64_t q = p & (h - 1), b = (p - q) << 1;
        const int64_t lo = b + q, hi = flip ? b + 2 * h - 1 - q : lo + h;
        if (hi >= L) continue;   // the partner is +inf: nothing moves
        const uint64_t x = g[lo], y = g[hi];
        if (y < x) {
          g[lo] = y;
          g[hi] = x;
        }
      }
      __syncthreads();
    }
    for (int64_t c0 = 0; c0 < L; c0 += CH) chunk(c0, k, CH >> 1);
  }
}

// Short lists (up to 1024 keys), one block per tile; also writes every tile's range.
constexpr int kShortKeys = 1024;
constexpr int kLongThreads = 1024;
constexpr int kLongKeys = 8192;

__global__ __launch_bounds__(256) void k_tile_sort_short(const uint32_t* __restrict__ offs, int nblk, int n_tiles,
                                                         const uint64_t* __restrict__ dtotal, int64_t cap,
                                                         const uint64_t* __restrict__ tmp,
                                                         const float* __restrict__ depth,
                                                         const gs_item* __restrict__ items, int n_items, int64_t n,
                                                         uint32_t* __restrict__ ranges, uint32_t* __restrict__ vals,
                                                         uint64_t* __restrict__ keys) {
  __shared__ __align__(16) uint64_t s[kShortKeys];
  const int t = blockIdx.x;
  int64_t start, L;
  tile_span(offs, nblk, n_tiles, dtotal, cap, t, start, L);
  if (threadIdx.x == 0) {
    ranges[2 * (int64_t)t] = L > 0 ? (uint32_t)start : 0u;
    ranges[2 * (int64_t)t + 1] = L > 0 ? (uint32_t)(start + L) : 0u;
  }
  if (L <= 0 || L > kShortKeys) return;
  sort_tile<256, kShortKeys>(s, tmp + start, (int)L, t, start, depth, items, n_items, n, vals, keys);
}

// Longer lists: blocks of 1024 threads walk the tiles; up to 8192 keys by rank, beyond that
// the bitonic network.
__global__ __launch_bounds__(kLongThreads) void k_tile_sort_long(const uint32_t* __restrict__ offs, int nblk,
                                                                 int n_tiles, const uint64_t* __restrict__ dtotal,
                                                                 int64_t cap, uint64_t* tmp,
                                                                 const float* __restrict__ depth,
                                                                 const gs_item* __restrict__ items, int n_items,
                                                                 int64_t n, uint32_t* __restrict__ vals,
                                                                 uint64_t* __restrict__ keys) {
  __shared__ __align__(16) uint64_t s[kLongKeys];
  __shared__ int s_list[kLongThreads];
  __shared__ int s_n;
  // the block's tiles are blockIdx.x + gridDim.x i: their spans are read in parallel, the long
  // ones listed in LDS (kLongThreads per round)
  for (int64_t t0 = blockIdx.x; t0 < n_tiles; t0 += (int64_t)gridDim.x * kLongThreads) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const int64_t tt = t0 + (int64_t)gridDim.x * threadIdx.x;
    if (tt < n_tiles) {
      int64_t st, ln;
      tile_span(offs, nblk, n_tiles, dtotal, cap, (int)tt, st, ln);
      if (ln > kShortKeys) s_list[atomicAdd(&s_n, 1)] = (int)tt;
    }
    __syncthreads();
    const int nl = s_n;
    for (int li = 0; li < nl; ++li) {
      const int t = s_list[li];
      int64_t start, L;
      tile_span(offs, nblk, n_tiles, dtotal, cap, t, start, L);
      if (L <= kLongKeys) {
        sort_tile<kLongThreads, kLongKeys>(s, tmp + start, (int)L, t, start, depth, items, n_items, n, vals, keys);
      } else {
        uint64_t* g = tmp + start;
        bitonic_tile<kLongThreads, kLongKeys>(s, g, L);
        const int64_t item = keys ? item_of_tile(items, n_items, t) : 0;
        for (int64_t i = threadIdx.x; i < L; i += kLongThreads) {
          const uint64_t key = g[i];
          const uint32_t gi = (uint32_t)key;
          vals[start + i] = gi;
          if (keys) {
            const uint32_t db = gi < (uint64_t)n ? __float_as_uint(depth[item * n + gi]) : 0u;
            keys[start + i] = ((uint64_t)(uint32_t)t << 32) | (uint64_t)db;
          }
        }
      }
      __syncthreads();   // s is reused by the block's next tile
    }
    __syncthreads();     // s_n and s_list are rewritten by the next round
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct SortWs {
  uint32_t* flags;     // [E]   per-block visible counts, then the blocks' first slots
  uint32_t* partial;   // [max(E, cap, hist) / 4096 + 2]
  uint64_t* vkeys[2];  // [E]
  uint32_t* vvals[2];  // [E]
  uint32_t* touched;   // [E]   touched counts, then duplicate offsets
  uint32_t* tkeys[2];  // [cap]
  uint32_t* tvals;     // [cap] (the second value buffer is the caller's vals)
  uint32_t* hist;      // [256 * nblk_max]
  uint64_t* counters;  // [4]: n_visible, D total, D live, scratch
  size_t bytes;
};

int bits_for(uint64_t x) {  // bits needed to represent values < x
  int b = 0;
  while (b < 64 && (1ull << b) < x) ++b;
  return b;
}

SortWs plan_sort(int64_t E, int64_t cap, void* base) {
  SortWs w{};
  const int64_t nmax = std::max<int64_t>(E, cap);
  const int64_t nblk = ceil_div(std::max<int64_t>(nmax, 1), kRadixTile);
  const int64_t hist_n = ((int64_t)1 << kDigitMax) * nblk;   // the largest digit with one sub-tile per block
  const int64_t np = ceil_div(std::max<int64_t>(std::max(nmax, hist_n), 1), kScanTile) + 2;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  size_t o_flags = take(4 * E), o_part = take(4 * np), o_vk0 = take(8 * E), o_vk1 = take(8 * E),
         o_vv0 = take(4 * E), o_vv1 = take(4 * E), o_touch = take(4 * E), o_tk0 = take(4 * cap),
         o_tk1 = take(4 * cap), o_tv = take(4 * cap), o_hist = take(4 * hist_n), o_cnt = take(8 * 4);
  w.bytes = off;
  if (base) {
    char* b = static_cast<char*>(base);
    w.flags = (uint32_t*)(b + o_flags);
    w.partial = (uint32_t*)(b + o_part);
    w.vkeys[0] = (uint64_t*)(b + o_vk0);
    w.vkeys[1] = (uint64_t*)(b + o_vk1);
    w.vvals[0] = (uint32_t*)(b + o_vv0);
    w.vvals[1] = (uint32_t*)(b + o_vv1);
    w.touched = (uint32_t*)(b + o_touch);
    w.tkeys[0] = (uint32_t*)(b + o_tk0);
    w.tkeys[1] = (uint32_t*)(b + o_tk1);
    w.tvals = (uint32_t*)(b + o_tv);
    w.hist = (uint32_t*)(b + o_hist);
    w.counters = (uint64_t*)(b + o_cnt);
  }
  return w;
}

// Exclusive scan of in[0..count) into out; total (if non-null) to *total.
int device_scan(const uint32_t* in, uint32_t* out, const uint64_t* count_dev, int64_t count_host, int64_t cap_count,
                uint32_t* partial, uint64_t* total, hipStream_t s) {
  if (cap_count <= kOneMax) {
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kOneThreads), 0, s, in, count_dev, count_host, out, total);
    return launch_status();
  }
  const int64_t nb = std::max<int64_t>(1, ceil_div(cap_count, kScanTile));
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, count_dev, count_host, partial);
  if (nb <= kDirectTiles) {
    hipLaunchKernelGGL(k_scan_apply_direct, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, count_dev, count_host,
                       partial, out, total);
    return launch_status();
  }
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partial, nb, count_dev, count_host, total);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, count_dev, count_host, partial, out);
  return launch_status();
}

// Sub-tiles per radix block for cap_count keys: about 8K blocks at most, so that the
// per-block histograms stay a small fraction of the keys.
int radix_sub(int64_t cap_count) {
  return (int)std::min<int64_t>(16, std::max<int64_t>(1, ceil_div(cap_count, (int64_t)kRadixTile * 8192)));
}

template <class Key, int B>
int radix_pass(Key* kin, Key* kout, uint32_t* vin, uint32_t* vout, const uint64_t* count_dev, int64_t cap_count,
               int shift, SortWs& w, hipStream_t s) {
  const int sub = radix_sub(cap_count);
  const int nblk = (int)std::max<int64_t>(1, ceil_div(cap_count, (int64_t)kRadixTile * sub));
  const int64_t nh = ((int64_t)1 << B) * nblk;
  hipLaunchKernelGGL((k_radix_hist<Key, B>), dim3(nblk), dim3(kRadixThreads), 0, s, kin, count_dev, shift, nblk, sub,
                     w.hist);
  const int st = device_scan(w.hist, w.hist, nullptr, nh, nh, w.partial, nullptr, s);
  if (st) return st;
  hipLaunchKernelGGL((k_radix_scatter<Key, B>), dim3(nblk), dim3(kRadixThreads), 0, s, kin, vin, kout, vout, count_dev,
                     shift, nblk, sub, w.hist);
  return launch_status();
}

// Stable sort of `bits`-bit keys in ceil(bits / 11) passes of equal digits (8 to 11 bits).
template <class Key>
int radix_sort(Key* k0, Key* k1, uint32_t* v0, uint32_t* v1, const uint64_t* count_dev, int64_t cap_count, int bits,
               SortWs& w, hipStream_t s, int* final_buf) {
  const int passes = std::max(1, (bits + kDigitMax - 1) / kDigitMax);
  const int B = std::max(8, (bits + passes - 1) / passes);
  Key* kb[2] = {k0, k1};
  uint32_t* vb[2] = {v0, v1};
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * B;
    int st = GS_OK;
    switch (B) {
      case 8: st = radix_pass<Key, 8>(kb[cur], kb[cur ^ 1], vb[cur], vb[cur ^ 1], count_dev, cap_count, shift, w, s); break;
      case 9: st = radix_pass<Key, 9>(kb[cur], kb[cur ^ 1], vb[cur], vb[cur ^ 1], count_dev, cap_count, shift, w, s); break;
      case 10: st = radix_pass<Key, 10>(kb[cur], kb[cur ^ 1], vb[cur], vb[cur ^ 1], count_dev, cap_count, shift, w, s); break;
      default: st = radix_pass<Key, 11>(kb[cur], kb[cur ^ 1], vb[cur], vb[cur ^ 1], count_dev, cap_count, shift, w, s); break;
    }
    if (st) return st;
    cur ^= 1;
  }
  *final_buf = cur;
  return GS_OK;
}

// Number of passes radix_sort takes for `bits`-bit keys, and the key bits they examine
// (passes x digit width, at least `bits`).
int radix_passes(int bits) { return std::max(1, (bits + kDigitMax - 1) / kDigitMax); }
int radix_covered_bits(int bits) {
  const int passes = radix_passes(bits);
  return passes * std::max(8, (bits + passes - 1) / passes);
}

}  // namespace

// Bucket path: block count of the pair kernels. Every block writes (and the scan reads) one
// counter per tile, while fewer blocks leave each wave more groups of entries to walk one
// after another; the two costs balance near 11 sqrt(E / tiles) blocks (at most 512, two per
// compute unit, and at most 2^22 counters).
int bucket_blocks(int64_t E, int64_t n_tiles) {
  const int64_t groups = ceil_div(std::max<int64_t>(E, 1), 64);
  const double bal = 11.0 * std::sqrt((double)std::max<int64_t>(E, 1) / (double)std::max<int64_t>(n_tiles, 1));
  int64_t nb = std::min<int64_t>({(int64_t)512, ceil_div(groups, kBkWaves), std::max<int64_t>(16, (int64_t)bal)});
  nb = std::min<int64_t>(nb, ((int64_t)1 << 22) / std::max<int64_t>(n_tiles, 1));
  return (int)std::max<int64_t>(1, nb);
}

struct BucketWs {
  uint32_t* hist;      // [n_tiles * nblk]
  uint32_t* partial;   // scan partials
  uint64_t* tmp;       // [cap]
  uint64_t* counters;  // [0]: duplicate total
  int nblk;
  int64_t hist_n;
  size_t bytes;
};

BucketWs plan_bucket(int64_t E, int64_t n_tiles, int64_t cap, void* base) {
  BucketWs w{};
  w.nblk = bucket_blocks(E, n_tiles);
  w.hist_n = std::max<int64_t>(n_tiles, 0) * w.nblk;
  const int64_t np = ceil_div(std::max<int64_t>(w.hist_n, 1), kScanTile) + 2;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t o_hist = take(4 * (size_t)std::max<int64_t>(w.hist_n, 1)), o_part = take(4 * (size_t)np),
               o_tmp = take(8 * (size_t)std::max<int64_t>(cap, 1)), o_cnt = take(8 * 4);
  w.bytes = off;
  if (base) {
    char* b = static_cast<char*>(base);
    w.hist = (uint32_t*)(b + o_hist);
    w.partial = (uint32_t*)(b + o_part);
    w.tmp = (uint64_t*)(b + o_tmp);
    w.counters = (uint64_t*)(b + o_cnt);
  }
  return w;
}

// Automatic choice: the bucket path up to this many (item, Gaussian) entries (and up to
// kBkMaxTiles tiles). Its per-tile sorts cost more than linear time in a list's length, and
// the lists grow with the scene; the radix path's passes cost the same per duplicate whatever
// the lists. (The autotuner times both methods on the workload itself.)
constexpr int64_t kBucketMaxEntries = (int64_t)1 << 22;

bool bucket_path(const gs_config& cfg, int64_t E, int n_tiles) {
  if (n_tiles > kBkMaxTiles) return false;
  return cfg.sort_mode == 2 || (cfg.sort_mode == 0 && E <= kBucketMaxEntries);
}

int launch_bucket_sort(const gs_config& cfg, const gs_projected& proj, const gs_item* items, int n_items, int64_t n,
                       int n_tiles, int64_t cap, void* ws, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                       int64_t* n_dup_dev, int32_t* status_dev, hipStream_t s) {
  const int64_t E = (int64_t)n_items * n;
  BucketWs w = plan_bucket(E, n_tiles, cap, ws);
  uint64_t* d_total = w.counters;
  hipLaunchKernelGGL(k_bucket_pairs<true>, dim3(w.nblk), dim3(kBkThreads), 0, s, cfg, proj.radius, proj.depth,
                     proj.rec, items, E, n, n_tiles, w.nblk, w.hist, cap, w.tmp, (const uint64_t*)nullptr,
                     (int64_t*)nullptr, (int32_t*)nullptr);
  const int st = device_scan(w.hist, w.hist, nullptr, w.hist_n, w.hist_n, w.partial, d_total, s);
  if (st) return st;
  hipLaunchKernelGGL(k_bucket_pairs<false>, dim3(w.nblk), dim3(kBkThreads), 0, s, cfg, proj.radius, proj.depth,
                     proj.rec, items, E, n, n_tiles, w.nblk, w.hist, cap, w.tmp, (const uint64_t*)d_total, n_dup_dev,
                     status_dev);
  if (n_tiles > 0) {
    hipLaunchKernelGGL(k_tile_sort_short, dim3((unsigned)n_tiles), dim3(256), 0, s, w.hist, w.nblk, n_tiles,
                       (const uint64_t*)d_total, cap, w.tmp, proj.depth, items, n_items, n, ranges, vals, keys);
    hipLaunchKernelGGL(k_tile_sort_long, dim3((unsigned)std::min(n_tiles, 512)), dim3(kLongThreads), 0, s, w.hist,
                       w.nblk, n_tiles, (const uint64_t*)d_total, cap, w.tmp, proj.depth, items, n_items, n, vals,
                       keys);
  }
  return launch_status();
}

size_t bin_sort_workspace(int64_t E, int64_t cap, int64_t n_tiles) {
  return std::max(plan_sort(E, cap, nullptr).bytes, plan_bucket(E, n_tiles, cap, nullptr).bytes);
}

int64_t scan_partials_needed(int64_t n) { return ceil_div(std::max<int64_t>(n, 1), kScanTile) + 2; }

int scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partial, uint64_t* total, hipStream_t s) {
  return device_scan(in, out, nullptr, n, n, partial, total, s);
}

int launch_bin_sort(const gs_config& cfg, const gs_projected& proj, const gs_item* items, int n_items, int64_t n,
                    int n_tiles, int64_t cap, void* ws, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                    int64_t* n_dup_dev, int32_t* status_dev, hipStream_t s) {
  const int64_t E = (int64_t)n_items * n;
  if (cfg.sort_mode == 2 && n_tiles > kBkMaxTiles) return GS_ERR_UNSUPPORTED;
  if (bucket_path(cfg, E, n_tiles))
    return launch_bucket_sort(cfg, proj, items, n_items, n, n_tiles, cap, ws, keys, vals, ranges, n_dup_dev,
                              status_dev, s);
  SortWs w = plan_sort(E, cap, ws);
  uint64_t* n_vis = w.counters + 0;
  uint64_t* d_total = w.counters + 1;
  uint64_t* d_live = w.counters + 2;
  const unsigned eb = (unsigned)std::max<int64_t>(1, ceil_div(E, 256));
  // 1. compaction of the visible entries: block counts (into the flags buffer), their scan
  // (the total is the visible count), the blocks' ordered writes
  // the sort key's bits; an entry's tile count (at most the tiles of all items) rides in the
  // top bits when they lie above every bit the radix passes examine
  const int kbits = 31 + bits_for((uint64_t)n_items);
  const int cbits = bits_for((uint64_t)n_tiles + 1);
  const int cnt_shift = 64 - cbits >= radix_covered_bits(kbits) ? 64 - cbits : 0;
  const int64_t nblk_c = std::max<int64_t>(1, ceil_div(E, kCpTile));
  hipLaunchKernelGGL(k_vis_count, dim3((unsigned)nblk_c), dim3(256), 0, s, proj.radius, E, w.flags);
  int st = device_scan(w.flags, w.flags, nullptr, nblk_c, nblk_c, w.partial, n_vis, s);
  if (st) return st;
  hipLaunchKernelGGL(k_compact, dim3((unsigned)nblk_c), dim3(256), 0, s, cfg, proj.radius, proj.depth, proj.rec, items,
                     E, n, cnt_shift, w.flags, w.vkeys[0], w.vvals[0]);
  // 2. stable sort of the visible entries by (item, depth)
  int fin = 0;
  st = radix_sort<uint64_t>(w.vkeys[0], w.vkeys[1], w.vvals[0], w.vvals[1], n_vis, E, kbits, w, s, &fin);
  if (st) return st;
  const uint32_t* svals = w.vvals[fin];
  // 3. duplicates in depth order
  if (cnt_shift > 0)
    hipLaunchKernelGGL(k_touched_keys, dim3(eb), dim3(256), 0, s, w.vkeys[fin], n_vis, cnt_shift, w.touched);
  else
    hipLaunchKernelGGL(k_touched, dim3(eb), dim3(256), 0, s, cfg, svals, n_vis, proj.rec, proj.radius, items, n,
                       w.touched);
  st = device_scan(w.touched, w.touched, n_vis, 0, E, w.partial, d_total, s);
  if (st) return st;
  // the tile sort must end in the caller's vals: start there after an even pass count
  const int tbits = std::max(1, bits_for((uint64_t)n_tiles));
  const int passes = radix_passes(tbits);
  uint32_t* v_first = (passes % 2 == 0) ? vals : w.tvals;
  uint32_t* v_other = (passes % 2 == 0) ? w.tvals : vals;
  hipLaunchKernelGGL(k_duplicate, dim3((unsigned)std::max<int64_t>(1, ceil_div(E, 256))), dim3(256), 0, s, cfg, svals,
                     n_vis, w.touched, proj.rec, proj.radius, items, n, cap, w.tkeys[0], v_first, d_total, d_live,
                     n_dup_dev, status_dev, ranges, 2ll * n_tiles);
  // 4. stable sort of the duplicates by tile
  st = radix_sort<uint32_t>(w.tkeys[0], w.tkeys[1], v_first, v_other, d_live, cap, tbits, w, s, &fin);
  if (st) return st;
  const uint32_t* tk = w.tkeys[fin];
  // 5. tile ranges
  const unsigned cb = (unsigned)std::max<int64_t>(1, ceil_div(cap, 256));
  hipLaunchKernelGGL(k_ranges, dim3(cb), dim3(256), 0, s, tk, d_live, ranges);
  if (keys)
    hipLaunchKernelGGL(k_full_keys, dim3(cb), dim3(256), 0, s, tk, vals, d_live, proj.depth, items, n_items, n, keys);
  return launch_status();
}

}  // namespace gs
