// View-dependent features by spherical harmonics (paper Sec. III-B: each Gaussian's colour
// and semantic features are represented with SH). Per view v, Gaussian i and channel c,
//   f_vic = dc_ic + sum_{1 <= j < (degree+1)^2} Y_j(d_vi) k_ijc,
// d_vi = (mu_i - c_v) / |mu_i - c_v|, c_v = -R_v^T t_v the camera centre, Y_j the real
// spherical harmonics (index j = l^2 + l + m, the sign convention of the 3DGS renderer).
// The constant band is the plain feature, so degree 0 reproduces view-independent features.
//
// The forward writes one feature block per view for the render kernels (cfg.view_features).
// The backward takes the render's per-view feature gradients back to the constant band, the
// coefficients, the means (through d) and each view's pose (through c_v, which moves by
// -R^T rho under T_cw <- Exp(xi) T_cw and not with phi).
#include <math.h>

#include "common.h"

namespace gs {
namespace {

constexpr double kPiD = 3.14159265358979323846;
constexpr double csqrt(double x) {   // Newton's iteration, for the constants below
  double r = x > 1.0 ? x : 1.0;
  for (int k = 0; k < 100; ++k) r = 0.5 * (r + x / r);
  return r;
}
constexpr float kC1 = (float)csqrt(3.0 / (4.0 * kPiD));
constexpr float kC2a = (float)(csqrt(15.0 / kPiD) / 2.0);   // xy, -yz, -xz
constexpr float kC2b = (float)(csqrt(5.0 / kPiD) / 4.0);    // 2zz - xx - yy
constexpr float kC2c = (float)(csqrt(15.0 / kPiD) / 4.0);   // xx - yy
constexpr float kC3a = (float)(csqrt(35.0 / (2.0 * kPiD)) / 4.0);
constexpr float kC3b = (float)(csqrt(105.0 / kPiD) / 2.0);
constexpr float kC3c = (float)(csqrt(21.0 / (2.0 * kPiD)) / 4.0);
constexpr float kC3d = (float)(csqrt(7.0 / kPiD) / 4.0);
constexpr float kC3e = (float)(csqrt(105.0 / kPiD) / 4.0);

// Y_1 .. Y_{K-1} at the unit direction (x, y, z).
__device__ __forceinline__ void sh_basis(float x, float y, float z, int deg, float* Y) {
  if (deg < 1) return;
  Y[1] = -kC1 * y;
  Y[2] = kC1 * z;
  Y[3] = -kC1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kC2a * x * y;
  Y[5] = -kC2a * y * z;
  Y[6] = kC2b * (2.0f * zz - xx - yy);
  Y[7] = -kC2a * x * z;
  Y[8] = kC2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -kC3a * y * (3.0f * xx - yy);
  Y[10] = kC3b * x * y * z;
  Y[11] = -kC3c * y * (4.0f * zz - xx - yy);
  Y[12] = kC3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -kC3c * x * (4.0f * zz - xx - yy);
  Y[14] = kC3e * z * (xx - yy);
  Y[15] = -kC3a * x * (xx - 3.0f * yy);
}

// sum_j a_j dY_j/dd (the polynomials' gradient in the ambient coordinates), j >= 1.
__device__ __forceinline__ void sh_grad_dot(float x, float y, float z, int deg, const float* a, float& gx, float& gy,
                                            float& gz) {
  gx = gy = gz = 0.0f;
  if (deg < 1) return;
  gy += -kC1 * a[1];
  gz += kC1 * a[2];
  gx += -kC1 * a[3];
  if (deg < 2) return;
  gx += kC2a * y * a[4];
  gy += kC2a * x * a[4];
  gy += -kC2a * z * a[5];
  gz += -kC2a * y * a[5];
  gx += -2.0f * kC2b * x * a[6];
  gy += -2.0f * kC2b * y * a[6];
  gz += 4.0f * kC2b * z * a[6];
  gx += -kC2a * z * a[7];
  gz += -kC2a * x * a[7];
  gx += 2.0f * kC2c * x * a[8];
  gy += -2.0f * kC2c * y * a[8];
  if (deg < 3) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx += -kC3a * 6.0f * x * y * a[9];
  gy += -kC3a * (3.0f * xx - 3.0f * yy) * a[9];
  gx += kC3b * y * z * a[10];
  gy += kC3b * x * z * a[10];
  gz += kC3b * x * y * a[10];
  gx += -kC3c * (-2.0f * x * y) * a[11];
  gy += -kC3c * (4.0f * zz - xx - 3.0f * yy) * a[11];
  gz += -kC3c * 8.0f * y * z * a[11];
  gx += kC3d * (-6.0f * x * z) * a[12];
  gy += kC3d * (-6.0f * y * z) * a[12];
  gz += kC3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * a[12];
  gx += -kC3c * (4.0f * zz - 3.0f * xx - yy) * a[13];
  gy += -kC3c * (-2.0f * x * y) * a[13];
  gz += -kC3c * 8.0f * x * z * a[13];
  gx += kC3e * 2.0f * x * z * a[14];
  gy += kC3e * (-2.0f * y * z) * a[14];
  gz += kC3e * (xx - yy) * a[14];
  gx += -kC3a * (3.0f * xx - 3.0f * yy) * a[15];
  gy += -kC3a * (-6.0f * x * y) * a[15];
}

// Lane mapping of both kernels: each Gaussian takes an aligned group of `gsz` lanes (the
// channel count 3 + n_sem <= 63 rounded up to a power of two), its channels on consecutive
// lanes, so loads and stores of a Gaussian's channels are contiguous and a reduction over
// them is a butterfly within the group.
__device__ __forceinline__ int group_size(int ct) {
  int g = 1;
  while (g < ct) g <<= 1;
  return g;
}

constexpr int kViewChunk = 256;   // camera centres staged in LDS per pass over the views

__device__ __forceinline__ void stage_centres(const gs_view* __restrict__ views, int v0, int nv, float* s_c) {
  for (int k = threadIdx.x; k < nv; k += blockDim.x) {
    const gs_view V = views[v0 + k];
    for (int a = 0; a < 3; ++a)
      s_c[3 * k + a] = -(V.R[a] * V.t[0] + V.R[3 + a] * V.t[1] + V.R[6 + a] * V.t[2]);
  }
}

// Channel c of Gaussian i: the constant band, the degree and the coefficient walk of its
// feature array (rgb: c < 3; semantics: c >= 3).
struct ShChan {
  const float* rest;   // first coefficient of the channel, or null
  int stride, deg;
  float dc;
};

__device__ __forceinline__ ShChan sh_chan(const gs_gaussians& g, const gs_sh& sh, int n_sem, int64_t i, int c) {
  ShChan h;
  const bool rgb = c < 3;
  const int ch = rgb ? 3 : n_sem;
  const int k = rgb ? c : c - 3;
  h.deg = rgb ? sh.rgb_degree : sh.sem_degree;
  h.dc = rgb ? g.rgb[3 * i + k] : g.sem[(int64_t)n_sem * i + k];
  const int nk = (h.deg + 1) * (h.deg + 1) - 1;
  const float* base = rgb ? sh.rgb_rest : sh.sem_rest;
  h.rest = (h.deg > 0) ? base + ((int64_t)i * nk) * ch + k : nullptr;
  h.stride = ch;
  return h;
}

__global__ __launch_bounds__(256) void k_sh_fwd(gs_gaussians g, gs_sh sh, int n_sem, const gs_view* __restrict__ views,
                                                int n_views, float* __restrict__ rgb_out, float* __restrict__ sem_out) {
  __shared__ float s_c[3 * kViewChunk];
  const int Ct = 3 + n_sem, gsz = group_size(Ct);
  const int64_t i0 = (int64_t)blockIdx.x * (256 / gsz) + threadIdx.x / gsz;
  const int c0 = (int)(threadIdx.x % gsz);
  const bool live = i0 < g.n && c0 < Ct;
  const int64_t i = live ? i0 : 0;
  const int c = live ? c0 : 0;
  ShChan h{};
  float coef[16];
  float mx = 0.0f, my = 0.0f, mz = 0.0f;
  if (live) {
    h = sh_chan(g, sh, n_sem, i, c);
    const int K = (h.deg + 1) * (h.deg + 1);
#pragma unroll
    for (int j = 1; j < 16; ++j) coef[j] = j < K ? h.rest[(int64_t)(j - 1) * h.stride] : 0.0f;
    mx = g.mean[3 * i];
    my = g.mean[3 * i + 1];
    mz = g.mean[3 * i + 2];
  }
  for (int v0 = 0; v0 < n_views; v0 += kViewChunk) {
    const int nv = min(kViewChunk, n_views - v0);
    __syncthreads();
    stage_centres(views, v0, nv, s_c);
    __syncthreads();
    if (!live) continue;
    for (int k = 0; k < nv; ++k) {
      float f = h.dc;
      if (h.deg > 0) {
        const float ux = mx - s_c[3 * k], uy = my - s_c[3 * k + 1], uz = mz - s_c[3 * k + 2];
        const float ir = rsqrtf(ux * ux + uy * uy + uz * uz);
        float Y[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) Y[j] = 0.0f;
        sh_basis(ux * ir, uy * ir, uz * ir, h.deg, Y);
#pragma unroll
        for (int j = 1; j < 16; ++j) f = fmaf(Y[j], coef[j], f);
      }
      const int64_t v = v0 + k;
      if (c < 3) rgb_out[(v * g.n + i) * 3 + c] = f;
      else sem_out[(v * g.n + i) * n_sem + (c - 3)] = f;
    }
  }
}

// The backward, one lane per (Gaussian, channel), persistent blocks of 256 lanes walking the
// Gaussians: the constant band and the bands sum the feature gradient (times Y_j) over views;
// the channel's share of d L/d d, g_c sum_j k_jc dY_j/dd, goes through the normalisation
// (linear, so channels can be summed in any order) to the mean, summed over the Gaussian's
// lane group by a butterfly, and to the pose's rho (gpose[v][0..2] += R_v sum). Views are
// taken kPoseViews at a time: each lane keeps that many rho sums in registers over all its
// Gaussians, so a block adds to each pose once per chunk (a grid of few blocks keeps those
// same-address atomics few). The bands of a later chunk are added to the first chunk's.
constexpr int kPoseViews = 4;
constexpr int kShBwdThreads = 256;

// What one lane reads for one Gaussian: its channel's bands, the mean, the feature gradient
// of each view of the chunk.
struct ShIn {
  float coef[16];
  float m[3];
  float gm0[3];   // the mean gradient so far (read by the lane that adds to it, the only writer)
  float gf[kPoseViews];
};

__device__ __forceinline__ void sh_load(const gs_gaussians& g, const gs_sh& sh, int n_sem, int64_t i, int c, bool live,
                                        int v0, int nv, const float* __restrict__ grgb,
                                        const float* __restrict__ gsem, const float* gmean, ShIn& in) {
  const bool rgb = c < 3;
  const int ch = rgb ? 3 : n_sem, kc = rgb ? c : c - 3;
  const int deg = rgb ? sh.rgb_degree : sh.sem_degree;
  const int K = (deg + 1) * (deg + 1);
  const float* rest = rgb ? sh.rgb_rest : sh.sem_rest;
  const float* r = (live && deg > 0) ? rest + (int64_t)i * (K - 1) * ch + kc : nullptr;
#pragma unroll
  for (int j = 0; j < 16; ++j) in.coef[j] = (r && j >= 1 && j < K) ? r[(int64_t)(j - 1) * ch] : 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) in.m[a] = live ? g.mean[3 * i + a] : 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) in.gm0[a] = (live && c == 0 && gmean) ? gmean[3 * i + a] : 0.0f;
#pragma unroll
  for (int k = 0; k < kPoseViews; ++k) {
    const int64_t v = v0 + k;
    in.gf[k] = (live && k < nv) ? (rgb ? grgb[(v * g.n + i) * 3 + c] : gsem[(v * g.n + i) * n_sem + kc]) : 0.0f;
  }
}

__global__ __launch_bounds__(kShBwdThreads) void k_sh_bwd(gs_gaussians g, gs_sh sh, int n_sem,
                                                          const gs_view* __restrict__ views, int n_views,
                                                          const float* __restrict__ grgb,
                                                          const float* __restrict__ gsem, float* __restrict__ gdc_rgb,
                                                          float* __restrict__ grest_rgb, float* __restrict__ gdc_sem,
                                                          float* __restrict__ grest_sem, float* __restrict__ gmean,
                                                          float* __restrict__ gpose) {
  __shared__ double red[kShBwdThreads / 64][3 * kPoseViews];
  const int Ct = 3 + n_sem, gsz = group_size(Ct);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int per_block = kShBwdThreads / gsz;          // Gaussians per block and pass
  const int64_t step = (int64_t)gridDim.x * per_block;
  const int c0 = tid % gsz;
  const int c = c0 < Ct ? c0 : 0;
  const bool rgb = c < 3;
  const int ch = rgb ? 3 : n_sem, kc = rgb ? c : c - 3;
  const int deg = rgb ? sh.rgb_degree : sh.sem_degree;
  const int nk = (deg + 1) * (deg + 1);
  const bool any_dir = sh.rgb_degree > 0 || sh.sem_degree > 0;
  for (int v0 = 0; v0 < n_views; v0 += kPoseViews) {
    const int nv = min(kPoseViews, n_views - v0);
    float pr[kPoseViews][3];
#pragma unroll
    for (int k = 0; k < kPoseViews; ++k) pr[k][0] = pr[k][1] = pr[k][2] = 0.0f;
    float Rv[kPoseViews][9], cv[kPoseViews][3];   // the chunk's rotations and camera centres
#pragma unroll
    for (int k = 0; k < kPoseViews; ++k) {
      const gs_view V = views[v0 + min(k, nv - 1)];
#pragma unroll
      for (int e = 0; e < 9; ++e) Rv[k][e] = V.R[e];
#pragma unroll
      for (int a = 0; a < 3; ++a) cv[k][a] = -(V.R[a] * V.t[0] + V.R[3 + a] * V.t[1] + V.R[6 + a] * V.t[2]);
    }
    int64_t gb = (int64_t)blockIdx.x * per_block;
    ShIn cur;
    {
      const int64_t i0 = gb + tid / gsz;
      const bool live = i0 < g.n && c0 < Ct;
      sh_load(g, sh, n_sem, live ? i0 : 0, c, live && c0 < Ct, v0, nv, grgb, gsem, any_dir ? gmean : nullptr, cur);
    }
    for (; gb < g.n; gb += step) {
      const int64_t i0 = gb + tid / gsz;
      const bool live = i0 < g.n && c0 < Ct;
      const int64_t i = live ? i0 : 0;
      ShIn nxt;                               // the next Gaussian's inputs, in flight meanwhile
      {
        const int64_t j0 = gb + step + tid / gsz;
        const bool nlive = j0 < g.n && c0 < Ct;
        sh_load(g, sh, n_sem, nlive ? j0 : 0, c, nlive, v0, nv, grgb, gsem, any_dir ? gmean : nullptr, nxt);
      }
      float acc[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
      float gm[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < kPoseViews; ++k) {
        const float gf = cur.gf[k];
        acc[0] += gf;
        if (deg == 0 || gf == 0.0f) continue;
        const float ux = cur.m[0] - cv[k][0], uy = cur.m[1] - cv[k][1], uz = cur.m[2] - cv[k][2];
        const float ir = rsqrtf(ux * ux + uy * uy + uz * uz);
        const float dx = ux * ir, dy = uy * ir, dz = uz * ir;
        float Y[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) Y[j] = 0.0f;
        sh_basis(dx, dy, dz, deg, Y);
#pragma unroll
        for (int j = 1; j < 16; ++j) acc[j] = fmaf(Y[j], gf, acc[j]);
        float gx, gy, gz;   // sum_j k_jc dY_j/dd, times g_c below (linear in g_c)
        sh_grad_dot(dx, dy, dz, deg, cur.coef, gx, gy, gz);
        const float dd = dx * gx + dy * gy + dz * gz;
        const float gi = gf * ir;
        const float u0 = (gx - dx * dd) * gi, u1 = (gy - dy * dd) * gi, u2 = (gz - dz * dd) * gi;
        gm[0] += u0;
        gm[1] += u1;
        gm[2] += u2;
        // rho: R_v (d L/d mu), the camera centre -R^T t moving by -R^T rho
        pr[k][0] += Rv[k][0] * u0 + Rv[k][1] * u1 + Rv[k][2] * u2;
        pr[k][1] += Rv[k][3] * u0 + Rv[k][4] * u1 + Rv[k][5] * u2;
        pr[k][2] += Rv[k][6] * u0 + Rv[k][7] * u1 + Rv[k][8] * u2;
      }
      if (live) {
        float* gdc = rgb ? gdc_rgb : gdc_sem;
        float* grest = rgb ? grest_rgb : grest_sem;
        // the first chunk of views stores, later chunks add (no read before the first store)
        if (gdc) {
          float* o = gdc + (int64_t)ch * i + kc;
          if (v0 == 0) *o = acc[0];
          else *o += acc[0];
        }
        if (deg > 0 && grest) {
          float* o = grest + (int64_t)i * (nk - 1) * ch + kc;
          if (v0 == 0) {
#pragma unroll
            for (int j = 1; j < 16; ++j)
              if (j < nk) o[(int64_t)(j - 1) * ch] = acc[j];
          } else {
#pragma unroll
            for (int j = 1; j < 16; ++j)
              if (j < nk) o[(int64_t)(j - 1) * ch] += acc[j];
          }
        }
      }
      if (any_dir) {   // the mean's share over the Gaussian's channels, added by the group's first lane
        for (int o = 1; o < gsz; o <<= 1)
          for (int k = 0; k < 3; ++k) gm[k] += __shfl_xor(gm[k], o, 64);
        if (live && c0 == 0)
          for (int k = 0; k < 3; ++k) gmean[3 * i + k] = cur.gm0[k] + gm[k];
      }
      cur = nxt;
    }
    if (any_dir) {   // the chunk's rho sums: one block reduction, one atomic per (view, component)
#pragma unroll
      for (int k = 0; k < kPoseViews; ++k)
        for (int a = 0; a < 3; ++a) {
          const double sum = wave_sum_d((double)pr[k][a]);
          if (lane == 0) red[wid][3 * k + a] = sum;
        }
      __syncthreads();
      if (tid < 3 * nv) {
        double S = 0.0;
        for (int w = 0; w < kShBwdThreads / 64; ++w) S += red[w][tid];
        if (S != 0.0) atomicAdd(gpose + 6 * (v0 + tid / 3) + tid % 3, (float)S);
      }
      __syncthreads();
    }
  }
}

}  // namespace

int launch_sh_fwd(const gs_gaussians& g, const gs_sh& sh, int n_sem, const gs_view* views, int n_views, float* rgb_out,
                  float* sem_out, hipStream_t s) {
  const int64_t work = g.n * (3 + n_sem);
  if (work == 0 || n_views == 0) return GS_OK;
  int gsz = 1;
  while (gsz < 3 + n_sem) gsz <<= 1;
  hipLaunchKernelGGL(k_sh_fwd, dim3((unsigned)ceil_div(g.n, 256 / gsz)), dim3(256), 0, s, g, sh, n_sem, views,
                     n_views, rgb_out, sem_out);
  return launch_status();
}

int launch_sh_bwd(const gs_gaussians& g, const gs_sh& sh, int n_sem, const gs_view* views, int n_views,
                  const float* grgb, const float* gsem, float* gdc_rgb, float* grest_rgb, float* gdc_sem,
                  float* grest_sem, float* gmean, float* gpose, hipStream_t s) {
  if (g.n == 0 || n_views == 0) return GS_OK;
  int gsz = 1;
  while (gsz < 3 + n_sem) gsz <<= 1;
  // a few blocks per CU: enough lanes in flight, few same-address atomics on the poses
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  const int64_t blocks = std::min<int64_t>(ceil_div(g.n, kShBwdThreads / gsz), 4 * (int64_t)cus);
  hipLaunchKernelGGL(k_sh_bwd, dim3((unsigned)blocks), dim3(kShBwdThreads), 0, s, g, sh, n_sem, views, n_views, grgb,
                     gsem, gdc_rgb, grest_rgb, gdc_sem, grest_sem, gmean, gpose);
  return launch_status();
}

}  // namespace gs
