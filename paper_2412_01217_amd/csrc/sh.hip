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
  const int Ct = 3 + n_sem;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < g.n * Ct;
  const int64_t i = live ? t / Ct : 0;
  const int c = live ? (int)(t - i * Ct) : 0;
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

// Constant band and coefficients: sums over views of the feature gradient (times Y_j).
__global__ __launch_bounds__(256) void k_sh_bwd_coef(gs_gaussians g, gs_sh sh, int n_sem,
                                                     const gs_view* __restrict__ views, int n_views,
                                                     const float* __restrict__ grgb, const float* __restrict__ gsem,
                                                     float* __restrict__ gdc_rgb, float* __restrict__ grest_rgb,
                                                     float* __restrict__ gdc_sem, float* __restrict__ grest_sem) {
  __shared__ float s_c[3 * kViewChunk];
  const int Ct = 3 + n_sem;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < g.n * Ct;
  const int64_t i = live ? t / Ct : 0;
  const int c = live ? (int)(t - i * Ct) : 0;
  const bool rgb = c < 3;
  const int deg = rgb ? sh.rgb_degree : sh.sem_degree;
  const int nk = (deg + 1) * (deg + 1);
  float acc[16];
  for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
  const float mx = live ? g.mean[3 * i] : 0.0f, my = live ? g.mean[3 * i + 1] : 0.0f;
  const float mz = live ? g.mean[3 * i + 2] : 0.0f;
  for (int v0 = 0; v0 < n_views; v0 += kViewChunk) {
    const int nv = min(kViewChunk, n_views - v0);
    __syncthreads();
    stage_centres(views, v0, nv, s_c);
    __syncthreads();
    if (!live) continue;
    for (int k = 0; k < nv; ++k) {
      const int64_t v = v0 + k;
      const float gf = rgb ? grgb[(v * g.n + i) * 3 + c] : gsem[(v * g.n + i) * n_sem + (c - 3)];
      acc[0] += gf;
      if (deg > 0) {
        const float ux = mx - s_c[3 * k], uy = my - s_c[3 * k + 1], uz = mz - s_c[3 * k + 2];
        const float ir = rsqrtf(ux * ux + uy * uy + uz * uz);
        float Y[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) Y[j] = 0.0f;
        sh_basis(ux * ir, uy * ir, uz * ir, deg, Y);
#pragma unroll
        for (int j = 1; j < 16; ++j) acc[j] = fmaf(Y[j], gf, acc[j]);
      }
    }
  }
  if (!live) return;
  const int ch = rgb ? 3 : n_sem, kc = rgb ? c : c - 3;
  float* gdc = rgb ? gdc_rgb : gdc_sem;
  float* grest = rgb ? grest_rgb : grest_sem;
  if (gdc) gdc[(int64_t)ch * i + kc] = acc[0];
  if (deg > 0 && grest) {
#pragma unroll
    for (int j = 1; j < 16; ++j)
      if (j < nk) grest[((int64_t)i * (nk - 1) + (j - 1)) * ch + kc] = acc[j];
  }
}

// Direction: d L/d d = sum_c g_c sum_j k_jc dY_j/dd, through the normalisation to the mean
// (added to gmean) and, summed over the block, to the pose's rho (gpose[v][0..2] += R_v sum).
__global__ __launch_bounds__(256) void k_sh_bwd_dir(gs_gaussians g, gs_sh sh, int n_sem,
                                                    const gs_view* __restrict__ views, int n_views,
                                                    const float* __restrict__ grgb, const float* __restrict__ gsem,
                                                    float* __restrict__ gmean, float* __restrict__ gpose) {
  __shared__ double red[4][3];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < g.n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const float mx = live ? g.mean[3 * i] : 0.0f, my = live ? g.mean[3 * i + 1] : 0.0f;
  const float mz = live ? g.mean[3 * i + 2] : 0.0f;
  double am[3] = {0, 0, 0};
  const int nkr = (sh.rgb_degree + 1) * (sh.rgb_degree + 1) - 1, nks = (sh.sem_degree + 1) * (sh.sem_degree + 1) - 1;
  for (int v = 0; v < n_views; ++v) {
    const gs_view V = views[v];
    double gu[3] = {0, 0, 0};
    if (live) {
      float cc[3];
      for (int a = 0; a < 3; ++a) cc[a] = -(V.R[a] * V.t[0] + V.R[3 + a] * V.t[1] + V.R[6 + a] * V.t[2]);
      const float ux = mx - cc[0], uy = my - cc[1], uz = mz - cc[2];
      const float ir = rsqrtf(ux * ux + uy * uy + uz * uz);
      const float dx = ux * ir, dy = uy * ir, dz = uz * ir;
      float gd[3] = {0.0f, 0.0f, 0.0f};
      for (int part = 0; part < 2; ++part) {
        const int deg = part == 0 ? sh.rgb_degree : sh.sem_degree;
        if (deg == 0) continue;
        const int ch = part == 0 ? 3 : n_sem, nk = part == 0 ? nkr : nks;
        const float* rest = (part == 0 ? sh.rgb_rest : sh.sem_rest) + (int64_t)i * nk * ch;
        const float* gf = part == 0 ? grgb + ((int64_t)v * g.n + i) * 3 : gsem + ((int64_t)v * g.n + i) * n_sem;
        float a[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) a[j] = 0.0f;
        for (int k = 0; k < ch; ++k) {
          const float gk = gf[k];
          if (gk == 0.0f) continue;
#pragma unroll
          for (int j = 1; j < 16; ++j)
            if (j <= nk) a[j] = fmaf(gk, rest[(j - 1) * ch + k], a[j]);
        }
        float gx, gy, gz;
        sh_grad_dot(dx, dy, dz, deg, a, gx, gy, gz);
        gd[0] += gx;
        gd[1] += gy;
        gd[2] += gz;
      }
      const float dd = dx * gd[0] + dy * gd[1] + dz * gd[2];
      gu[0] = (double)((gd[0] - dx * dd) * ir);
      gu[1] = (double)((gd[1] - dy * dd) * ir);
      gu[2] = (double)((gd[2] - dz * dd) * ir);
      for (int a = 0; a < 3; ++a) am[a] += gu[a];
    }
    // pose: c_v = -R^T t moves by -R^T rho, so d L/d rho = R sum_i d L/d mu (direction part)
    for (int a = 0; a < 3; ++a) {
      const double s = wave_sum_d(gu[a]);
      if (lane == 0) red[wid][a] = s;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      double S[3];
      for (int a = 0; a < 3; ++a) S[a] = red[0][a] + red[1][a] + red[2][a] + red[3][a];
      const int r = threadIdx.x;
      const double p = V.R[3 * r] * S[0] + V.R[3 * r + 1] * S[1] + V.R[3 * r + 2] * S[2];
      if (p != 0.0) atomicAdd(gpose + 6 * v + r, (float)p);
    }
    __syncthreads();
  }
  if (!live) return;
  for (int a = 0; a < 3; ++a) gmean[3 * i + a] += (float)am[a];
}

}  // namespace

int launch_sh_fwd(const gs_gaussians& g, const gs_sh& sh, int n_sem, const gs_view* views, int n_views, float* rgb_out,
                  float* sem_out, hipStream_t s) {
  const int64_t work = g.n * (3 + n_sem);
  if (work == 0 || n_views == 0) return GS_OK;
  hipLaunchKernelGGL(k_sh_fwd, dim3((unsigned)ceil_div(work, 256)), dim3(256), 0, s, g, sh, n_sem, views, n_views,
                     rgb_out, sem_out);
  return launch_status();
}

int launch_sh_bwd(const gs_gaussians& g, const gs_sh& sh, int n_sem, const gs_view* views, int n_views,
                  const float* grgb, const float* gsem, float* gdc_rgb, float* grest_rgb, float* gdc_sem,
                  float* grest_sem, float* gmean, float* gpose, hipStream_t s) {
  const int64_t work = g.n * (3 + n_sem);
  if (work == 0) return GS_OK;
  hipLaunchKernelGGL(k_sh_bwd_coef, dim3((unsigned)ceil_div(work, 256)), dim3(256), 0, s, g, sh, n_sem, views, n_views,
                     grgb, gsem, gdc_rgb, grest_rgb, gdc_sem, grest_sem);
  if ((sh.rgb_degree > 0 || sh.sem_degree > 0) && n_views > 0)
    hipLaunchKernelGGL(k_sh_bwd_dir, dim3((unsigned)ceil_div(g.n, 256)), dim3(256), 0, s, g, sh, n_sem, views, n_views,
                       grgb, gsem, gmean, gpose);
  return launch_status();
}

}  // namespace gs
