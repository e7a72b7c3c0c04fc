// Mapping update after back-propagation (paper Sec. III-D): Adam (Kingma and Ba 2015,
// Algorithm 1) on every Gaussian parameter group in one launch, and on each camera pose's
// tangent, the pose then moved by the left-multiplied SE(3) exponential.
//
// The parameter update is elementwise and bound by HBM traffic (4 reads, 3 writes of 4
// bytes per element): each thread takes 4 consecutive elements of one group, as 16-byte
// vector accesses where the group's arrays allow it.
#include <math.h>

#include "common.h"

namespace gs {
namespace {

constexpr int kGroups = 6;

struct AdamGroups {
  float* p[kGroups];
  const float* g[kGroups];
  float* m[kGroups];
  float* v[kGroups];
  int64_t n[kGroups];
  int64_t quad_end[kGroups];   // running totals of ceil(n / 4)
  float lr[kGroups];
  int vec[kGroups];            // 1: all four arrays 16-byte aligned
};

__device__ __forceinline__ void adam1(float& p, float g, float& m, float& v, float lr, float b1, float b2, float eps,
                                      float c1, float c2) {
  m = b1 * m + (1.0f - b1) * g;
  v = b2 * v + (1.0f - b2) * g * g;
  p = p - lr * (m * c1) / (sqrtf(v * c2) + eps);
}

__global__ __launch_bounds__(256) void k_adam_groups(AdamGroups a, float b1, float b2, float eps, float c1, float c2) {
  const int64_t total = a.quad_end[kGroups - 1];
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    int k = 0;
#pragma unroll
    for (int j = 0; j < kGroups - 1; ++j) k += q >= a.quad_end[j];
    const int64_t lq = q - (k > 0 ? a.quad_end[k - 1] : 0);
    const int64_t i0 = 4 * lq;
    const float lr = a.lr[k];
    float* P = a.p[k];
    const float* G = a.g[k];
    float* M = a.m[k];
    float* V = a.v[k];
    if (a.vec[k] && i0 + 4 <= a.n[k]) {
      float4 p = *(const float4*)(P + i0), g = *(const float4*)(G + i0);
      float4 m = *(const float4*)(M + i0), v = *(const float4*)(V + i0);
      adam1(p.x, g.x, m.x, v.x, lr, b1, b2, eps, c1, c2);
      adam1(p.y, g.y, m.y, v.y, lr, b1, b2, eps, c1, c2);
      adam1(p.z, g.z, m.z, v.z, lr, b1, b2, eps, c1, c2);
      adam1(p.w, g.w, m.w, v.w, lr, b1, b2, eps, c1, c2);
      *(float4*)(P + i0) = p;
      *(float4*)(M + i0) = m;
      *(float4*)(V + i0) = v;
    } else {
      const int64_t e = min(i0 + 4, a.n[k]);
      for (int64_t i = i0; i < e; ++i) {
        float p = P[i], m = M[i], v = V[i];
        adam1(p, G[i], m, v, lr, b1, b2, eps, c1, c2);
        P[i] = p;
        M[i] = m;
        V[i] = v;
      }
    }
  }
}

// Exp of the tangent (rho, phi) in double precision: R = I + s K + c K^2, t = (I + c K + d K^2) rho,
// K = [phi]x, a = |phi|, s = sin a / a, c = (1 - cos a) / a^2 = 2 sin^2(a/2) / a^2,
// d = (a - sin a) / a^3 (its Taylor series below a = 0.1, where the difference cancels).
__device__ void exp_se3(const double xi[6], double R[9], double t[3]) {
  const double w0 = xi[3], w1 = xi[4], w2 = xi[5];
  const double a2 = w0 * w0 + w1 * w1 + w2 * w2, a = sqrt(a2);
  double s, c, d;
  if (a == 0.0) {
    s = 1.0;
    c = 0.5;
    d = 1.0 / 6.0;
  } else {
    s = sin(a) / a;
    const double h = sin(0.5 * a);
    c = 2.0 * h * h / a2;
    d = a < 0.1 ? 1.0 / 6.0 - a2 / 120.0 + a2 * a2 / 5040.0 - a2 * a2 * a2 / 362880.0 : (a - sin(a)) / (a2 * a);
  }
  const double K[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
  double V[9];
  for (int e = 0; e < 9; ++e) {
    const double I = (e % 4 == 0) ? 1.0 : 0.0;
    R[e] = I + s * K[e] + c * K2[e];
    V[e] = I + c * K[e] + d * K2[e];
  }
  for (int i = 0; i < 3; ++i) t[i] = V[3 * i] * xi[0] + V[3 * i + 1] * xi[1] + V[3 * i + 2] * xi[2];
}

// One thread per view: Adam on the 6 tangent components, then T_cw <- Exp(delta) T_cw, the
// product's rows re-orthonormalised (Gram-Schmidt, double precision) before they are
// stored in single precision, so that rounding does not accumulate over many steps.
__global__ void k_pose_adam(gs_view* __restrict__ views, int n_views, const float* __restrict__ grad,
                            float* __restrict__ m, float* __restrict__ v, float lr_rho, float lr_phi, float b1,
                            float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_views) return;
  double xi[6];
  for (int k = 0; k < 6; ++k) {
    float p = 0.0f, mk = m[6 * i + k], vk = v[6 * i + k];
    adam1(p, grad[6 * i + k], mk, vk, k < 3 ? lr_rho : lr_phi, b1, b2, eps, c1, c2);
    m[6 * i + k] = mk;
    v[6 * i + k] = vk;
    xi[k] = (double)p;
  }
  double Rd[9], td[3];
  exp_se3(xi, Rd, td);
  gs_view& vw = views[i];
  double R0[9], t0[3], R[9], t[3];
  for (int e = 0; e < 9; ++e) R0[e] = (double)vw.R[e];
  for (int e = 0; e < 3; ++e) t0[e] = (double)vw.t[e];
  for (int r = 0; r < 3; ++r) {
    for (int cc = 0; cc < 3; ++cc) R[3 * r + cc] = Rd[3 * r] * R0[cc] + Rd[3 * r + 1] * R0[3 + cc] + Rd[3 * r + 2] * R0[6 + cc];
    t[r] = Rd[3 * r] * t0[0] + Rd[3 * r + 1] * t0[1] + Rd[3 * r + 2] * t0[2] + td[r];
  }
  // rows: r0 normalised, r1 made orthogonal to r0 and normalised, r2 = r0 x r1
  double* r0 = R;
  double* r1 = R + 3;
  double* r2 = R + 6;
  double n0 = rsqrt(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
  for (int e = 0; e < 3; ++e) r0[e] *= n0;
  const double dp = r0[0] * r1[0] + r0[1] * r1[1] + r0[2] * r1[2];
  for (int e = 0; e < 3; ++e) r1[e] -= dp * r0[e];
  const double n1 = rsqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
  for (int e = 0; e < 3; ++e) r1[e] *= n1;
  r2[0] = r0[1] * r1[2] - r0[2] * r1[1];
  r2[1] = r0[2] * r1[0] - r0[0] * r1[2];
  r2[2] = r0[0] * r1[1] - r0[1] * r1[0];
  for (int e = 0; e < 9; ++e) vw.R[e] = (float)R[e];
  for (int e = 0; e < 3; ++e) vw.t[e] = (float)t[e];
}

// T_cw <- Exp(xi) T_cw for a pose tangent xi = (rho, phi) at a nonzero point: the product in
// double precision, rounded once (no re-orthonormalisation, so that the result is the smooth
// function of xi whose derivative k_pose_perturb_bwd gives).
__global__ void k_pose_perturb(const gs_view* __restrict__ vin, int n_views, const float* __restrict__ xi_in,
                               gs_view* vout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_views) return;
  double xi[6];
  for (int k = 0; k < 6; ++k) xi[k] = (double)xi_in[6 * i + k];
  double Rd[9], td[3];
  exp_se3(xi, Rd, td);
  const gs_view v0 = vin[i];
  gs_view v1 = v0;
  for (int r = 0; r < 3; ++r) {
    double t = td[r];
    for (int cc = 0; cc < 3; ++cc) {
      double a = 0.0;
      for (int k = 0; k < 3; ++k) a += Rd[3 * r + k] * (double)v0.R[3 * k + cc];
      v1.R[3 * r + cc] = (float)a;
      t += Rd[3 * r + cc] * (double)v0.t[cc];
    }
    v1.t[r] = (float)t;
  }
  vout[i] = v1;
}

// The left Jacobian of SE(3) at xi = (rho, phi), J_l = [[J, Q], [0, J]], for which
// Exp(xi + d) = Exp(J_l d + O(d^2)) Exp(xi): J is SO(3)'s left Jacobian (the V of exp_se3,
// J = I + c K + e3 K^2 with c = (1 - cos a) / a^2, e3 = (a - sin a) / a^3, K = [phi]x), and,
// matching the translations of both sides, Q = d(J rho)/d phi + [J rho]x J. With
// J rho = rho + c phi x rho + e3 phi x (phi x rho):
//   d(J rho)/d phi = -c [rho]x + e3 ((phi . rho) I + phi rho^T - 2 rho phi^T)
//                    + (phi x rho) c' phi^T + (phi x (phi x rho)) e3' phi^T,
// c' = (dc/da) / a and e3' = (de3/da) / a (Taylor series below a = 0.1, where they cancel).
// grad_xi = J_l^T grad at the perturbed pose.
__global__ void k_pose_perturb_bwd(const float* __restrict__ xi_in, int n_views, const float* __restrict__ g_in,
                                   float* __restrict__ g_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_views) return;
  double rho[3], w[3], g_r[3], g_w[3];
  for (int k = 0; k < 3; ++k) {
    rho[k] = (double)xi_in[6 * i + k];
    w[k] = (double)xi_in[6 * i + 3 + k];
    g_r[k] = (double)g_in[6 * i + k];
    g_w[k] = (double)g_in[6 * i + 3 + k];
  }
  const double a2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], a = sqrt(a2);
  double c, e3, cp, ep;
  if (a < 0.1) {
    c = 0.5 - a2 / 24.0 + a2 * a2 / 720.0 - a2 * a2 * a2 / 40320.0;
    e3 = 1.0 / 6.0 - a2 / 120.0 + a2 * a2 / 5040.0 - a2 * a2 * a2 / 362880.0;
    cp = -1.0 / 12.0 + a2 / 180.0 - a2 * a2 / 6720.0 + a2 * a2 * a2 / 453600.0;
    ep = -1.0 / 60.0 + a2 / 1260.0 - a2 * a2 / 60480.0 + a2 * a2 * a2 / 4989600.0;
  } else {
    const double sa = sin(a), ca = cos(a);
    c = (1.0 - ca) / a2;
    e3 = (a - sa) / (a2 * a);
    cp = sa / (a2 * a) - 2.0 * (1.0 - ca) / (a2 * a2);
    ep = (1.0 - ca) / (a2 * a2) - 3.0 * (a - sa) / (a2 * a2 * a);
  }
  const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
  double J[9];
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc) {
      const double k2 = K[3 * r] * K[cc] + K[3 * r + 1] * K[3 + cc] + K[3 * r + 2] * K[6 + cc];
      J[3 * r + cc] = (r == cc ? 1.0 : 0.0) + c * K[3 * r + cc] + e3 * k2;
    }
  const double wxr[3] = {w[1] * rho[2] - w[2] * rho[1], w[2] * rho[0] - w[0] * rho[2], w[0] * rho[1] - w[1] * rho[0]};
  const double wxwxr[3] = {w[1] * wxr[2] - w[2] * wxr[1], w[2] * wxr[0] - w[0] * wxr[2], w[0] * wxr[1] - w[1] * wxr[0]};
  const double wr = w[0] * rho[0] + w[1] * rho[1] + w[2] * rho[2];
  double Jr[3];
  for (int k = 0; k < 3; ++k) Jr[k] = rho[k] + c * wxr[k] + e3 * wxwxr[k];
  const double Rx[9] = {0.0, -rho[2], rho[1], rho[2], 0.0, -rho[0], -rho[1], rho[0], 0.0};
  const double JRx[9] = {0.0, -Jr[2], Jr[1], Jr[2], 0.0, -Jr[0], -Jr[1], Jr[0], 0.0};
  double Q[9];
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc) {
      double q = -c * Rx[3 * r + cc] + e3 * ((r == cc ? wr : 0.0) + w[r] * rho[cc] - 2.0 * rho[r] * w[cc]) +
                 cp * wxr[r] * w[cc] + ep * wxwxr[r] * w[cc];
      for (int k = 0; k < 3; ++k) q += JRx[3 * r + k] * J[3 * k + cc];
      Q[3 * r + cc] = q;
    }
  for (int cc = 0; cc < 3; ++cc) {
    double dr = 0.0, dw = 0.0;
    for (int r = 0; r < 3; ++r) {
      dr += J[3 * r + cc] * g_r[r];
      dw += Q[3 * r + cc] * g_r[r] + J[3 * r + cc] * g_w[r];
    }
    g_out[6 * i + cc] = (float)dr;
    g_out[6 * i + 3 + cc] = (float)dw;
  }
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

int launch_gaussians_adam(int64_t n, int n_sem, const gs_param_arrays& P, const gs_grads& G, const gs_param_arrays& M,
                          const gs_param_arrays& V, const gs_adam_config& hp, int step, hipStream_t s) {
  AdamGroups a{};
  float* ps[kGroups] = {P.mean, P.log_scale, P.quat, P.opacity, P.rgb, P.sem};
  const float* gs_[kGroups] = {G.mean, G.log_scale, G.quat, G.opacity, G.rgb, G.sem};
  float* ms[kGroups] = {M.mean, M.log_scale, M.quat, M.opacity, M.rgb, M.sem};
  float* vs[kGroups] = {V.mean, V.log_scale, V.quat, V.opacity, V.rgb, V.sem};
  const int64_t per[kGroups] = {3, 3, 4, 1, 3, n_sem};
  const float lrs[kGroups] = {hp.lr_mean, hp.lr_log_scale, hp.lr_quat, hp.lr_opacity, hp.lr_rgb, hp.lr_sem};
  int64_t run = 0;
  for (int k = 0; k < kGroups; ++k) {
    const bool use = lrs[k] != 0.0f && per[k] > 0 && n > 0;
    a.p[k] = ps[k];
    a.g[k] = gs_[k];
    a.m[k] = ms[k];
    a.v[k] = vs[k];
    a.n[k] = use ? per[k] * n : 0;
    a.lr[k] = lrs[k];
    a.vec[k] = aligned16(ps[k]) && aligned16(gs_[k]) && aligned16(ms[k]) && aligned16(vs[k]);
    run += ceil_div(a.n[k], 4);
    a.quad_end[k] = run;
  }
  if (run == 0) return GS_OK;
  const double c1 = 1.0 / (1.0 - pow((double)hp.beta1, step));
  const double c2 = 1.0 / (1.0 - pow((double)hp.beta2, step));
  const int64_t blocks = std::min<int64_t>(ceil_div(run, 256), 8192);
  hipLaunchKernelGGL(k_adam_groups, dim3((unsigned)blocks), dim3(256), 0, s, a, hp.beta1, hp.beta2, hp.eps, (float)c1,
                     (float)c2);
  return launch_status();
}

int launch_pose_adam(gs_view* views, int n_views, const float* grad, float* m, float* v, const gs_adam_config& hp,
                     int step, hipStream_t s) {
  if (n_views == 0) return GS_OK;
  const double c1 = 1.0 / (1.0 - pow((double)hp.beta1, step));
  const double c2 = 1.0 / (1.0 - pow((double)hp.beta2, step));
  hipLaunchKernelGGL(k_pose_adam, dim3((unsigned)ceil_div(n_views, 64)), dim3(64), 0, s, views, n_views, grad, m, v,
                     hp.lr_rho, hp.lr_phi, hp.beta1, hp.beta2, hp.eps, (float)c1, (float)c2);
  return launch_status();
}

int launch_pose_perturb(const gs_view* vin, int n_views, const float* xi, gs_view* vout, hipStream_t s) {
  if (n_views == 0) return GS_OK;
  hipLaunchKernelGGL(k_pose_perturb, dim3((unsigned)ceil_div(n_views, 64)), dim3(64), 0, s, vin, n_views, xi, vout);
  return launch_status();
}

int launch_pose_perturb_bwd(const float* xi, int n_views, const float* g_in, float* g_out, hipStream_t s) {
  if (n_views == 0) return GS_OK;
  hipLaunchKernelGGL(k_pose_perturb_bwd, dim3((unsigned)ceil_div(n_views, 64)), dim3(64), 0, s, xi, n_views, g_in, g_out);
  return launch_status();
}

}  // namespace gs
