// Projection of 3D Gaussians to 2D footprints (paper Sec. III-B, eq. 2-3, in the EWA
// form, or literally with cfg.isotropic: one scale, no rotation, r2D = f r / d per image
// axis) and its backward pass, including the pose tangent.
//
// One thread per Gaussian walks every view and, per view, every pyramid level. The
// arithmetic is double precision (these kernels are bound by HBM traffic, and the
// FP64 vector rate of gfx950 equals its unpacked FP32 rate); results are stored in
// single precision. The projected mean is stored as a hi + lo float pair so that the
// per-pixel offsets in the compositing kernels keep full single precision.
#include "common.h"

namespace gs {
namespace {

struct Geo {            // view-independent part of one Gaussian
  double mu[3];
  double qn[4], qlen;
  double Rq[9], s[3];
  double Sig[6];        // world covariance, upper triangle xx xy xz yy yz zz
  double o;
  bool ok;
};

__device__ inline void quat_rot(const double* q, double* R) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ inline Geo load_geo(const gs_gaussians& g, int64_t i, bool iso) {
  Geo G;
  const float* m = g.mean + 3 * i;
  G.mu[0] = m[0]; G.mu[1] = m[1]; G.mu[2] = m[2];
  if (iso) {   // eq. 1: one scale; the rotation and covariance are not used
    G.s[0] = exp((double)g.log_scale[3 * i]);
    G.s[1] = G.s[2] = G.s[0];
    for (int k = 0; k < 4; ++k) G.qn[k] = 0.0;
    G.qlen = 1.0;
    for (int k = 0; k < 9; ++k) G.Rq[k] = (k % 4 == 0) ? 1.0 : 0.0;
    for (int k = 0; k < 6; ++k) G.Sig[k] = 0.0;
    G.o = 1.0 / (1.0 + exp(-(double)g.opacity[i]));
    G.ok = true;
    return G;
  }
  const float4 q = *reinterpret_cast<const float4*>(g.quat + 4 * i);
  double qv[4] = {q.x, q.y, q.z, q.w};
  G.qlen = sqrt(qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3]);
  G.ok = G.qlen > 0.0 && isfinite(G.qlen);
  const double inv = G.ok ? 1.0 / G.qlen : 0.0;
  for (int k = 0; k < 4; ++k) G.qn[k] = qv[k] * inv;
  quat_rot(G.qn, G.Rq);
  const float* ls = g.log_scale + 3 * i;
  for (int k = 0; k < 3; ++k) G.s[k] = exp((double)ls[k]);
  // Sigma = Rq diag(s^2) Rq^T
  double s2[3] = {G.s[0] * G.s[0], G.s[1] * G.s[1], G.s[2] * G.s[2]};
  const double* R = G.Rq;
  auto sig = [&](int a, int b) { return R[3 * a] * R[3 * b] * s2[0] + R[3 * a + 1] * R[3 * b + 1] * s2[1] + R[3 * a + 2] * R[3 * b + 2] * s2[2]; };
  G.Sig[0] = sig(0, 0); G.Sig[1] = sig(0, 1); G.Sig[2] = sig(0, 2);
  G.Sig[3] = sig(1, 1); G.Sig[4] = sig(1, 2); G.Sig[5] = sig(2, 2);
  G.o = 1.0 / (1.0 + exp(-(double)g.opacity[i]));
  return G;
}

__device__ inline double sym(const double* S, int a, int b) {  // upper-triangle accessor
  if (a > b) { int t = a; a = b; b = t; }
  const int idx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  return S[idx[a][b]];
}

struct Cam {           // one view applied to one Gaussian
  double mc[3];        // camera-space mean
  double Sc[6];        // camera covariance, upper triangle
};

__device__ inline Cam to_camera(const gs_view& V, const Geo& G) {
  Cam c;
  for (int r = 0; r < 3; ++r)
    c.mc[r] = ((double)V.R[3 * r] * G.mu[0] + (double)V.R[3 * r + 1] * G.mu[1]) + (double)V.R[3 * r + 2] * G.mu[2] + (double)V.t[r];
  double RS[9];  // R * Sigma
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)
      RS[3 * r + k] = V.R[3 * r] * sym(G.Sig, 0, k) + V.R[3 * r + 1] * sym(G.Sig, 1, k) + V.R[3 * r + 2] * sym(G.Sig, 2, k);
  int n = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b)
      c.Sc[n++] = RS[3 * a] * V.R[3 * b] + RS[3 * a + 1] * V.R[3 * b + 1] + RS[3 * a + 2] * V.R[3 * b + 2];
  return c;
}

struct Lvl {           // one level's 2D footprint
  double J[4];         // nonzero Jacobian entries: J00 = fx/z, J02, J11 = fy/z, J12
  double ux, uy;       // clamped x/z, y/z
  bool clx, cly;
  double cov[3];       // dilated 2D covariance a, b, c
  double conic[3];
  double m2[2];
  int radius;
  int rect[4];
  bool vis;
};

__device__ inline Lvl footprint(const gs_config& cfg, const gs_item& it, const Cam& c, double s0) {
  Lvl L;
  L.vis = false;
  const double z = c.mc[2], x = c.mc[0], y = c.mc[1];
  const double fx = it.fx, fy = it.fy;
  if (cfg.isotropic) {
    // eq. 2-3: standard deviation f r / d along each image axis
    const double rx = fx * s0 / z, ry = fy * s0 / z;
    L.clx = L.cly = false;
    L.ux = x / z;
    L.uy = y / z;
    L.J[0] = L.J[1] = L.J[2] = L.J[3] = 0.0;
    L.cov[0] = rx * rx + cfg.eps_dilate;
    L.cov[1] = 0.0;
    L.cov[2] = ry * ry + cfg.eps_dilate;
  } else {
  const double limx = (double)cfg.guard * (0.5 * it.W) / fx;
  const double limy = (double)cfg.guard * (0.5 * it.H) / fy;
  const double tx = x / z, ty = y / z;
  L.clx = fabs(tx) > limx;
  L.cly = fabs(ty) > limy;
  L.ux = fmin(limx, fmax(-limx, tx));
  L.uy = fmin(limy, fmax(-limy, ty));
  L.J[0] = fx / z;
  L.J[1] = -fx * L.ux / z;
  L.J[2] = fy / z;
  L.J[3] = -fy * L.uy / z;
  // rows of J: r0 = (J0, 0, J1), r1 = (0, J2, J3)
  const double* S = c.Sc;  // xx xy xz yy yz zz
  const double r0S0 = L.J[0] * S[0] + L.J[1] * S[2];
  const double r0S1 = L.J[0] * S[1] + L.J[1] * S[4];
  const double r0S2 = L.J[0] * S[2] + L.J[1] * S[5];
  const double r1S1 = L.J[2] * S[3] + L.J[3] * S[4];
  const double r1S2 = L.J[2] * S[4] + L.J[3] * S[5];
  L.cov[0] = r0S0 * L.J[0] + r0S2 * L.J[1] + cfg.eps_dilate;
  L.cov[1] = r0S1 * L.J[2] + r0S2 * L.J[3];
  L.cov[2] = r1S1 * L.J[2] + r1S2 * L.J[3] + cfg.eps_dilate;
  }
  const double det = L.cov[0] * L.cov[2] - L.cov[1] * L.cov[1];
  if (!(det > 0.0)) return L;
  const double id = 1.0 / det;
  L.conic[0] = L.cov[2] * id;
  L.conic[1] = -L.cov[1] * id;
  L.conic[2] = L.cov[0] * id;
  L.m2[0] = fx * (x / z) + (double)it.cx;
  L.m2[1] = fy * (y / z) + (double)it.cy;
  const double mid = 0.5 * (L.cov[0] + L.cov[2]);
  const double lam = mid + sqrt(fmax(0.1, mid * mid - det));
  L.radius = (int)ceil(3.0 * sqrt(lam));
  if (L.radius <= 0) return L;
  if (cfg.full_rect) {
    L.rect[0] = 0; L.rect[1] = 0; L.rect[2] = it.tiles_x; L.rect[3] = it.tiles_y;
  } else {
    const double r = L.radius;
    // tile sides are powers of two, so the products by their reciprocals are the quotients exactly
    const double iw = 1.0 / 256.0 * (double)(256 / cfg.tile_w), ih = 1.0 / 256.0 * (double)(256 / cfg.tile_h);
    L.rect[0] = min(it.tiles_x, max(0, (int)floor((L.m2[0] - r) * iw)));
    L.rect[1] = min(it.tiles_y, max(0, (int)floor((L.m2[1] - r) * ih)));
    L.rect[2] = min(it.tiles_x, max(0, (int)floor((L.m2[0] + r) * iw) + 1));
    L.rect[3] = min(it.tiles_y, max(0, (int)floor((L.m2[1] + r) * ih) + 1));
  }
  L.vis = L.rect[2] > L.rect[0] && L.rect[3] > L.rect[1];
  return L;
}

__global__ __launch_bounds__(256) void k_preprocess(gs_config cfg, gs_gaussians g, const gs_view* __restrict__ views,
                                                    int n_views, const gs_item* __restrict__ items,
                                                    gs_projected out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int64_t n = g.n;
  const Geo G = load_geo(g, i, cfg.isotropic != 0);
  for (int v = 0; v < n_views; ++v) {
    const gs_view V = views[v];
    const Cam c = to_camera(V, G);
    const bool front = G.ok && c.mc[2] > (double)cfg.z_near;
    for (int k = V.item_first; k < V.item_first + V.item_count; ++k) {
      const int64_t e = (int64_t)k * n + i;
      if (!front) { out.radius[e] = 0; continue; }
      const Lvl L = footprint(cfg, items[k], c, G.s[0]);
      if (!L.vis) { out.radius[e] = 0; continue; }
      float4 a, b;
      a.x = (float)L.m2[0];
      a.y = (float)L.m2[1];
      a.z = (float)(L.m2[0] - (double)a.x);
      a.w = (float)(L.m2[1] - (double)a.y);
      b.x = (float)L.conic[0];
      b.y = (float)L.conic[1];
      b.z = (float)L.conic[2];
      b.w = (float)G.o;
      float4* r = reinterpret_cast<float4*>(out.rec + kRecFloats * e);
      r[0] = a;
      r[1] = b;
      out.depth[e] = (float)c.mc[2];
      out.radius[e] = L.radius;
    }
  }
}

// Backward. g2d holds, per (item, Gaussian), the gradient of the loss with respect to
// mean2d (x, y), conic (A, B, C), opacity and the composited depth channel, [E][8].
__global__ __launch_bounds__(256) void k_preprocess_bwd(gs_config cfg, gs_gaussians g,
                                                        const gs_view* __restrict__ views, int n_views,
                                                        const gs_item* __restrict__ items,
                                                        const float* __restrict__ g2d, const int32_t* __restrict__ radius,
                                                        gs_grads out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < g.n;
  const int64_t n = g.n;
  const int64_t ii = live ? i : 0;
  const bool iso = cfg.isotropic != 0;
  const Geo G = load_geo(g, ii, iso);
  double gmu[3] = {0, 0, 0}, gsig[6] = {0, 0, 0, 0, 0, 0}, gop = 0, gls0 = 0;
  __shared__ double red[4][6];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int v = 0; v < n_views; ++v) {
    const gs_view V = views[v];
    double gpose[6] = {0, 0, 0, 0, 0, 0};
    bool any = false;
    if (live) {
      for (int k = V.item_first; k < V.item_first + V.item_count; ++k)
        any |= radius[(int64_t)k * n + i] > 0;
    }
    if (any) {
      const Cam c = to_camera(V, G);
      double gmc[3] = {0, 0, 0}, gSc[6] = {0, 0, 0, 0, 0, 0};
      for (int k = V.item_first; k < V.item_first + V.item_count; ++k) {
        const int64_t e = (int64_t)k * n + i;
        if (radius[e] <= 0) continue;
        const gs_item it = items[k];
        const Lvl L = footprint(cfg, it, c, G.s[0]);
        const float4 ga = *reinterpret_cast<const float4*>(g2d + 8 * e);
        const float4 gb = *reinterpret_cast<const float4*>(g2d + 8 * e + 4);
        const double dmx = ga.x, dmy = ga.y, dA = ga.z, dB = ga.w, dC = gb.x, dO = gb.y, dZ = gb.z;
        gop += dO * G.o * (1.0 - G.o);
        // conic = cov^-1: dcov = -Q Gq Q with Gq = [[dA, dB/2], [dB/2, dC]]
        const double Q00 = L.conic[0], Q01 = L.conic[1], Q11 = L.conic[2];
        const double G00 = dA, G01 = 0.5 * dB, G11 = dC;
        const double T00 = Q00 * G00 + Q01 * G01, T01 = Q00 * G01 + Q01 * G11;
        const double T10 = Q01 * G00 + Q11 * G01, T11 = Q01 * G01 + Q11 * G11;
        const double C00 = -(T00 * Q00 + T01 * Q01);
        const double C01 = -(T00 * Q01 + T01 * Q11);
        const double C11 = -(T10 * Q01 + T11 * Q11);
        if (iso) {
          // cov = diag((fx r/z)^2, (fy r/z)^2) + eps: each diagonal entry v has dv/dz = -2v/z and
          // dv/d(log r) = 2v
          const double z = c.mc[2], x = c.mc[0], y = c.mc[1];
          const double rx = it.fx * G.s[0] / z, ry = it.fy * G.s[0] / z;
          const double dv = C00 * rx * rx + C11 * ry * ry;
          gls0 += 2.0 * dv;
          gmc[2] += -2.0 * dv / z;
          gmc[0] += dmx * it.fx / z;
          gmc[1] += dmy * it.fy / z;
          gmc[2] += -(dmx * it.fx * x + dmy * it.fy * y) / (z * z);
          gmc[2] += dZ;
          continue;
        }
        // cov = J Sc J^T: dSc = J^T C J (symmetric), dJ = 2 C J Sc
        const double j00 = L.J[0], j02 = L.J[1], j11 = L.J[2], j12 = L.J[3];
        // J^T C J, J rows r0 = (j00, 0, j02), r1 = (0, j11, j12)
        const double cr0[3] = {C00 * j00, C01 * j11, C00 * j02 + C01 * j12};  // row0 of C*J
        const double cr1[3] = {C01 * j00, C11 * j11, C01 * j02 + C11 * j12};  // row1 of C*J
        // dSc[a][b] = sum_r J[r][a] (C J)[r][b]
        const double Jc0[3] = {j00, 0.0, j02};
        const double Jc1[3] = {0.0, j11, j12};
        int m = 0;
        for (int a = 0; a < 3; ++a)
          for (int b = a; b < 3; ++b) {
            // symmetric matrix stored once; off-diagonal entries hold the (a,b) value
            gSc[m++] += Jc0[a] * cr0[b] + Jc1[a] * cr1[b];
          }
        // dJ[r][b] = 2 sum_m (C J)[r][m] Sc[m][b]
        double dJ0[3], dJ1[3];
        for (int b = 0; b < 3; ++b) {
          dJ0[b] = 2.0 * (cr0[0] * sym(c.Sc, 0, b) + cr0[1] * sym(c.Sc, 1, b) + cr0[2] * sym(c.Sc, 2, b));
          dJ1[b] = 2.0 * (cr1[0] * sym(c.Sc, 0, b) + cr1[1] * sym(c.Sc, 1, b) + cr1[2] * sym(c.Sc, 2, b));
        }
        const double z = c.mc[2], x = c.mc[0], y = c.mc[1];
        const double fx = it.fx, fy = it.fy;
        const double iz2 = 1.0 / (z * z);
        gmc[2] += dJ0[0] * (-fx * iz2) + dJ1[1] * (-fy * iz2);
        if (L.clx) {
          gmc[2] += dJ0[2] * (fx * L.ux * iz2);
        } else {
          gmc[0] += dJ0[2] * (-fx * iz2);
          gmc[2] += dJ0[2] * (2.0 * fx * x * iz2 / z);
        }
        if (L.cly) {
          gmc[2] += dJ1[2] * (fy * L.uy * iz2);
        } else {
          gmc[1] += dJ1[2] * (-fy * iz2);
          gmc[2] += dJ1[2] * (2.0 * fy * y * iz2 / z);
        }
        gmc[0] += dmx * fx / z;
        gmc[1] += dmy * fy / z;
        gmc[2] += -(dmx * fx * x + dmy * fy * y) * iz2;
        gmc[2] += dZ;
      }
      // mc = R mu + t
      for (int a = 0; a < 3; ++a) gmu[a] += V.R[a] * gmc[0] + V.R[3 + a] * gmc[1] + V.R[6 + a] * gmc[2];
      // Sc = R Sigma R^T -> dSigma = R^T dSc R; full symmetric dSc
      double D[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) D[3 * a + b] = (a == b) ? sym(gSc, a, b) : sym(gSc, a, b);
      // off-diagonal entries of gSc hold d/d(Sc_ab) for the matrix entry (both halves equal)
      double RtD[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) RtD[3 * a + b] = V.R[a] * D[b] + V.R[3 + a] * D[3 + b] + V.R[6 + a] * D[6 + b];
      int m = 0;
      for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b)
          gsig[m++] += RtD[3 * a] * V.R[b] + RtD[3 * a + 1] * V.R[3 + b] + RtD[3 * a + 2] * V.R[6 + b];
      // pose: d mc = rho + phi x mc; d Sc = phi^ Sc - Sc phi^  -> 2 * axial(Sc D - D Sc)
      gpose[0] = gmc[0]; gpose[1] = gmc[1]; gpose[2] = gmc[2];
      gpose[3] = c.mc[1] * gmc[2] - c.mc[2] * gmc[1];
      gpose[4] = c.mc[2] * gmc[0] - c.mc[0] * gmc[2];
      gpose[5] = c.mc[0] * gmc[1] - c.mc[1] * gmc[0];
      double X[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s1 = 0, s2 = 0;
          for (int k = 0; k < 3; ++k) {
            s1 += sym(c.Sc, a, k) * D[3 * k + b];
            s2 += D[3 * a + k] * sym(c.Sc, k, b);
          }
          X[3 * a + b] = s1 - s2;
        }
      gpose[3] += 2.0 * X[5];
      gpose[4] += 2.0 * X[6];
      gpose[5] += 2.0 * X[1];
    }
    // block reduction of the pose gradient of view v
    const bool block_any = __syncthreads_or(any);
    if (block_any) {
      for (int k = 0; k < 6; ++k) {
        const double s = wave_sum_d(gpose[k]);
        if (lane == 0) red[wid][k] = s;
      }
      __syncthreads();
      if (threadIdx.x < 6) {
        const double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        if (s != 0.0) atomicAdd(out.pose + 6 * v + threadIdx.x, (float)s);
      }
      __syncthreads();
    }
  }
  if (!live) return;
  if (iso) {   // no covariance: only the first log-scale has a gradient
    for (int a = 0; a < 3; ++a) out.mean[3 * i + a] = (float)gmu[a];
    out.log_scale[3 * i] = (float)gls0;
    out.log_scale[3 * i + 1] = 0.0f;
    out.log_scale[3 * i + 2] = 0.0f;
    for (int a = 0; a < 4; ++a) out.quat[4 * i + a] = 0.0f;
    out.opacity[i] = (float)gop;
    return;
  }
  // Sigma = M M^T, M = Rq diag(s): dM = 2 dSigma M, with dSigma the full symmetric gradient
  double D[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) D[3 * a + b] = sym(gsig, a, b);
  double M[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) M[3 * r + k] = G.Rq[3 * r + k] * G.s[k];
  double dM[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) dM[3 * r + k] = 2.0 * (D[3 * r] * M[k] + D[3 * r + 1] * M[3 + k] + D[3 * r + 2] * M[6 + k]);
  double dls[3];
  for (int k = 0; k < 3; ++k) dls[k] = (dM[k] * G.Rq[k] + dM[3 + k] * G.Rq[3 + k] + dM[6 + k] * G.Rq[6 + k]) * G.s[k];
  double d[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) d[3 * r + k] = dM[3 * r + k] * G.s[k];
  const double w = G.qn[0], qx = G.qn[1], qy = G.qn[2], qz = G.qn[3];
  double dq[4];
  dq[0] = 2.0 * (qz * (d[3] - d[1]) + qy * (d[2] - d[6]) + qx * (d[7] - d[5]));
  dq[1] = 2.0 * (qy * (d[1] + d[3]) + qz * (d[2] + d[6]) + w * (d[7] - d[5]) - 2.0 * qx * (d[4] + d[8]));
  dq[2] = 2.0 * (qx * (d[1] + d[3]) + w * (d[2] - d[6]) + qz * (d[5] + d[7]) - 2.0 * qy * (d[0] + d[8]));
  dq[3] = 2.0 * (w * (d[3] - d[1]) + qx * (d[2] + d[6]) + qy * (d[5] + d[7]) - 2.0 * qz * (d[0] + d[4]));
  const double dot = w * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
  const double iq = G.ok ? 1.0 / G.qlen : 0.0;
  for (int a = 0; a < 3; ++a) out.mean[3 * i + a] = (float)gmu[a];
  for (int a = 0; a < 3; ++a) out.log_scale[3 * i + a] = (float)dls[a];
  for (int a = 0; a < 4; ++a) out.quat[4 * i + a] = (float)((dq[a] - G.qn[a] * dot) * iq);
  out.opacity[i] = (float)gop;
}

}  // namespace

int launch_preprocess(const gs_config& cfg, const gs_gaussians& g, const gs_view* views, int n_views,
                      const gs_item* items, const gs_projected& out, hipStream_t s) {
  const int64_t blocks = ceil_div(g.n, 256);
  if (blocks == 0) return GS_OK;
  hipLaunchKernelGGL(k_preprocess, dim3((unsigned)blocks), dim3(256), 0, s, cfg, g, views, n_views, items, out);
  return launch_status();
}

int launch_preprocess_bwd(const gs_config& cfg, const gs_gaussians& g, const gs_view* views, int n_views,
                          const gs_item* items, const float* g2d, const int32_t* radius, const gs_grads& out,
                          hipStream_t s) {
  const int64_t blocks = ceil_div(g.n, 256);
  if (blocks == 0) return GS_OK;
  hipLaunchKernelGGL(k_preprocess_bwd, dim3((unsigned)blocks), dim3(256), 0, s, cfg, g, views, n_views, items, g2d,
                     radius, out);
  return launch_status();
}

}  // namespace gs
