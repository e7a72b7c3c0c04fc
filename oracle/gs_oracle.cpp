// Test infrastructure only: a plain, slow, single-threaded FP64 reference of the
// pyramid Gaussian-splatting rasterizer (projection, tile binning and depth sort,
// front-to-back compositing of RGB / depth / semantics, pyramid loss and the exact
// reverse-mode gradient). Only the test-suite, the smoke check and the benchmark's
// CPU-baseline leg load it; the HIP library never does, and the two share no code.
//
// What it computes (paper Sec. III-B .. III-D):
//   * projection of a 3D Gaussian to a 2D footprint (eq. 2-3), generalised to the
//     anisotropic EWA form: Sigma = R(q) S S^T R(q)^T, Sigma' = J W Sigma W^T J^T;
//     eq. 2's r2D = f r / d is the on-axis isotropic special case;
//   * the image pyramid (eq. 4-6): level l uses K_l = diag(2^-l, 2^-l, 1) K_0 and a
//     W/2^l x H/2^l image; targets are 2x2 box means of the level above;
//   * compositing of RGB (eq. 7), depth (eq. 8) and semantics (eq. 9) over the
//     depth-sorted set N of primitives touching the pixel's tile;
//   * the per-level losses (eq. 10-13): mean L1 on RGB, mean L1 on valid depth and
//     a per-pixel cross-entropy on the composited class logits, summed over levels;
//   * back-propagation of that loss to every Gaussian parameter (Sec. III-D) and to a
//     left-multiplied SE(3) tangent of every camera pose.
// Readings where the paper is silent (cut-offs, pixel centres, sort key, ...) are
// the ones listed with the design notes: pixel (u,v) is sampled at (u+1/2, v+1/2);
// z_near cull; x/z, y/z clamped to +-guard*(W/2f) inside the Jacobian; eps added to
// the 2D covariance diagonal; radius ceil(3 sqrt(lambda_max)); a Gaussian belongs to
// the tiles meeting [mu-r, mu+r]^2; order = (float32 depth, index); alpha =
// min(alpha_max, o exp(power)), skipped below alpha_min; a pixel stops before the
// Gaussian that would take T below t_min; background 0.
//
// Near-threshold decisions (alpha_min / alpha_max / t_min, z_near, the guard band,
// rect and radius rounding) are flagged per pixel, and per Gaussian, so that a
// single-precision implementation can be compared away from them.
//
// Items (view, level) are independent given the Gaussians, so the render and its backward
// take one item at a time (project every Gaussian, bin and sort the item's tiles, composite,
// chain the item's 2D gradients back to the parameters) and hold one item's projections at
// once; with a tile mask, items without a masked tile are skipped.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

struct Cfg {
  int tw, th, full_rect, S;
  int isotropic;      // 1: the primitive of eq. 1-3 (one scale, no rotation, r2D = f r / d)
  double z_near, eps, a_min, a_max, t_min, guard;
  double margin;      // relative closeness that flags a per-pixel decision
  double margin_pre;  // the same for the projection's decisions
};

Cfg read_cfg(const double* cd, const int* ci) {
  Cfg c;
  c.z_near = cd[0];
  c.eps = cd[1];
  c.a_min = cd[2];
  c.a_max = cd[3];
  c.t_min = cd[4];
  c.guard = cd[5];
  c.margin = cd[6];
  c.margin_pre = cd[7];
  c.tw = ci[0];
  c.th = ci[1];
  c.full_rect = ci[2];
  c.S = ci[3];
  c.isotropic = ci[4];
  return c;
}

struct Item {
  int view, level, W, H, ntx, nty, tile0;
  int64_t pix0;
  double fx, fy, cx, cy;
};

// A view: pose R (row-major), t; base intrinsics; base size; pyramid depth.
std::vector<Item> make_items(const Cfg& c, int n_views, const double* vd, const int* vi) {
  std::vector<Item> items;
  int64_t pix = 0;
  int tile = 0;
  for (int v = 0; v < n_views; ++v) {
    const double* d = vd + 16 * v;
    int W0 = vi[3 * v + 0], H0 = vi[3 * v + 1], L = vi[3 * v + 2];
    for (int l = 0; l < L; ++l) {
      Item it;
      it.view = v;
      it.level = l;
      double s = std::ldexp(1.0, -l);
      it.fx = d[12] * s;
      it.fy = d[13] * s;
      it.cx = d[14] * s;
      it.cy = d[15] * s;
      it.W = W0 >> l;
      it.H = H0 >> l;
      it.ntx = (it.W + c.tw - 1) / c.tw;
      it.nty = (it.H + c.th - 1) / c.th;
      it.tile0 = tile;
      it.pix0 = pix;
      tile += it.ntx * it.nty;
      pix += int64_t(it.W) * it.H;
      items.push_back(it);
    }
  }
  return items;
}

struct Gauss {
  int64_t n;
  const double *mean, *lsc, *quat, *opac, *rgb, *sem;
};

// Everything the forward derives for one (item, Gaussian), kept for the backward.
struct Proj {
  bool vis = false;
  int flag = 0;
  double mc[3];           // camera-space mean
  double qn[4], qlen;     // normalised quaternion and the input's norm
  double Rq[9], s[3];     // rotation of the Gaussian, per-axis std
  double M[9];            // Rq * diag(s)
  double Sc[9];           // camera-space 3D covariance
  double ux, uy;          // x/z, y/z after the guard clamp
  bool clx, cly;          // guard clamp active
  double J[6];            // 2x3 Jacobian of the projection
  double cov[3];          // dilated 2D covariance (a, b, c)
  double conic[3];        // its inverse (A, B, C)
  double m2[2];           // projected mean, pixel units
  double o;               // opacity
  double z;               // camera depth of the mean
  float z32;              // the same depth rounded to single precision (sort key)
  int radius;
  int rect[4];            // x0, y0, x1, y1 in tiles, half open
};

bool near_rel(double v, double thr, double m) { return std::fabs(v - thr) <= m * std::fabs(thr); }
bool near_int(double v, double m) { return std::fabs(v - std::nearbyint(v)) <= m * std::max(1.0, std::fabs(v)); }

void quat_to_rot(const double* q, double* R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

// 3x3 helpers, row-major.
void mm(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}
void mmT(const double* A, const double* B, double* C) {  // A * B^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * j + k];
      C[3 * i + j] = s;
    }
}
void mTm(const double* A, const double* B, double* C) {  // A^T * B
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * k + i] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

Proj project(const Cfg& c, const Gauss& g, int64_t i, const double* Rv, const double* tv, const Item& it) {
  Proj p;
  const double* mu = g.mean + 3 * i;
  for (int r = 0; r < 3; ++r) p.mc[r] = Rv[3 * r] * mu[0] + Rv[3 * r + 1] * mu[1] + Rv[3 * r + 2] * mu[2] + tv[r];
  p.z = p.mc[2];
  if (near_rel(p.z, c.z_near, c.margin_pre)) p.flag |= 1;
  if (!(p.z > c.z_near)) return p;
  if (c.isotropic) {
    // eq. 1-3: g3D = o exp(-|x - mu|^2 / (2 r^2)) with r = exp(first log-scale) projects to a
    // 2D Gaussian of standard deviation r2D = f r / d about mu2D, f taken per image axis
    p.s[0] = std::exp(g.lsc[3 * i]);
    const double rx = it.fx * p.s[0] / p.z, ry = it.fy * p.s[0] / p.z;
    p.cov[0] = rx * rx + c.eps;
    p.cov[1] = 0.0;
    p.cov[2] = ry * ry + c.eps;
  } else {
  const double* q = g.quat + 4 * i;
  p.qlen = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(p.qlen > 0) || !std::isfinite(p.qlen)) return p;
  for (int k = 0; k < 4; ++k) p.qn[k] = q[k] / p.qlen;
  quat_to_rot(p.qn, p.Rq);
  for (int k = 0; k < 3; ++k) p.s[k] = std::exp(g.lsc[3 * i + k]);
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) p.M[3 * r + k] = p.Rq[3 * r + k] * p.s[k];
  double Sig[9], RS[9];
  mmT(p.M, p.M, Sig);          // Sigma = M M^T
  mm(Rv, Sig, RS);
  mmT(RS, Rv, p.Sc);           // Sigma_c = W Sigma W^T
  double limx = c.guard * (0.5 * it.W) / it.fx;
  double limy = c.guard * (0.5 * it.H) / it.fy;
  double ux = p.mc[0] / p.z, uy = p.mc[1] / p.z;
  if (near_rel(std::fabs(ux), limx, c.margin_pre) || near_rel(std::fabs(uy), limy, c.margin_pre)) p.flag |= 2;
  p.clx = std::fabs(ux) > limx;
  p.cly = std::fabs(uy) > limy;
  p.ux = std::min(limx, std::max(-limx, ux));
  p.uy = std::min(limy, std::max(-limy, uy));
  p.J[0] = it.fx / p.z; p.J[1] = 0;              p.J[2] = -it.fx * p.ux / p.z;
  p.J[3] = 0;           p.J[4] = it.fy / p.z;    p.J[5] = -it.fy * p.uy / p.z;
  // Sigma' = J Sigma_c J^T
  double JS[6];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += p.J[3 * r + m] * p.Sc[3 * m + k];
      JS[3 * r + k] = s;
    }
  double C2[4];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 2; ++k) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += JS[3 * r + m] * p.J[3 * k + m];
      C2[2 * r + k] = s;
    }
  p.cov[0] = C2[0] + c.eps;
  p.cov[1] = C2[1];
  p.cov[2] = C2[3] + c.eps;
  }
  double det = p.cov[0] * p.cov[2] - p.cov[1] * p.cov[1];
  if (!(det > 0)) return p;
  p.conic[0] = p.cov[2] / det;
  p.conic[1] = -p.cov[1] / det;
  p.conic[2] = p.cov[0] / det;
  p.m2[0] = it.fx * (p.mc[0] / p.z) + it.cx;
  p.m2[1] = it.fy * (p.mc[1] / p.z) + it.cy;
  double mid = 0.5 * (p.cov[0] + p.cov[2]);
  double lam = mid + std::sqrt(std::max(0.1, mid * mid - det));
  double rr = 3.0 * std::sqrt(lam);
  if (near_int(rr, c.margin_pre)) p.flag |= 4;
  p.radius = int(std::ceil(rr));
  if (p.radius <= 0) return p;
  if (c.full_rect) {
    p.rect[0] = 0; p.rect[1] = 0; p.rect[2] = it.ntx; p.rect[3] = it.nty;
  } else {
    double ex[4] = {(p.m2[0] - p.radius) / c.tw, (p.m2[1] - p.radius) / c.th,
                    (p.m2[0] + p.radius) / c.tw, (p.m2[1] + p.radius) / c.th};
    for (int k = 0; k < 4; ++k)
      if (near_int(ex[k], c.margin_pre)) p.flag |= 8;
    int lim[2] = {it.ntx, it.nty};
    for (int k = 0; k < 2; ++k) {
      p.rect[k] = std::min(lim[k], std::max(0, int(std::floor(ex[k]))));
      p.rect[k + 2] = std::min(lim[k], std::max(0, int(std::floor(ex[k + 2])) + 1));
    }
  }
  if (p.rect[2] <= p.rect[0] || p.rect[3] <= p.rect[1]) return p;
  double a = g.opac[i];
  p.o = 1.0 / (1.0 + std::exp(-a));
  p.z32 = float(p.z);
  p.vis = true;
  return p;
}

struct Scene {
  Cfg c;
  Gauss g;
  int n_views;
  const double* vd;
  std::vector<Item> items;
  // The item being processed: the projections of every Gaussian for it and its tiles'
  // sorted lists. One item is held at a time, so the memory is that of one item.
  int cur = -1;
  std::vector<Proj> proj;                       // [gaussian]
  std::vector<std::vector<uint32_t>> lists;     // [tile of item cur] -> sorted Gaussian ids
  int K() const { return 4 + c.S; }
};

// Projects every Gaussian for item k and, unless brute, bins and depth-sorts its tiles.
void build_item(Scene& s, int k, bool brute) {
  const Item& it = s.items[k];
  const double* Rv = s.vd + 16 * it.view;
  s.cur = k;
  s.proj.assign(size_t(s.g.n), Proj());
  s.lists.assign(size_t(it.ntx) * it.nty, {});
  for (int64_t i = 0; i < s.g.n; ++i) {
    Proj p = project(s.c, s.g, i, Rv, Rv + 9, it);
    s.proj[i] = p;
    if (!p.vis || brute) continue;
    for (int ty = p.rect[1]; ty < p.rect[3]; ++ty)
      for (int tx = p.rect[0]; tx < p.rect[2]; ++tx) s.lists[ty * it.ntx + tx].push_back(uint32_t(i));
  }
  if (brute) return;
  const auto& P = s.proj;
  for (auto& L : s.lists)
    std::sort(L.begin(), L.end(), [&](uint32_t a, uint32_t b) {
      if (P[a].z32 != P[b].z32) return P[a].z32 < P[b].z32;
      return a < b;
    });
}

// The list a pixel of the current item iterates in brute-force mode: every Gaussian whose
// rect holds the pixel's tile, in (float depth, index) order, found without tile lists.
std::vector<uint32_t> brute_list(const Scene& s, int tx, int ty) {
  std::vector<uint32_t> L;
  const auto& P = s.proj;
  for (int64_t i = 0; i < s.g.n; ++i) {
    const Proj& p = P[i];
    if (p.vis && tx >= p.rect[0] && tx < p.rect[2] && ty >= p.rect[1] && ty < p.rect[3]) L.push_back(uint32_t(i));
  }
  std::stable_sort(L.begin(), L.end(), [&](uint32_t a, uint32_t b) { return P[a].z32 < P[b].z32; });
  return L;
}

void features(const Scene& s, const Proj& p, int64_t i, double* f) {
  f[0] = s.g.rgb[3 * i];
  f[1] = s.g.rgb[3 * i + 1];
  f[2] = s.g.rgb[3 * i + 2];
  f[3] = p.z;
  for (int c = 0; c < s.c.S; ++c) f[4 + c] = s.g.sem[int64_t(s.c.S) * i + c];
}

struct Contrib {
  uint32_t id;
  double alpha, araw, G, T, dx, dy;
};

// Composites one pixel front to back; returns the contributions in order.
// out[K] accumulates; Tfinal, ncontrib returned; flag set for near-threshold cases.
void composite_pixel(const Scene& s, const std::vector<uint32_t>& L, double px, double py,
                     std::vector<Contrib>& contrib, double* out, double& Tfinal, int& ncontrib, int& flag) {
  const Cfg& c = s.c;
  const auto& P = s.proj;
  int K = s.K();
  std::vector<double> f(K);
  double T = 1.0;
  ncontrib = 0;
  contrib.clear();
  for (size_t pos = 0; pos < L.size(); ++pos) {
    uint32_t i = L[pos];
    const Proj& p = P[i];
    double dx = px - p.m2[0], dy = py - p.m2[1];
    double power = -0.5 * (p.conic[0] * dx * dx + p.conic[2] * dy * dy) - p.conic[1] * dx * dy;
    power = std::min(0.0, power);   // a positive-definite conic gives power <= 0
    double G = std::exp(power);
    double araw = p.o * G;
    if (c.a_min > 0 && near_rel(araw, c.a_min, c.margin)) flag |= 1;
    if (araw < c.a_min) continue;
    if (near_rel(araw, c.a_max, c.margin)) flag |= 2;
    double alpha = std::min(c.a_max, araw);
    double Tn = T * (1.0 - alpha);
    if (c.t_min > 0 && near_rel(Tn, c.t_min, c.margin)) flag |= 4;
    if (Tn < c.t_min) break;
    features(s, p, i, f.data());
    for (int ch = 0; ch < K; ++ch) out[ch] += f[ch] * alpha * T;
    contrib.push_back({i, alpha, araw, G, T, dx, dy});
    T = Tn;
    ncontrib = int(pos) + 1;
  }
  Tfinal = T;
}

struct Views {
  int n;
  const double* vd;
  const int* vi;
};

void setup(Scene& s, const double* cd, const int* ci, int64_t n, const double* mean, const double* lsc,
           const double* quat, const double* opac, const double* rgb, const double* sem, int n_views,
           const double* vd, const int* vi) {
  s.c = read_cfg(cd, ci);
  s.g = {n, mean, lsc, quat, opac, rgb, sem};
  s.n_views = n_views;
  s.vd = vd;
  s.items = make_items(s.c, n_views, vd, vi);
}


// Visits every pixel of every item (optionally only the tiles whose mask byte is set),
// composites it and calls fn(item, u, v, contributions, flag, out). Items are taken one
// at a time (projected, binned, composited); after an item's pixels, done(item) is called
// while its projections are still held. An item with no tile in the mask is skipped.
template <class Fn, class Done>
void for_each_pixel(Scene& s, bool brute, const uint8_t* tile_mask, Fn&& fn, Done&& done) {
  int K = s.K();
  std::vector<Contrib> contrib;
  std::vector<double> out(K);
  for (size_t k = 0; k < s.items.size(); ++k) {
    const Item& it = s.items[k];
    if (tile_mask) {
      bool any = false;
      for (int t = it.tile0; t < it.tile0 + it.ntx * it.nty && !any; ++t) any = tile_mask[t] != 0;
      if (!any) continue;
    }
    build_item(s, int(k), brute);
    for (int ty = 0; ty < it.nty; ++ty)
      for (int tx = 0; tx < it.ntx; ++tx) {
        int tile = it.tile0 + ty * it.ntx + tx;
        if (tile_mask && !tile_mask[tile]) continue;
        std::vector<uint32_t> bl;
        const std::vector<uint32_t>* L = &s.lists[ty * it.ntx + tx];
        if (brute) {
          bl = brute_list(s, tx, ty);
          L = &bl;
        }
        for (int v = ty * s.c.th; v < std::min(it.H, (ty + 1) * s.c.th); ++v)
          for (int u = tx * s.c.tw; u < std::min(it.W, (tx + 1) * s.c.tw); ++u) {
            std::fill(out.begin(), out.end(), 0.0);
            double T;
            int ncontrib, flag = 0;
            composite_pixel(s, *L, u + 0.5, v + 0.5, contrib, out.data(), T, ncontrib, flag);
            for (auto& cb : contrib)
              if (s.proj[cb.id].flag) flag |= 16;
            fn(int(k), u, v, contrib, flag, out.data(), T, ncontrib);
          }
      }
    done(int(k));
  }
}

// Per (item, Gaussian) gradient of the loss with respect to the 2D quantities.
struct G2 {
  double m2[2] = {0, 0}, conic[3] = {0, 0, 0}, o = 0, zf = 0;
};

// Chain rule from the 2D quantities of one (item, Gaussian) back to the Gaussian's
// parameters and the view's pose tangent (rho, phi), T_cw <- Exp(xi) T_cw.
void project_backward(const Scene& s, int k, int64_t i, const G2& g2, double* gmean, double* glsc, double* gquat,
                      double* gopac, double* gpose) {
  const Item& it = s.items[k];
  const Proj& p = s.proj[i];     // item k is the one held
  const double* Rv = s.vd + 16 * it.view;
  double z = p.z, x = p.mc[0], y = p.mc[1];
  // opacity = sigmoid(a)
  gopac[i] += g2.o * p.o * (1.0 - p.o);
  // conic = inverse(cov):  dL/dcov = -Q G Q  with G the symmetric gradient of Q.
  double Q[4] = {p.conic[0], p.conic[1], p.conic[1], p.conic[2]};
  double G[4] = {g2.conic[0], 0.5 * g2.conic[1], 0.5 * g2.conic[1], g2.conic[2]};
  double QG[4], GC[4];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) QG[2 * r + c] = Q[2 * r] * G[c] + Q[2 * r + 1] * G[2 + c];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) GC[2 * r + c] = -(QG[2 * r] * Q[c] + QG[2 * r + 1] * Q[2 + c]);
  if (s.c.isotropic) {
    // cov = diag((fx r/z)^2, (fy r/z)^2) + eps I, r = exp(l): d/dz = -2/z, d/dl = 2 per diagonal entry
    const double vx = std::pow(it.fx * p.s[0] / z, 2), vy = std::pow(it.fy * p.s[0] / z, 2);
    double dmc[3] = {0, 0, -2.0 * (GC[0] * vx + GC[3] * vy) / z};
    glsc[3 * i] += 2.0 * (GC[0] * vx + GC[3] * vy);
    dmc[0] += g2.m2[0] * it.fx / z;
    dmc[1] += g2.m2[1] * it.fy / z;
    dmc[2] += -g2.m2[0] * it.fx * x / (z * z) - g2.m2[1] * it.fy * y / (z * z);
    dmc[2] += g2.zf;
    for (int a = 0; a < 3; ++a) gmean[3 * i + a] += Rv[a] * dmc[0] + Rv[3 + a] * dmc[1] + Rv[6 + a] * dmc[2];
    double* gp = gpose + 6 * it.view;
    for (int a = 0; a < 3; ++a) gp[a] += dmc[a];
    gp[3] += p.mc[1] * dmc[2] - p.mc[2] * dmc[1];
    gp[4] += p.mc[2] * dmc[0] - p.mc[0] * dmc[2];
    gp[5] += p.mc[0] * dmc[1] - p.mc[1] * dmc[0];
    return;
  }
  // cov = J Sc J^T + eps I:  dSc = J^T GC J,  dJ = 2 GC J Sc
  double dSc[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0;
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) acc += p.J[3 * r + a] * GC[2 * r + c] * p.J[3 * c + b];
      dSc[3 * a + b] = acc;
    }
  double dJ[6];
  for (int r = 0; r < 2; ++r)
    for (int b = 0; b < 3; ++b) {
      double acc = 0;
      for (int c = 0; c < 2; ++c)
        for (int m = 0; m < 3; ++m) acc += GC[2 * r + c] * p.J[3 * c + m] * p.Sc[3 * m + b];
      dJ[3 * r + b] = 2.0 * acc;
    }
  double dmc[3] = {0, 0, 0};
  // J = [[fx/z, 0, -fx ux/z], [0, fy/z, -fy uy/z]], ux = clamp(x/z)
  dmc[2] += dJ[0] * (-it.fx / (z * z)) + dJ[4] * (-it.fy / (z * z));
  if (p.clx) {
    dmc[2] += dJ[2] * (it.fx * p.ux / (z * z));
  } else {
    dmc[0] += dJ[2] * (-it.fx / (z * z));
    dmc[2] += dJ[2] * (2.0 * it.fx * x / (z * z * z));
  }
  if (p.cly) {
    dmc[2] += dJ[5] * (it.fy * p.uy / (z * z));
  } else {
    dmc[1] += dJ[5] * (-it.fy / (z * z));
    dmc[2] += dJ[5] * (2.0 * it.fy * y / (z * z * z));
  }
  // m2 = (fx x/z + cx, fy y/z + cy)
  dmc[0] += g2.m2[0] * it.fx / z;
  dmc[1] += g2.m2[1] * it.fy / z;
  dmc[2] += -g2.m2[0] * it.fx * x / (z * z) - g2.m2[1] * it.fy * y / (z * z);
  // composited depth channel
  dmc[2] += g2.zf;
  // mc = W mu + t
  for (int a = 0; a < 3; ++a) gmean[3 * i + a] += Rv[a] * dmc[0] + Rv[3 + a] * dmc[1] + Rv[6 + a] * dmc[2];
  // Sc = W Sigma W^T  ->  dSigma = W^T dSc W
  double tmp[9], dSig[9];
  mTm(Rv, dSc, tmp);
  mm(tmp, Rv, dSig);
  // pose: d mc = rho + phi x mc ;  d Sc = phi^ Sc - Sc phi^
  double* gp = gpose + 6 * it.view;
  for (int a = 0; a < 3; ++a) gp[a] += dmc[a];
  gp[3] += p.mc[1] * dmc[2] - p.mc[2] * dmc[1];
  gp[4] += p.mc[2] * dmc[0] - p.mc[0] * dmc[2];
  gp[5] += p.mc[0] * dmc[1] - p.mc[1] * dmc[0];
  double A1[9], A2[9], X[9];
  mm(p.Sc, dSc, A1);
  mm(dSc, p.Sc, A2);
  for (int a = 0; a < 9; ++a) X[a] = A1[a] - A2[a];
  gp[3] += 2.0 * X[5];
  gp[4] += 2.0 * X[6];
  gp[5] += 2.0 * X[1];
  // Sigma = M M^T  ->  dM = 2 dSigma M
  double dM[9];
  mm(dSig, p.M, dM);
  for (int a = 0; a < 9; ++a) dM[a] *= 2.0;
  double dRq[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) dRq[3 * r + c] = dM[3 * r + c] * p.s[c];
  for (int c = 0; c < 3; ++c) {
    double ds = dM[c] * p.Rq[c] + dM[3 + c] * p.Rq[3 + c] + dM[6 + c] * p.Rq[6 + c];
    glsc[3 * i + c] += ds * p.s[c];
  }
  double w = p.qn[0], qx = p.qn[1], qy = p.qn[2], qz = p.qn[3];
  const double* d = dRq;
  double dq[4];
  dq[0] = 2 * (-qz * d[1] + qy * d[2] + qz * d[3] - qx * d[5] - qy * d[6] + qx * d[7]);
  dq[1] = 2 * (qy * d[1] + qz * d[2] + qy * d[3] - 2 * qx * d[4] - w * d[5] + qz * d[6] + w * d[7] - 2 * qx * d[8]);
  dq[2] = 2 * (-2 * qy * d[0] + qx * d[1] + w * d[2] + qx * d[3] + qz * d[5] - w * d[6] + qz * d[7] - 2 * qy * d[8]);
  dq[3] = 2 * (-2 * qz * d[0] - w * d[1] + qx * d[2] + w * d[3] - 2 * qz * d[4] + qy * d[5] + qx * d[6] + qy * d[7]);
  double dot = w * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
  for (int a = 0; a < 4; ++a) gquat[4 * i + a] += (dq[a] - p.qn[a] * dot) / p.qlen;
}

}  // namespace

extern "C" {

// Sizes of the item table the oracle derives from the views.
int or_layout(const int* ci, int n_views, const int* vi, int* n_items, int64_t* n_pix, int* n_tiles) {
  double cd[8] = {0};
  Cfg c = read_cfg(cd, ci);
  double vd_dummy[16] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 0, 0};
  std::vector<double> vd(16 * size_t(n_views));
  for (int v = 0; v < n_views; ++v) std::memcpy(&vd[16 * v], vd_dummy, sizeof vd_dummy);
  auto items = make_items(c, n_views, vd.data(), vi);
  *n_items = int(items.size());
  int64_t p = 0;
  int t = 0;
  for (auto& it : items) {
    p += int64_t(it.W) * it.H;
    t += it.ntx * it.nty;
  }
  *n_pix = p;
  *n_tiles = t;
  return 0;
}

// Projection of every (item, Gaussian). Outputs are [n_items][n]-indexed:
// m2 x2, conic x3, opacity, depth, radius, rect x4 (tiles), flags; invisible => radius 0.
int or_preprocess(const double* cd, const int* ci, int64_t n, const double* mean, const double* lsc,
                  const double* quat, const double* opac, int n_views, const double* vd, const int* vi, double* m2,
                  double* conic, double* opa, double* depth, int* radius, int* rect, int* flag) {
  Scene s;
  setup(s, cd, ci, n, mean, lsc, quat, opac, nullptr, nullptr, n_views, vd, vi);
  for (size_t k = 0; k < s.items.size(); ++k) {
    const Item& it = s.items[k];
    const double* Rv = vd + 16 * it.view;
    for (int64_t i = 0; i < n; ++i) {
      Proj p = project(s.c, s.g, i, Rv, Rv + 9, it);
      int64_t e = int64_t(k) * n + i;
      radius[e] = p.vis ? p.radius : 0;
      flag[e] = p.flag;
      m2[2 * e] = p.vis ? p.m2[0] : 0;
      m2[2 * e + 1] = p.vis ? p.m2[1] : 0;
      for (int a = 0; a < 3; ++a) conic[3 * e + a] = p.vis ? p.conic[a] : 0;
      opa[e] = p.vis ? p.o : 0;
      depth[e] = p.vis ? p.z : 0;
      for (int a = 0; a < 4; ++a) rect[4 * e + a] = p.vis ? p.rect[a] : 0;
    }
  }
  return 0;
}

// Forward render of every item. img is planar per item: [pix0*K + ch*H*W + y*W + x],
// channels rgb(3), depth(1), semantic(S). brute=1 finds each pixel's set without tile
// lists. tile_mask (may be null) restricts the work to the tiles whose byte is set.
int or_render(const double* cd, const int* ci, int64_t n, const double* mean, const double* lsc, const double* quat,
              const double* opac, const double* rgb, const double* sem, int n_views, const double* vd, const int* vi,
              int brute, const uint8_t* tile_mask, double* img, double* Tout, int* ncontrib, int* pflag,
              int* nblend) {
  Scene s;
  setup(s, cd, ci, n, mean, lsc, quat, opac, rgb, sem, n_views, vd, vi);
  int K = s.K();
  for_each_pixel(s, brute != 0, tile_mask,
                 [&](int k, int u, int v, const std::vector<Contrib>& cb, int flag, const double* out, double T,
                     int nc) {
                   const Item& it = s.items[k];
                   int64_t HW = int64_t(it.W) * it.H, pix = int64_t(v) * it.W + u;
                   for (int ch = 0; ch < K; ++ch) img[it.pix0 * K + ch * HW + pix] = out[ch];
                   Tout[it.pix0 + pix] = T;
                   ncontrib[it.pix0 + pix] = nc;
                   pflag[it.pix0 + pix] = flag;
                   if (nblend) nblend[it.pix0 + pix] = int(cb.size());
                 },
                 [](int) {});
  return 0;
}

// Gradient of sum(gimg * img) with respect to every input (the backward of or_render for
// an upstream gradient gimg in the same planar layout). g2d gets the per (item, Gaussian)
// 2D gradients [m2 x2, conic x3, opacity, depth-channel]; gflag[i] is set when Gaussian i
// contributes to a flagged pixel.
int or_backward(const double* cd, const int* ci, int64_t n, const double* mean, const double* lsc,
                const double* quat, const double* opac, const double* rgb, const double* sem, int n_views,
                const double* vd, const int* vi, const uint8_t* tile_mask, const double* gimg, double* gmean,
                double* glsc, double* gquat, double* gopac, double* grgb, double* gsem, double* gpose, double* g2d,
                int* gflag) {
  Scene s;
  setup(s, cd, ci, n, mean, lsc, quat, opac, rgb, sem, n_views, vd, vi);
  int K = s.K(), S = s.c.S;
  std::vector<G2> g2;                    // [gaussian] of the item being processed
  std::vector<double> f(K), suffix(K), gp(K);
  for_each_pixel(s, false, tile_mask,
                 [&](int k, int u, int v, const std::vector<Contrib>& cb, int flag, const double*, double, int) {
                   const Item& it = s.items[k];
                   if (g2.empty()) g2.assign(size_t(n), G2());
                   int64_t HW = int64_t(it.W) * it.H, pix = int64_t(v) * it.W + u;
                   for (int ch = 0; ch < K; ++ch) gp[ch] = gimg[it.pix0 * K + ch * HW + pix];
                   std::fill(suffix.begin(), suffix.end(), 0.0);
                   for (int q = int(cb.size()) - 1; q >= 0; --q) {
                     const Contrib& c = cb[q];
                     const Proj& p = s.proj[c.id];
                     features(s, p, c.id, f.data());
                     double wgt = c.alpha * c.T;
                     double dalpha = 0;
                     for (int ch = 0; ch < K; ++ch)
                       dalpha += gp[ch] * (f[ch] * c.T - suffix[ch] / (1.0 - c.alpha));
                     for (int ch = 0; ch < K; ++ch) suffix[ch] += f[ch] * wgt;
                     for (int ch = 0; ch < 3; ++ch) grgb[3 * int64_t(c.id) + ch] += wgt * gp[ch];
                     for (int ch = 0; ch < S; ++ch) gsem[int64_t(S) * c.id + ch] += wgt * gp[4 + ch];
                     G2& G = g2[c.id];
                     G.zf += wgt * gp[3];
                     if (c.araw < s.c.a_max) {
                       G.o += dalpha * c.G;
                       double dpow = dalpha * c.araw;
                       G.m2[0] += dpow * (p.conic[0] * c.dx + p.conic[1] * c.dy);
                       G.m2[1] += dpow * (p.conic[2] * c.dy + p.conic[1] * c.dx);
                       G.conic[0] += dpow * (-0.5 * c.dx * c.dx);
                       G.conic[1] += dpow * (-c.dx * c.dy);
                       G.conic[2] += dpow * (-0.5 * c.dy * c.dy);
                     }
                     if (flag && gflag) gflag[c.id] = 1;
                   }
                 },
                 [&](int k) {
                   // the item's 2D gradients back to the parameters and the pose, while its
                   // projections are held (an item without pixels in the mask adds nothing)
                   if (g2.empty()) return;
                   for (int64_t i = 0; i < n; ++i) {
                     const G2& G = g2[i];
                     if (g2d) {
                       double* o = g2d + 7 * (int64_t(k) * n + i);
                       o[0] = G.m2[0]; o[1] = G.m2[1]; o[2] = G.conic[0]; o[3] = G.conic[1]; o[4] = G.conic[2];
                       o[5] = G.o; o[6] = G.zf;
                     }
                     if (!s.proj[i].vis) continue;
                     project_backward(s, k, i, G, gmean, glsc, gquat, gopac, gpose);
                   }
                   g2.clear();
                 });
  return 0;
}

// SSIM of Wang et al. 2004 as used by the RGB term of eq. 10: an 11 x 11 Gaussian window of
// standard deviation 1.5 (normalised to sum 1), applied at every pixel with the image
// taken as zero outside (a same-size map), C1 = 0.01^2, C2 = 0.03^2. Window sums here are
// the plain 2D sums of the definition.
static void ssim_window(double g[11]) {
  double t = 0;
  for (int i = 0; i < 11; ++i) {
    g[i] = std::exp(-double((i - 5) * (i - 5)) / (2.0 * 1.5 * 1.5));
    t += g[i];
  }
  for (int i = 0; i < 11; ++i) g[i] /= t;
}

// out(q) = sum over the window of g(u) g(v) in(q + (u - 5, v - 5)), zero outside.
static void ssim_filter(const double* in, int W, int H, double* out) {
  double g[11];
  ssim_window(g);
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      double a = 0;
      for (int v = 0; v < 11; ++v) {
        const int yy = y + v - 5;
        if (yy < 0 || yy >= H) continue;
        for (int u = 0; u < 11; ++u) {
          const int xx = x + u - 5;
          if (xx < 0 || xx >= W) continue;
          a += g[u] * g[v] * in[int64_t(yy) * W + xx];
        }
      }
      out[int64_t(y) * W + x] = a;
    }
}

// Mean SSIM of one channel x against y; grad (may be null) receives d(mean SSIM)/dx.
static double ssim_channel(const double* x, const double* y, int W, int H, double* grad) {
  const int64_t HW = int64_t(W) * H;
  const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  std::vector<double> xx(HW), yy(HW), xy(HW), m1(HW), m2(HW), e11(HW), e22(HW), e12(HW);
  for (int64_t p = 0; p < HW; ++p) {
    xx[p] = x[p] * x[p];
    yy[p] = y[p] * y[p];
    xy[p] = x[p] * y[p];
  }
  ssim_filter(x, W, H, m1.data());
  ssim_filter(y, W, H, m2.data());
  ssim_filter(xx.data(), W, H, e11.data());
  ssim_filter(yy.data(), W, H, e22.data());
  ssim_filter(xy.data(), W, H, e12.data());
  double sum = 0;
  std::vector<double> A(HW), B(HW), Cc(HW);
  for (int64_t q = 0; q < HW; ++q) {
    const double mu1 = m1[q], mu2 = m2[q];
    const double s11 = e11[q] - mu1 * mu1, s22 = e22[q] - mu2 * mu2, s12 = e12[q] - mu1 * mu2;
    const double a = 2 * mu1 * mu2 + C1, b = 2 * s12 + C2, c = mu1 * mu1 + mu2 * mu2 + C1, d = s11 + s22 + C2;
    const double S = a * b / (c * d);
    sum += S;
    // partial derivatives of S with respect to the window sums of x, x^2 and x y
    A[q] = S * (2 * mu2 / a - 2 * mu2 / b - 2 * mu1 / c + 2 * mu1 / d);
    B[q] = -S / d;
    Cc[q] = 2 * S / b;
  }
  if (grad) {
    // d S(q) / d x(p) reaches p through the window of q: the same (symmetric) window sums
    std::vector<double> fA(HW), fB(HW), fC(HW);
    ssim_filter(A.data(), W, H, fA.data());
    ssim_filter(B.data(), W, H, fB.data());
    ssim_filter(Cc.data(), W, H, fC.data());
    for (int64_t p = 0; p < HW; ++p) grad[p] = (fA[p] + 2 * x[p] * fB[p] + y[p] * fC[p]) / double(HW);
  }
  return sum / double(HW);
}

// Pyramid loss, summed over items: w0 * L_rgb + w1 * mean|D-Dgt| over valid (Dgt > 0)
// pixels + w2 * L_sem, per item, with
//   L_rgb = (1 - lambda_r) mean|R-Rgt| over 3HW + lambda_r (1 - mean SSIM over the 3 channels)
// (eq. 10 with the SSIM term read as 1 - SSIM), lambda_r = w[3], and L_sem either
//   - (tsem == null) the mean cross-entropy of softmax(S) against the label (a label outside
//     [0, S) marks an unlabelled pixel, which adds no term but counts in the mean), or
//   - (tsem != null, S = 3: the semantic feature is a colour) eq. 12, the same form as L_rgb
//     on the semantic colour image against tsem: (1 - lambda_s) mean|S-Sgt| over 3HW +
//     lambda_s (1 - mean SSIM over its 3 channels), lambda_s = w[4].
// loss: [n_items][3] unweighted terms. gimg: dLoss/dimg in the image layout.
int or_loss(const int* ci, int n_views, const int* vi, const double* img, const double* trgb, const double* tdepth,
            const int* tlabel, const double* tsem, const double* w, double* loss, double* gimg) {
  double cd[8] = {0};
  Cfg c = read_cfg(cd, ci);
  if (tsem && c.S != 3) return -1;
  std::vector<double> vd(16 * size_t(n_views), 1.0);
  auto items = make_items(c, n_views, vd.data(), vi);
  int S = c.S, K = 4 + S;
  std::vector<double> sm(S);
  for (size_t k = 0; k < items.size(); ++k) {
    const Item& it = items[k];
    int64_t HW = int64_t(it.W) * it.H;
    const double* I = img + it.pix0 * K;
    double* GI = gimg + it.pix0 * K;
    const double* TR = trgb + it.pix0 * 3;
    const double* TD = tdepth + it.pix0;
    const int* TL = tsem ? nullptr : tlabel + it.pix0;
    const double* TS = tsem ? tsem + it.pix0 * 3 : nullptr;
    int64_t nvalid = 0;
    for (int64_t p = 0; p < HW; ++p) nvalid += TD[p] > 0;
    double lr = 0, ld = 0, ls = 0;
    for (int64_t p = 0; p < HW; ++p) {
      for (int ch = 0; ch < 3; ++ch) {
        double d = I[ch * HW + p] - TR[ch * HW + p];
        lr += std::fabs(d);
        GI[ch * HW + p] = w[0] * ((d > 0) - (d < 0)) / (3.0 * HW);
      }
      double dd = I[3 * HW + p] - TD[p];
      if (TD[p] > 0) {
        ld += std::fabs(dd);
        GI[3 * HW + p] = w[1] * ((dd > 0) - (dd < 0)) / double(nvalid);
      } else {
        GI[3 * HW + p] = 0;
      }
      if (TS) {
        // eq. 12's L1 part: the semantic colour channels against their targets
        for (int ch = 0; ch < 3; ++ch) {
          double d = I[(4 + ch) * HW + p] - TS[ch * HW + p];
          ls += std::fabs(d);
          GI[(4 + ch) * HW + p] = w[2] * ((d > 0) - (d < 0)) / (3.0 * HW);
        }
      } else if (S > 0 && (TL[p] < 0 || TL[p] >= S)) {
        // a label outside [0, S) marks an unlabelled pixel: no cross-entropy term
        for (int ch = 0; ch < S; ++ch) GI[(4 + ch) * HW + p] = 0.0;
      } else if (S > 0) {
        double m = -INFINITY;
        for (int ch = 0; ch < S; ++ch) m = std::max(m, I[(4 + ch) * HW + p]);
        double z = 0;
        for (int ch = 0; ch < S; ++ch) z += std::exp(I[(4 + ch) * HW + p] - m);
        double lse = m + std::log(z);
        ls += lse - I[(4 + TL[p]) * HW + p];
        for (int ch = 0; ch < S; ++ch) {
          double pr = std::exp(I[(4 + ch) * HW + p] - lse);
          GI[(4 + ch) * HW + p] = w[2] * (pr - (ch == TL[p] ? 1.0 : 0.0)) / double(HW);
        }
      }
    }
    const double lam = w[3];
    double ssim = 1.0;
    if (lam != 0.0) {
      double sm3 = 0;
      std::vector<double> gs(HW);
      for (int ch = 0; ch < 3; ++ch) {
        sm3 += ssim_channel(I + ch * HW, TR + ch * HW, it.W, it.H, gs.data());
        for (int64_t p = 0; p < HW; ++p)
          GI[ch * HW + p] = (1.0 - lam) * GI[ch * HW + p] - w[0] * lam * gs[p] / 3.0;
      }
      ssim = sm3 / 3.0;
    }
    loss[3 * k] = (1.0 - lam) * lr / (3.0 * HW) + lam * (1.0 - ssim);
    loss[3 * k + 1] = nvalid ? ld / double(nvalid) : 0.0;
    if (TS) {
      // eq. 12: L1 and SSIM of the semantic colour image, with its own lambda_s
      const double lam_s = w[4];
      double ssim_s = 1.0;
      if (lam_s != 0.0) {
        double sm3 = 0;
        std::vector<double> gs(HW);
        for (int ch = 0; ch < 3; ++ch) {
          sm3 += ssim_channel(I + (4 + ch) * HW, TS + ch * HW, it.W, it.H, gs.data());
          for (int64_t p = 0; p < HW; ++p)
            GI[(4 + ch) * HW + p] = (1.0 - lam_s) * GI[(4 + ch) * HW + p] - w[2] * lam_s * gs[p] / 3.0;
        }
        ssim_s = sm3 / 3.0;
      }
      loss[3 * k + 2] = (1.0 - lam_s) * ls / (3.0 * HW) + lam_s * (1.0 - ssim_s);
    } else {
      loss[3 * k + 2] = S > 0 ? ls / double(HW) : 0.0;
    }
  }
  return 0;
}

// Image pyramid (eq. 4-6) as repeated 2x2 box means of level 0 of every view.
// img holds K planar channels per item in the item layout; level 0 of each view is read,
// the other levels written: channels < 3 and >= 4 by plain means, channel 3 (depth) by the
// mean of its positive children (0 if none). labels (may be null) receive, for every item,
// the argmax over channels >= 4 (ties to the lowest class).
int or_downsample(const int* ci, int n_views, const int* vi, double* img, int* labels) {
  double cd[8] = {0};
  Cfg c = read_cfg(cd, ci);
  std::vector<double> vd(16 * size_t(n_views), 1.0);
  auto items = make_items(c, n_views, vd.data(), vi);
  int K = 4 + c.S;
  for (size_t k = 0; k < items.size(); ++k) {
    const Item& it = items[k];
    int64_t HW = int64_t(it.W) * it.H;
    if (it.level > 0) {
      const Item& up = items[k - 1];
      int64_t HWu = int64_t(up.W) * up.H;
      for (int y = 0; y < it.H; ++y)
        for (int x = 0; x < it.W; ++x)
          for (int ch = 0; ch < K; ++ch) {
            double v[4];
            for (int a = 0; a < 4; ++a)
              v[a] = img[up.pix0 * K + ch * HWu + int64_t(2 * y + a / 2) * up.W + 2 * x + a % 2];
            double r;
            if (ch == 3) {
              double sum = 0;
              int cnt = 0;
              for (int a = 0; a < 4; ++a)
                if (v[a] > 0) { sum += v[a]; ++cnt; }
              r = cnt ? sum / cnt : 0.0;
            } else {
              r = (v[0] + v[1] + v[2] + v[3]) / 4.0;
            }
            img[it.pix0 * K + ch * HW + int64_t(y) * it.W + x] = r;
          }
    }
    if (labels && c.S > 0)
      for (int64_t p = 0; p < HW; ++p) {
        int best = 0;
        for (int ch = 1; ch < c.S; ++ch)
          if (img[it.pix0 * K + (4 + ch) * HW + p] > img[it.pix0 * K + (4 + best) * HW + p]) best = ch;
        labels[it.pix0 + p] = best;
      }
  }
  return 0;
}

// Sort stage on given single-precision projections: for every (item, Gaussian) with
// radius > 0 and a non-empty rect, one entry per tile of its rect with key
// (global tile << 32) | bits(depth) and value = Gaussian index; entries sorted by
// (key, value); ranges[2t], ranges[2t+1] = first and one-past-last entry of tile t,
// (0,0) when empty. The rect uses m = hi + lo of the projected mean and the integer
// radius, exactly. Returns the entry count, or -1 if it exceeds cap.
int64_t or_sort_stage(const int* ci, int n_views, const int* vi, int64_t n, const float* m2hi, const float* m2lo,
                      const int* radius, const float* depth, int64_t cap, uint64_t* keys, uint32_t* vals,
                      uint32_t* ranges) {
  double cd[8] = {0};
  Cfg c = read_cfg(cd, ci);
  std::vector<double> vd(16 * size_t(n_views), 1.0);
  auto items = make_items(c, n_views, vd.data(), vi);
  std::vector<std::pair<uint64_t, uint32_t>> e;
  int tiles = 0;
  for (size_t k = 0; k < items.size(); ++k) {
    const Item& it = items[k];
    tiles += it.ntx * it.nty;
    for (int64_t i = 0; i < n; ++i) {
      int64_t q = int64_t(k) * n + i;
      int r = radius[q];
      if (r <= 0) continue;
      double mx = double(m2hi[2 * q]) + double(m2lo[2 * q]);
      double my = double(m2hi[2 * q + 1]) + double(m2lo[2 * q + 1]);
      int x0 = std::min(it.ntx, std::max(0, int(std::floor((mx - r) / c.tw))));
      int y0 = std::min(it.nty, std::max(0, int(std::floor((my - r) / c.th))));
      int x1 = std::min(it.ntx, std::max(0, int(std::floor((mx + r) / c.tw)) + 1));
      int y1 = std::min(it.nty, std::max(0, int(std::floor((my + r) / c.th)) + 1));
      uint32_t zb;
      std::memcpy(&zb, &depth[q], 4);
      for (int ty = y0; ty < y1; ++ty)
        for (int tx = x0; tx < x1; ++tx)
          e.push_back({(uint64_t(it.tile0 + ty * it.ntx + tx) << 32) | zb, uint32_t(i)});
    }
  }
  if (int64_t(e.size()) > cap) return -1;
  std::sort(e.begin(), e.end());
  for (int t = 0; t < 2 * tiles; ++t) ranges[t] = 0;
  for (size_t j = 0; j < e.size(); ++j) {
    keys[j] = e[j].first;
    vals[j] = e[j].second;
    uint32_t t = uint32_t(e[j].first >> 32);
    if (j == 0 || uint32_t(e[j - 1].first >> 32) != t) ranges[2 * t] = uint32_t(j);
    if (j + 1 == e.size() || uint32_t(e[j + 1].first >> 32) != t) ranges[2 * t + 1] = uint32_t(j + 1);
  }
  return int64_t(e.size());
}

// Learned semantic head on composited embeddings E [P][D]:
// h = relu(W1 E + b1) [P][Hd], logits = W2 h + b2 [P][C]; W1 [Hd][D], W2 [C][Hd].
int or_head_forward(int64_t P, int D, int Hd, int C, const double* E, const double* W1, const double* b1,
                    const double* W2, const double* b2, double* logits) {
  std::vector<double> h(Hd);
  for (int64_t p = 0; p < P; ++p) {
    for (int j = 0; j < Hd; ++j) {
      double a = b1[j];
      for (int d = 0; d < D; ++d) a += W1[int64_t(j) * D + d] * E[p * D + d];
      h[j] = a > 0 ? a : 0;
    }
    for (int c = 0; c < C; ++c) {
      double a = b2[c];
      for (int j = 0; j < Hd; ++j) a += W2[int64_t(c) * Hd + j] * h[j];
      logits[p * C + c] = a;
    }
  }
  return 0;
}

// Backward of or_head_forward for upstream gradient dlogits [P][C]: dE [P][D] and the
// weight gradients (summed over pixels). ReLU'(0) = 0.
int or_head_backward(int64_t P, int D, int Hd, int C, const double* E, const double* W1, const double* b1,
                     const double* W2, const double* dlogits, double* dE, double* dW1, double* db1, double* dW2,
                     double* db2) {
  std::vector<double> h(Hd), dh(Hd);
  for (int64_t p = 0; p < P; ++p) {
    for (int j = 0; j < Hd; ++j) {
      double a = b1[j];
      for (int d = 0; d < D; ++d) a += W1[int64_t(j) * D + d] * E[p * D + d];
      h[j] = a;
    }
    for (int j = 0; j < Hd; ++j) dh[j] = 0;
    for (int c = 0; c < C; ++c) {
      double g = dlogits[p * C + c];
      db2[c] += g;
      for (int j = 0; j < Hd; ++j) {
        double hj = h[j] > 0 ? h[j] : 0;
        dW2[int64_t(c) * Hd + j] += g * hj;
        dh[j] += g * W2[int64_t(c) * Hd + j];
      }
    }
    for (int d = 0; d < D; ++d) dE[p * D + d] = 0;
    for (int j = 0; j < Hd; ++j) {
      double g = h[j] > 0 ? dh[j] : 0;
      db1[j] += g;
      for (int d = 0; d < D; ++d) {
        dW1[int64_t(j) * D + d] += g * E[p * D + d];
        dE[p * D + d] += g * W1[int64_t(j) * D + d];
      }
    }
  }
  return 0;
}

// Distillation objective for fitting the learned head to the plain render (a reading;
// the paper has no learned head): per pixel, the soft-target cross-entropy
// -sum_c softmax(t)_c log softmax(s)_c plus mse_w * mean_c (s_c - t_c)^2, averaged over
// each item's pixels and summed over items. t, s: [P*C] planar per item. grad = dL/ds.
double or_distill(const int* ci, int n_views, const int* vi, int C, const double* t, const double* s, double mse_w,
                  double* grad) {
  double cd[8] = {0};
  Cfg c = read_cfg(cd, ci);
  std::vector<double> vd(16 * size_t(n_views), 1.0);
  auto items = make_items(c, n_views, vd.data(), vi);
  double total = 0;
  std::vector<double> pt(C), ps(C);
  for (const Item& it : items) {
    int64_t HW = int64_t(it.W) * it.H;
    for (int64_t p = 0; p < HW; ++p) {
      const double* T = t + it.pix0 * C + p;
      const double* S = s + it.pix0 * C + p;
      double mt = -INFINITY, ms = -INFINITY;
      for (int k = 0; k < C; ++k) {
        mt = std::max(mt, T[k * HW]);
        ms = std::max(ms, S[k * HW]);
      }
      double zt = 0, zs = 0;
      for (int k = 0; k < C; ++k) {
        zt += std::exp(T[k * HW] - mt);
        zs += std::exp(S[k * HW] - ms);
      }
      double lzt = mt + std::log(zt), lzs = ms + std::log(zs);
      for (int k = 0; k < C; ++k) {
        pt[k] = std::exp(T[k * HW] - lzt);
        ps[k] = std::exp(S[k * HW] - lzs);
      }
      double l = 0;
      for (int k = 0; k < C; ++k) {
        double d = S[k * HW] - T[k * HW];
        l += -pt[k] * (S[k * HW] - lzs) + mse_w * d * d / C;
        grad[it.pix0 * C + p + k * HW] = (ps[k] - pt[k] + 2.0 * mse_w * d / C) / double(HW);
      }
      total += l / double(HW);
    }
  }
  return total;
}

}  // extern "C"
