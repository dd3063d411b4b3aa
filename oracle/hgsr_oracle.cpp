// FP64 CPU oracle for the Gaussian-splat rasterizer -- TEST INFRASTRUCTURE ONLY.
//
// This file is the plain, slow definition of what the renderer computes.  Only
// the test suite, the smoke check and the benchmark's CPU-baseline leg load it;
// the HIP library never links, includes or calls it and the two share no code.
//
// What is computed (the paper's renderer, Sec. 3.1 and Sec. 3.4: colour c and
// feature f of each Gaussian primitive are alpha-blended by the same tile
// rasterization; depth is the camera-space z of Algorithm 1; the pinhole
// projection (U,V) = K (X/Z) is that of Algorithm 1):
//
//  per Gaussian i, world->camera pose (R, t), pinhole (fx, fy, cx, cy, W, H):
//   1. q <- q/|q| (w,x,y,z order), R_q its rotation, S = diag(exp(log_scale)),
//      Sigma_w = R_q S S R_q^T.
//   2. m_c = R mu + t, z = m_c.z; invisible if z <= near.
//   3. EWA: J = [[fx/z, 0, -fx xh/z], [0, fy/z, -fy yh/z]] with xh = m_c.x/z,
//      yh = m_c.y/z clamped to +-1.3 (W/2)/fx and +-1.3 (H/2)/fy;
//      Sigma' = J R Sigma_w R^T J^T + 0.3 I.
//   4. u = fx m_c.x/z + cx, v = fy m_c.y/z + cy (unclamped).
//   5. conic = Sigma'^-1; invisible if opacity o < 1/255.
//   6. colour = max(0, sum_lm k_lm Y_lm(d) + 0.5), d = unit(mu - C), C = -R^T t,
//      Y_lm the real spherical harmonics with the Condon-Shortley phase,
//      coefficient index l^2 + l + m.
//   7. support: k^2 = 2 ln(255 o) is the Mahalanobis radius at which
//      o exp(-q/2) = 1/255; the pixel-centre rectangle is
//      [ceil(u - r_x - 1/2), floor(u + r_x - 1/2)] x (same in v) clipped to the
//      image, r_x = sqrt(k^2 Sigma'_xx), r_y = sqrt(k^2 Sigma'_yy) (the exact
//      bounding box of the ellipse), so that every pair with alpha >= 1/255
//      lies inside it.
//  per pixel centre p = (px + 1/2, py + 1/2), Gaussians ascending by (z, i):
//   T = 1; for each: q = d^T conic d (d = p - (u,v)); alpha = min(0.99, o e^{-q/2});
//   skip if alpha < 1/255; T' = T (1 - alpha); stop (without blending) if
//   T' < 1e-4; else w = alpha T, C += w c, Z += w z, F += w f, T = T'.
//   rgb = C + T bg, alpha = 1 - T, depth = Z / (1 - T) (0 if nothing blended),
//   feat = F.
//
// Two renderers: brute force (every Gaussian at every pixel, one global sort)
// and tiled (per-tile candidate lists from the rectangle of step 7).  They
// must agree bit for bit.  The tiled one also flags "fragile" pixels: pixels
// at which a decision (the 1/255 gate, the 1e-4 stop, the depth order of two
// blended Gaussians) lies within an FP32 error bound of flipping.

#include <algorithm>
#include <limits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int64_t n;
  const float* means;       // n x 3
  const float* log_scales;  // n x 3
  const float* quats;       // n x 4 (w, x, y, z)
  const float* opacities;   // n
  const float* sh;          // n x (deg+1)^2 x 3
  int32_t sh_degree;
  int32_t feat_dim;
  const uint16_t* feat;     // n x feat_dim bf16 bits (may be null when feat_dim == 0)
  // optional double-precision replacements of the float32 arrays (finite
  // differences); each may be null
  const double* means64;
  const double* opac64;
  const double* log_scales64;
  const double* quats64;
  const double* sh64;
  const double* feat64;
} orc_scene;

typedef struct {
  double fx, fy, cx, cy;
  int32_t width, height;
  double near_z;
  double bg[3];
} orc_camera;

}  // extern "C"

namespace {

constexpr double kAlphaMin = 1.0 / 255.0;
constexpr double kAlphaMax = 0.99;
constexpr double kTMin = 1e-4;
constexpr double kDilation = 0.3;
constexpr double kGuard = 1.3;
constexpr double kEps32 = 5.9604644775390625e-08;  // 2^-24, FP32 unit roundoff

double bf16_to_double(uint16_t b) {
  uint32_t bits = static_cast<uint32_t>(b) << 16;
  float f;
  std::memcpy(&f, &bits, 4);
  return static_cast<double>(f);
}

// ---------------------------------------------------------------- SH basis
// Associated Legendre P_l^m(x), m >= 0, with the Condon-Shortley phase, from
// the standard three-term recurrence in l.
double assoc_legendre(int l, int m, double x) {
  double pmm = 1.0;
  if (m > 0) {
    const double s = std::sqrt(std::max(0.0, (1.0 - x) * (1.0 + x)));
    double fact = 1.0;
    for (int i = 1; i <= m; ++i) {
      pmm *= -fact * s;
      fact += 2.0;
    }
  }
  if (l == m) return pmm;
  double pmmp1 = x * (2 * m + 1) * pmm;
  if (l == m + 1) return pmmp1;
  double pll = 0.0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pll = (x * (2 * ll - 1) * pmmp1 - (ll + m - 1) * pmm) / (ll - m);
    pmm = pmmp1;
    pmmp1 = pll;
  }
  return pll;
}

double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

// Real SH value Y_lm at unit direction d (m in [-l, l]).
double real_sh(int l, int m, const double d[3]) {
  const int am = m < 0 ? -m : m;
  const double K = std::sqrt((2 * l + 1) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
  const double ct = std::max(-1.0, std::min(1.0, d[2]));
  const double phi = std::atan2(d[1], d[0]);
  const double P = assoc_legendre(l, am, ct);
  if (m > 0) return std::sqrt(2.0) * K * std::cos(am * phi) * P;
  if (m < 0) return std::sqrt(2.0) * K * std::sin(am * phi) * P;
  return K * P;
}

// ---------------------------------------------------------------- projection
struct Proj {
  int visible = 0;
  double mc[3]{};
  double u = 0, v = 0, z = 0;
  double cov2[3]{};   // Sigma' xx, xy, yy (with dilation)
  double conic[3]{};  // a, b, c
  double o = 0;
  double rgb[3]{};
  double rx = 0, ry = 0;
  double bx0 = 0, bx1 = 0, by0 = 0, by1 = 0;
  int px0 = 0, px1 = -1, py0 = 0, py1 = -1;
  double cov3[6]{};   // Sigma_w xx, xy, xz, yy, yz, zz
  double err_u = 0, err_v = 0, err_z = 0, err_conic = 0;
};

struct Pose {
  double R[3][3];
  double t[3];
};

// Smallest conic distance q(p - mean) = a dx^2 + 2 b dx dy + c dy^2 over the
// rectangle [x0, x1] x [y0, y1].  q is convex: 0 when the mean lies inside,
// otherwise the minimum lies on an edge, where q is a one-variable quadratic
// minimised at its stationary point clamped to the edge.
double min_q_box(double a, double b, double c, double u, double v, double x0, double x1, double y0, double y1) {
  if (u >= x0 && u <= x1 && v >= y0 && v <= y1) return 0.0;
  auto q = [&](double dx, double dy) { return a * dx * dx + 2.0 * b * dx * dy + c * dy * dy; };
  double best = std::numeric_limits<double>::infinity();
  for (double xe : {x0, x1}) {  // edges x = xe
    const double dx = xe - u;
    const double dy = std::min(std::max(-b * dx / c, y0 - v), y1 - v);
    best = std::min(best, q(dx, dy));
  }
  for (double ye : {y0, y1}) {  // edges y = ye
    const double dy = ye - v;
    const double dx = std::min(std::max(-b * dy / a, x0 - u), x1 - u);
    best = std::min(best, q(dx, dy));
  }
  return best;
}

Pose make_pose(const double* p) {
  Pose P;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) P.R[r][c] = p[r * 4 + c];
    P.t[r] = p[r * 4 + 3];
  }
  return P;
}

// Steps 1-8 of the header for Gaussian i.  When `force` is set the culls are
// not applied (used by the frozen-decision renderer for finite differences).
Proj project(const orc_scene& s, int64_t i, const Pose& P, const orc_camera& cam, bool force) {
  Proj g;
  double m[3];
  if (s.means64) {
    for (int k = 0; k < 3; ++k) m[k] = s.means64[3 * i + k];
  } else {
    for (int k = 0; k < 3; ++k) m[k] = s.means[3 * i + k];
  }
  // 1. covariance in the world frame
  double qw, qx, qy, qz;
  if (s.quats64) {
    qw = s.quats64[4 * i]; qx = s.quats64[4 * i + 1]; qy = s.quats64[4 * i + 2]; qz = s.quats64[4 * i + 3];
  } else {
    qw = s.quats[4 * i]; qx = s.quats[4 * i + 1]; qy = s.quats[4 * i + 2]; qz = s.quats[4 * i + 3];
  }
  const double qn = std::sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw /= qn; qx /= qn; qy /= qn; qz /= qn;
  const double Rq[3][3] = {
      {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
      {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
      {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
  double ls[3];
  for (int k = 0; k < 3; ++k) ls[k] = s.log_scales64 ? s.log_scales64[3 * i + k] : s.log_scales[3 * i + k];
  const double s2[3] = {std::exp(2.0 * ls[0]), std::exp(2.0 * ls[1]), std::exp(2.0 * ls[2])};
  double Sw[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += Rq[a][k] * s2[k] * Rq[b][k];
      Sw[a][b] = acc;
    }
  g.cov3[0] = Sw[0][0]; g.cov3[1] = Sw[0][1]; g.cov3[2] = Sw[0][2];
  g.cov3[3] = Sw[1][1]; g.cov3[4] = Sw[1][2]; g.cov3[5] = Sw[2][2];
  // 2. camera-space mean
  double mag[3];
  for (int r = 0; r < 3; ++r) {
    g.mc[r] = P.R[r][0] * m[0] + P.R[r][1] * m[1] + P.R[r][2] * m[2] + P.t[r];
    mag[r] = std::fabs(P.R[r][0] * m[0]) + std::fabs(P.R[r][1] * m[1]) + std::fabs(P.R[r][2] * m[2]) +
             std::fabs(P.t[r]);
  }
  g.z = g.mc[2];
  g.o = s.opac64 ? s.opac64[i] : static_cast<double>(s.opacities[i]);
  if (!force && (g.z <= cam.near_z || g.o < kAlphaMin)) return g;
  // 3. EWA projection of the covariance
  const double z = g.z;
  const double limx = kGuard * (0.5 * cam.width) / cam.fx;
  const double limy = kGuard * (0.5 * cam.height) / cam.fy;
  const double xh = std::max(-limx, std::min(limx, g.mc[0] / z));
  const double yh = std::max(-limy, std::min(limy, g.mc[1] / z));
  const double J[2][3] = {{cam.fx / z, 0.0, -cam.fx * xh / z}, {0.0, cam.fy / z, -cam.fy * yh / z}};
  double M[2][3];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b) M[a][b] = J[a][0] * P.R[0][b] + J[a][1] * P.R[1][b] + J[a][2] * P.R[2][b];
  double C2[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      double acc = 0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc += M[a][k] * Sw[k][l] * M[b][l];
      C2[a][b] = acc;
    }
  g.cov2[0] = C2[0][0] + kDilation;
  g.cov2[1] = C2[0][1];
  g.cov2[2] = C2[1][1] + kDilation;
  // 4. projected mean
  g.u = cam.fx * g.mc[0] / z + cam.cx;
  g.v = cam.fy * g.mc[1] / z + cam.cy;
  // 5. conic
  const double det = g.cov2[0] * g.cov2[2] - g.cov2[1] * g.cov2[1];
  g.conic[0] = g.cov2[2] / det;
  g.conic[1] = -g.cov2[1] / det;
  g.conic[2] = g.cov2[0] / det;
  // 6. colour from spherical harmonics, view direction from the camera centre
  double Cc[3];
  for (int r = 0; r < 3; ++r) Cc[r] = -(P.R[0][r] * P.t[0] + P.R[1][r] * P.t[1] + P.R[2][r] * P.t[2]);
  double d[3] = {m[0] - Cc[0], m[1] - Cc[1], m[2] - Cc[2]};
  const double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  d[0] /= dn; d[1] /= dn; d[2] /= dn;
  const int K = (s.sh_degree + 1) * (s.sh_degree + 1);
  const int64_t shb = static_cast<int64_t>(K) * 3 * i;
  for (int c = 0; c < 3; ++c) g.rgb[c] = 0.5;
  for (int l = 0; l <= s.sh_degree; ++l)
    for (int mm = -l; mm <= l; ++mm) {
      const double y = real_sh(l, mm, d);
      const int k = l * l + l + mm;
      for (int c = 0; c < 3; ++c)
        g.rgb[c] += (s.sh64 ? s.sh64[shb + 3 * k + c] : static_cast<double>(s.sh[shb + 3 * k + c])) * y;
    }
  for (int c = 0; c < 3; ++c) g.rgb[c] = std::max(0.0, g.rgb[c]);
  // 7. support rectangle
  if (g.o >= kAlphaMin) {
    const double k2 = 2.0 * std::log(255.0 * g.o);
    g.rx = std::sqrt(k2 * g.cov2[0]);
    g.ry = std::sqrt(k2 * g.cov2[2]);
    g.bx0 = g.u - g.rx - 0.5;
    g.bx1 = g.u + g.rx - 0.5;
    g.by0 = g.v - g.ry - 0.5;
    g.by1 = g.v + g.ry - 0.5;
    g.px0 = static_cast<int>(std::max(0.0, std::ceil(g.bx0)));
    g.px1 = static_cast<int>(std::min<double>(cam.width - 1, std::floor(g.bx1)));
    g.py0 = static_cast<int>(std::max(0.0, std::ceil(g.by0)));
    g.py1 = static_cast<int>(std::min<double>(cam.height - 1, std::floor(g.by1)));
    // guard against huge doubles converting out of int range
    if (g.bx1 < 0 || g.by1 < 0 || g.bx0 > cam.width || g.by0 > cam.height) {
      g.px0 = 0; g.px1 = -1; g.py0 = 0; g.py1 = -1;
    }
  }
  g.visible = (g.z > cam.near_z && g.o >= kAlphaMin && g.px0 <= g.px1 && g.py0 <= g.py1) ? 1 : 0;
  // FP32 error bounds of the renderer's arithmetic (for fragile-pixel flags):
  // each camera-space coordinate is a chain of three fused multiply-adds, so
  // its rounding error is at most 1.5 units in the last place of the largest
  // partial sum, bounded by the sum of the terms' magnitudes; the projection
  // adds a quotient and a fused multiply-add.  The conic inherits the relative
  // error of the covariance chain amplified by the conditioning of det.
  const double ex = 1.5 * kEps32 * mag[0], ey = 1.5 * kEps32 * mag[1], ez = 1.5 * kEps32 * mag[2];
  g.err_z = ez;
  g.err_u = cam.fx * (ex / z + std::fabs(g.mc[0]) * ez / (z * z)) +
            kEps32 * (cam.fx * std::fabs(g.mc[0] / z) + std::fabs(g.u));
  g.err_v = cam.fy * (ey / z + std::fabs(g.mc[1]) * ez / (z * z)) +
            kEps32 * (cam.fy * std::fabs(g.mc[1] / z) + std::fabs(g.v));
  g.err_conic = kEps32 * (12.0 + 2.0 * (g.cov2[0] * g.cov2[2] + g.cov2[1] * g.cov2[1]) / det);
  return g;
}

struct PixelOut {
  double rgb[3];
  double depth, alpha, T;
  int32_t nblend;
  uint8_t fragile;
};

// Per-pixel front-to-back walk over Gaussians already in (z, i) order.
// `feat_out` receives D values.  `list_out` (optional) receives the indices of
// blended Gaussians in order.  Returns the number of tested pairs.
int64_t walk_pixel(const orc_scene& s, const orc_camera& cam, const std::vector<Proj>& pr,
                   const int32_t* order, int64_t count, int px, int py, PixelOut& out, double* feat_out,
                   int32_t* list_out, int32_t list_cap, bool* list_overflow, int64_t* walked = nullptr) {
  const int D = s.feat_dim;
  double T = 1.0, C[3] = {0, 0, 0}, Z = 0.0;
  for (int k = 0; k < D; ++k) feat_out[k] = 0.0;
  int32_t nb = 0;
  bool frag = false;
  double lnT_err = 0.0;
  double prev_z = -1.0, prev_ez = 0.0;
  bool stopped = false;
  int64_t tested = 0;
  const double pxc = px + 0.5, pyc = py + 0.5;
  if (walked) *walked = count;
  for (int64_t j = 0; j < count; ++j) {
    const int32_t gi = order[j];
    const Proj& g = pr[gi];
    const double dx = pxc - g.u, dy = pyc - g.v;
    const double q = g.conic[0] * dx * dx + 2.0 * g.conic[1] * dx * dy + g.conic[2] * dy * dy;
    if (!stopped) ++tested;
    if (q < 0.0) continue;
    const double araw = g.o * std::exp(-0.5 * q);
    // FP32 error bound of ln(alpha) at this pair: position error through the
    // gradient of q, conic error, the rounding of the quadratic form, the
    // exponential (argument scaling and result) and the opacity product;
    // times a safety factor of 2.
    const double dqdu = 2.0 * std::fabs(g.conic[0] * dx + g.conic[1] * dy);
    const double dqdv = 2.0 * std::fabs(g.conic[1] * dx + g.conic[2] * dy);
    const double qabs = std::fabs(g.conic[0]) * dx * dx + 2.0 * std::fabs(g.conic[1] * dx * dy) +
                        std::fabs(g.conic[2]) * dy * dy;
    const double dln = 2.0 * (0.5 * (dqdu * g.err_u + dqdv * g.err_v) + 0.5 * q * g.err_conic +
                              2.0 * kEps32 * qabs + 2.0 * kEps32 * (2.0 + 0.5 * q));
    const double alpha = std::min(kAlphaMax, araw);
    if (alpha < kAlphaMin) {
      if (!stopped && std::fabs(std::log(araw * 255.0)) <= dln) frag = true;
      continue;
    }
    if (!stopped && std::fabs(std::log(araw * 255.0)) <= dln) frag = true;
    // depth-order near-ties among Gaussians that pass the gate
    const double ez = 2.0 * g.err_z;
    if (prev_z >= 0.0 && std::fabs(g.z - prev_z) <= ez + prev_ez) frag = true;
    prev_z = g.z;
    prev_ez = ez;
    if (stopped) {  // only the next gate-passing Gaussian matters after a stop
      if (walked) *walked = j + 1;
      break;
    }
    const double Tn = T * (1.0 - alpha);
    lnT_err += (alpha / (1.0 - alpha)) * dln + 4 * kEps32;
    if (std::fabs(std::log(Tn / kTMin)) <= 2.0 * lnT_err) frag = true;
    if (Tn < kTMin) {
      stopped = true;
      continue;
    }
    const double w = alpha * T;
    for (int c = 0; c < 3; ++c) C[c] += w * g.rgb[c];
    Z += w * g.z;
    if (D) {
      const int64_t fb = static_cast<int64_t>(D) * gi;
      for (int k = 0; k < D; ++k) feat_out[k] += w * (s.feat64 ? s.feat64[fb + k] : bf16_to_double(s.feat[fb + k]));
    }
    T = Tn;
    if (list_out) {
      if (nb < list_cap) list_out[nb] = gi;
      else *list_overflow = true;
    }
    ++nb;
  }
  for (int c = 0; c < 3; ++c) out.rgb[c] = C[c] + T * cam.bg[c];
  out.alpha = 1.0 - T;
  out.depth = (1.0 - T) > 0.0 ? Z / (1.0 - T) : 0.0;
  out.T = T;
  out.nblend = nb;
  out.fragile = frag ? 1 : 0;
  return tested;
}

bool z_index_less(const std::vector<Proj>& pr, int32_t a, int32_t b) {
  if (pr[a].z != pr[b].z) return pr[a].z < pr[b].z;
  return a < b;
}

void store_pixel(const PixelOut& po, const double* f, int D, int64_t pix, int64_t HW, double* rgb, double* depth,
                 double* alpha, double* feat, double* finalT, int32_t* nblend, uint8_t* fragile) {
  for (int c = 0; c < 3; ++c) rgb[c * HW + pix] = po.rgb[c];
  depth[pix] = po.depth;
  alpha[pix] = po.alpha;
  if (finalT) finalT[pix] = po.T;
  if (nblend) nblend[pix] = po.nblend;
  if (fragile) fragile[pix] = po.fragile;
  if (feat)
    for (int k = 0; k < D; ++k) feat[k * HW + pix] = f[k];
}

// Tile listing rule: a visible Gaussian is listed in the tiles of its pixel
// rectangle (step 7) whose rectangle of pixel centres (clipped to the image,
// grown by `grow` px on each side) meets the support ellipse q <= k^2,
// k^2 = 2 ln(255 o).  Every pixel where the Gaussian passes the 1/255 gate
// lies in such a tile, so the tiled render equals the per-pixel definition.
// slack widens the threshold to k^2 (1 + slack) + 10 slack (edge tests).
bool tile_meets(const Proj& g, int tx, int ty, int tile, int W, int H, double grow, double slack = 0.0) {
  const double x0 = tx * tile + 0.5 - grow, x1 = std::min((tx + 1) * tile, W) - 0.5 + grow;
  const double y0 = ty * tile + 0.5 - grow, y1 = std::min((ty + 1) * tile, H) - 0.5 + grow;
  const double k2 = 2.0 * std::log(255.0 * g.o);
  return min_q_box(g.conic[0], g.conic[1], g.conic[2], g.u, g.v, x0, x1, y0, y1) <= k2 * (1.0 + slack) + 10.0 * slack;
}

}  // namespace

extern "C" {

// Per-Gaussian projection dump.  dbl: n x 31 doubles in the order
// [u, v, z, cov_xx, cov_xy, cov_yy, conic_a, conic_b, conic_c, o, r, g, b, rx, ry,
//  mc_x, mc_y, mc_z, cov3_xx, cov3_xy, cov3_xz, cov3_yy, cov3_yz, cov3_zz,
//  bx0, bx1, by0, by1, err_u, err_v, err_z];  ints: n x 5 [visible, px0, px1, py0, py1].
int orc_project(const orc_scene* s, const double* pose, const orc_camera* cam, double* dbl, int32_t* ints) {
  const Pose P = make_pose(pose);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < s->n; ++i) {
    const Proj g = project(*s, i, P, *cam, false);
    double* o = dbl + 31 * i;
    const double vals[31] = {g.u, g.v, g.z, g.cov2[0], g.cov2[1], g.cov2[2], g.conic[0], g.conic[1], g.conic[2],
                             g.o, g.rgb[0], g.rgb[1], g.rgb[2], g.rx, g.ry, g.mc[0], g.mc[1], g.mc[2],
                             g.cov3[0], g.cov3[1], g.cov3[2], g.cov3[3], g.cov3[4], g.cov3[5],
                             g.bx0, g.bx1, g.by0, g.by1, g.err_u, g.err_v, g.err_z};
    std::memcpy(o, vals, sizeof(vals));
    int32_t* n = ints + 5 * i;
    n[0] = g.visible; n[1] = g.px0; n[2] = g.px1; n[3] = g.py0; n[4] = g.py1;
  }
  return 0;
}

// Render one pose.  mode 0: brute force (global (z, i) sort, every visible
// Gaussian tested at every pixel); mode 1: tiled (per-tile lists by the tile
// listing rule, with the pixel rectangle and the tiles' centre rectangles
// grown by `margin_px` pixels).
// Outputs (caller-allocated): rgb 3xHxW, depth HxW, alpha HxW, feat DxHxW (or
// null), finalT HxW, nblend HxW, fragile HxW (any may be null except rgb, depth,
// alpha).  stats[4] = {visible, keys, tested pairs, blended pairs}.
// lists (optional): H*W*list_cap indices of blended Gaussians per pixel.
// Returns 0, or 2 if a per-pixel list overflowed list_cap.
int orc_render(const orc_scene* s, const double* pose, const orc_camera* cam, int32_t mode, int32_t tile,
               int32_t margin_px, double* rgb, double* depth, double* alpha, double* feat, double* finalT,
               int32_t* nblend, uint8_t* fragile, int64_t* stats, int32_t* lists, int32_t list_cap) {
  const Pose P = make_pose(pose);
  const int W = cam->width, H = cam->height, D = s->feat_dim;
  const int64_t HW = static_cast<int64_t>(W) * H;
  std::vector<Proj> pr(s->n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < s->n; ++i) pr[i] = project(*s, i, P, *cam, false);
  int64_t visible = 0, keys = 0;
  for (int64_t i = 0; i < s->n; ++i) visible += pr[i].visible;
  int64_t tested = 0, blended = 0;
  bool overflow = false;
  if (mode == 0) {
    std::vector<int32_t> order;
    for (int64_t i = 0; i < s->n; ++i)
      if (pr[i].z > cam->near_z && pr[i].o >= kAlphaMin) order.push_back(static_cast<int32_t>(i));
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return z_index_less(pr, a, b); });
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tested, blended)
    for (int py = 0; py < H; ++py) {
      std::vector<double> f(D > 0 ? D : 1);
      bool ovf = false;
      for (int px = 0; px < W; ++px) {
        PixelOut po;
        const int64_t pix = static_cast<int64_t>(py) * W + px;
        tested += walk_pixel(*s, *cam, pr, order.data(), static_cast<int64_t>(order.size()), px, py, po, f.data(),
                             lists ? lists + pix * list_cap : nullptr, list_cap, &ovf);
        blended += po.nblend;
        store_pixel(po, f.data(), D, pix, HW, rgb, depth, alpha, feat, finalT, nblend, fragile);
      }
      if (ovf) {
#pragma omp critical
        overflow = true;
      }
    }
  } else {
    const int ntx = (W + tile - 1) / tile, nty = (H + tile - 1) / tile;
    std::vector<std::vector<int32_t>> bins(static_cast<size_t>(ntx) * nty);
    for (int64_t i = 0; i < s->n; ++i) {
      const Proj& g = pr[i];
      if (!g.visible) continue;
      const int x0 = std::max(0, g.px0 - margin_px), x1 = std::min(W - 1, g.px1 + margin_px);
      const int y0 = std::max(0, g.py0 - margin_px), y1 = std::min(H - 1, g.py1 + margin_px);
      for (int ty = y0 / tile; ty <= y1 / tile; ++ty)
        for (int tx = x0 / tile; tx <= x1 / tile; ++tx) {
          if (!tile_meets(g, tx, ty, tile, W, H, static_cast<double>(margin_px))) continue;
          bins[static_cast<size_t>(ty) * ntx + tx].push_back(static_cast<int32_t>(i));
          ++keys;
        }
    }
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tested, blended)
    for (int64_t b = 0; b < static_cast<int64_t>(bins.size()); ++b) {
      std::vector<int32_t>& lst = bins[b];
      std::sort(lst.begin(), lst.end(), [&](int32_t a, int32_t c) { return z_index_less(pr, a, c); });
      const int tx = static_cast<int>(b % ntx), ty = static_cast<int>(b / ntx);
      std::vector<double> f(D > 0 ? D : 1);
      bool ovf = false;
      for (int py = ty * tile; py < std::min(H, (ty + 1) * tile); ++py)
        for (int px = tx * tile; px < std::min(W, (tx + 1) * tile); ++px) {
          PixelOut po;
          const int64_t pix = static_cast<int64_t>(py) * W + px;
          tested += walk_pixel(*s, *cam, pr, lst.data(), static_cast<int64_t>(lst.size()), px, py, po, f.data(),
                               lists ? lists + pix * list_cap : nullptr, list_cap, &ovf);
          blended += po.nblend;
          store_pixel(po, f.data(), D, pix, HW, rgb, depth, alpha, feat, finalT, nblend, fragile);
        }
      if (ovf) {
#pragma omp critical
        overflow = true;
      }
    }
  }
  if (stats) {
    stats[0] = visible;
    stats[1] = keys;
    stats[2] = tested;
    stats[3] = blended;
  }
  return overflow ? 2 : 0;
}

// Render with frozen decisions: every pixel blends exactly the Gaussians
// listed for it (in the listed order), with alpha = min(0.99, o e^{-q/2}) and
// no 1/255 gate or 1e-4 stop.  This is the smooth branch of the renderer that
// contains the reference pose, used for finite differences.
int orc_render_frozen(const orc_scene* s, const double* pose, const orc_camera* cam, const int32_t* lists,
                      const int32_t* counts, int32_t list_cap, double* rgb, double* depth, double* alpha,
                      double* feat, double* finalT) {
  const Pose P = make_pose(pose);
  const int W = cam->width, H = cam->height, D = s->feat_dim;
  const int64_t HW = static_cast<int64_t>(W) * H;
  std::vector<uint8_t> used(s->n, 0);
  for (int64_t p = 0; p < HW; ++p)
    for (int32_t k = 0; k < counts[p]; ++k) used[lists[p * list_cap + k]] = 1;
  std::vector<Proj> pr(s->n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < s->n; ++i)
    if (used[i]) pr[i] = project(*s, i, P, *cam, true);
#pragma omp parallel for schedule(static)
  for (int py = 0; py < H; ++py) {
    std::vector<double> F(D > 0 ? D : 1);
    for (int px = 0; px < W; ++px) {
      const int64_t pix = static_cast<int64_t>(py) * W + px;
      double T = 1.0, C[3] = {0, 0, 0}, Z = 0.0;
      for (int k = 0; k < D; ++k) F[k] = 0.0;
      for (int32_t k = 0; k < counts[pix]; ++k) {
        const int32_t gi = lists[pix * list_cap + k];
        const Proj& g = pr[gi];
        const double dx = px + 0.5 - g.u, dy = py + 0.5 - g.v;
        const double q = g.conic[0] * dx * dx + 2.0 * g.conic[1] * dx * dy + g.conic[2] * dy * dy;
        const double a = std::min(kAlphaMax, g.o * std::exp(-0.5 * q));
        const double w = a * T;
        for (int c = 0; c < 3; ++c) C[c] += w * g.rgb[c];
        Z += w * g.z;
        if (D) {
          const int64_t fb = static_cast<int64_t>(D) * gi;
          for (int j = 0; j < D; ++j) F[j] += w * (s->feat64 ? s->feat64[fb + j] : bf16_to_double(s->feat[fb + j]));
        }
        T *= (1.0 - a);
      }
      PixelOut po;
      for (int c = 0; c < 3; ++c) po.rgb[c] = C[c] + T * cam->bg[c];
      po.alpha = 1.0 - T;
      po.depth = (1.0 - T) > 0.0 ? Z / (1.0 - T) : 0.0;
      po.T = T;
      po.nblend = counts[pix];
      po.fragile = 0;
      store_pixel(po, F.data(), D, pix, HW, rgb, depth, alpha, feat, finalT, nullptr, nullptr);
    }
  }
  return 0;
}

// Per-tile candidate lists in (z, i) order (the tile listing rule, no
// margin).  offsets: ntiles + 1 entries; ids: capacity `cap` (may be null to
// query the total, returned in *total).  edge[i] = 1 when Gaussian i's tile set
// changes if any pixel-rectangle bound, or the centre rectangle of any tile
// it may reach, moves by up to `edge_px` pixels, or the ellipse threshold by
// a relative 2e-5 (+2e-4).
int orc_tile_lists(const orc_scene* s, const double* pose, const orc_camera* cam, int32_t tile, double edge_px,
                   int64_t* offsets, int32_t* ids, int64_t cap, uint8_t* edge, int64_t* total) {
  const Pose P = make_pose(pose);
  const int W = cam->width, H = cam->height;
  const int ntx = (W + tile - 1) / tile, nty = (H + tile - 1) / tile;
  std::vector<Proj> pr(s->n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < s->n; ++i) pr[i] = project(*s, i, P, *cam, false);
  // tile rectangle from real-valued bounds (visible iff non-empty)
  auto tiles_of = [&](double bx0, double bx1, double by0, double by1, int r[4]) {
    const double x0 = std::max(0.0, std::ceil(bx0)), x1 = std::min<double>(W - 1, std::floor(bx1));
    const double y0 = std::max(0.0, std::ceil(by0)), y1 = std::min<double>(H - 1, std::floor(by1));
    if (x0 > x1 || y0 > y1) {
      r[0] = 0; r[1] = -1; r[2] = 0; r[3] = -1;
      return;
    }
    r[0] = static_cast<int>(x0) / tile; r[1] = static_cast<int>(x1) / tile;
    r[2] = static_cast<int>(y0) / tile; r[3] = static_cast<int>(y1) / tile;
  };
  std::vector<std::vector<int32_t>> bins(static_cast<size_t>(ntx) * nty);
  for (int64_t i = 0; i < s->n; ++i) {
    const Proj& g = pr[i];
    if (edge) edge[i] = 0;
    const bool front = g.z > cam->near_z && g.o >= kAlphaMin;
    if (front && edge) {
      int lo[4], hi[4];
      tiles_of(g.bx0 + edge_px, g.bx1 - edge_px, g.by0 + edge_px, g.by1 - edge_px, lo);
      tiles_of(g.bx0 - edge_px, g.bx1 + edge_px, g.by0 - edge_px, g.by1 + edge_px, hi);
      if (lo[0] != hi[0] || lo[1] != hi[1] || lo[2] != hi[2] || lo[3] != hi[3]) edge[i] = 1;
      for (int ty = std::max(hi[2], 0); ty <= hi[3] && !edge[i]; ++ty)
        for (int tx = std::max(hi[0], 0); tx <= hi[1]; ++tx)
          if (tile_meets(g, tx, ty, tile, W, H, edge_px, 2e-5) != tile_meets(g, tx, ty, tile, W, H, -edge_px)) {
            edge[i] = 1;
            break;
          }
    }
    if (!g.visible) continue;
    for (int ty = g.py0 / tile; ty <= g.py1 / tile; ++ty)
      for (int tx = g.px0 / tile; tx <= g.px1 / tile; ++tx)
        if (tile_meets(g, tx, ty, tile, W, H, 0.0))
          bins[static_cast<size_t>(ty) * ntx + tx].push_back(static_cast<int32_t>(i));
  }
  int64_t acc = 0;
  for (size_t b = 0; b < bins.size(); ++b) {
    std::sort(bins[b].begin(), bins[b].end(), [&](int32_t a, int32_t c) { return z_index_less(pr, a, c); });
    if (offsets) offsets[b] = acc;
    if (ids)
      for (size_t k = 0; k < bins[b].size(); ++k)
        if (acc + static_cast<int64_t>(k) < cap) ids[acc + k] = bins[b][k];
    acc += static_cast<int64_t>(bins[b].size());
  }
  if (offsets) offsets[bins.size()] = acc;
  *total = acc;
  return (ids && acc > cap) ? 2 : 0;
}

// Which Gaussians contribute to the rendered image (the render-gradient
// visibility check of Sec. 3.2 and its algorithm: after rendering and a
// backward pass of the summed RGB, a Gaussian is visible where its mean
// receives a nonzero gradient, i.e. where it is blended, with weight
// alpha T > 0, at one pixel at least).  Per Gaussian i:
//   contrib[i]  = 1 if it is blended at some pixel;
//   robust[i]   = 1 if it is blended at some pixel that is not fragile;
//   touched[i]  = 1 if some fragile pixel's walk reached it (tested it before
//                 the walk ended).
// A Gaussian with robust = 0 and touched = 1 may be decided either way by an
// FP32 renderer; every other Gaussian's contrib is fixed.  Tiled walk, lists by
// the tile listing rule (equal to the brute-force walk).
int orc_contrib(const orc_scene* s, const double* pose, const orc_camera* cam, int32_t tile, uint8_t* contrib,
                uint8_t* robust, uint8_t* touched) {
  const Pose P = make_pose(pose);
  const int W = cam->width, H = cam->height, D = s->feat_dim;
  const int ntx = (W + tile - 1) / tile, nty = (H + tile - 1) / tile;
  std::vector<Proj> pr(s->n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < s->n; ++i) pr[i] = project(*s, i, P, *cam, false);
  std::vector<std::vector<int32_t>> bins(static_cast<size_t>(ntx) * nty);
  for (int64_t i = 0; i < s->n; ++i) {
    contrib[i] = robust[i] = touched[i] = 0;
    const Proj& g = pr[i];
    if (!g.visible) continue;
    for (int ty = g.py0 / tile; ty <= g.py1 / tile; ++ty)
      for (int tx = g.px0 / tile; tx <= g.px1 / tile; ++tx)
        if (tile_meets(g, tx, ty, tile, W, H, 0.0))
          bins[static_cast<size_t>(ty) * ntx + tx].push_back(static_cast<int32_t>(i));
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < static_cast<int64_t>(bins.size()); ++b) {
    std::vector<int32_t>& lst = bins[b];
    std::sort(lst.begin(), lst.end(), [&](int32_t a, int32_t c) { return z_index_less(pr, a, c); });
    const int tx = static_cast<int>(b % ntx), ty = static_cast<int>(b / ntx);
    std::vector<double> f(D > 0 ? D : 1);
    std::vector<int32_t> blended(lst.size() + 1);
    for (int py = ty * tile; py < std::min(H, (ty + 1) * tile); ++py)
      for (int px = tx * tile; px < std::min(W, (tx + 1) * tile); ++px) {
        PixelOut po;
        bool ovf = false;
        int64_t walked = 0;
        walk_pixel(*s, *cam, pr, lst.data(), static_cast<int64_t>(lst.size()), px, py, po, f.data(), blended.data(),
                   static_cast<int32_t>(blended.size()), &ovf, &walked);
        for (int32_t k = 0; k < po.nblend; ++k) {
          const int32_t gi = blended[k];
#pragma omp atomic write
          contrib[gi] = 1;
          if (!po.fragile) {
#pragma omp atomic write
            robust[gi] = 1;
          }
        }
        if (po.fragile)
          for (int64_t j = 0; j < walked; ++j) {
#pragma omp atomic write
            touched[lst[j]] = 1;
          }
      }
  }
  return 0;
}

// Smallest conic distance over rectangles (tests): rows of 10 doubles
// [a, b, c, u, v, x0, x1, y0, y1, unused] -> out[i].
int orc_min_q_box(const double* rows, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    const double* r = rows + 10 * i;
    out[i] = min_q_box(r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], r[8]);
  }
  return 0;
}

// Real SH basis values at unit directions (tests): dirs n x 3, out n x (deg+1)^2.
int orc_sh_basis(int32_t degree, const double* dirs, int64_t n, double* out) {
  const int K = (degree + 1) * (degree + 1);
  for (int64_t i = 0; i < n; ++i)
    for (int l = 0; l <= degree; ++l)
      for (int m = -l; m <= l; ++m) out[i * K + l * l + l + m] = real_sh(l, m, dirs + 3 * i);
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
