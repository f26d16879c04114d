// Reference renderer for the hybrid 2D/3D Gaussian rasterizer: TEST
// INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
// CPU-baseline leg may load this library.  It shares no code with the GPU
// library, and neither one includes or links the other.
//
// What it computes (EGGS, "Exchangeable 2D/3D Gaussian Splatting"):
//   * Sec. 3.1 "Hybrid Gaussian Rasterization": each primitive has a centre,
//     scales, a quaternion, an opacity, SH colour coefficients and a type flag
//     t (0 = 2D surfel, 1 = 3D Gaussian).
//   * Eq. 1 (unified distance).  For t = 0 it is u^2 + v^2 at the ray-splat
//     intersection (appendix "Differentiable Rasterization for 2D/3D Gaussian
//     Splatting", Eq. uv).  For t = 1 it is the Mahalanobis distance to the
//     affine (EWA) projection Sigma' = J W Sigma W^T J^T (same appendix).
//   * Per-pair contribution alpha_i * exp(-d_i / 2), composited front to back
//     in one pass (Eq. 2).
//   * Scale modulation of 2D opacities, alpha* = alpha exp(-lambda_z s_z*),
//     with s_z* = sigmoid((s_z - theta_z) / T_z) s_z (Sec. 3.2, Eq. 6-7).
//
// Where the paper is silent, the readings are fixed here and listed in the
// design notes of the repository: pixel sample point (x + 1/2, y + 1/2);
// OpenCV camera axes; skip a pair whose contribution is below 1/255; clamp
// the contribution at 0.99; stop a pixel when the transmittance would fall
// below 1e-4 (that pair is not blended); screen-space dilation delta added to
// Sigma' only for 3D Gaussians; depth = sum of weight x camera z (3D: centre
// z, 2D: z of the ray-plane hit); normal = sum of weight x camera-space
// normal (2D: third tangent axis, 3D: axis of the smallest scale), turned to
// face the camera; real SH with the Condon-Shortley phase; colour =
// max(0, 1/2 + sum f Y(dir)).
//
// Three parts:
//   1. A structural module in IEEE binary32 with a fixed operation order and
//      no fused multiply-add.  It decides culling, the conservative pixel
//      rectangle of the support, tiles, the depth sort key and the normal's
//      sign.  These are the discrete decisions that must match the GPU bit
//      for bit, so both sides take them in the same precision.
//   2. A binary64 forward that evaluates the plain per-pixel definition.  For
//      each pixel it gathers the splats whose rectangle holds the pixel, keeps
//      the active ones, orders them by (depth key, index) and composites them.
//      There is also a brute-force mode that tests every splat at every pixel.
//   3. A binary64 backward.  A division-free suffix recursion gives dL/d(alpha~),
//      dL/dc, dL/ddepth and dL/dnormal for each blended pair.  Forward-mode dual
//      numbers then carry these to the parameters (mu, s, q, alpha) through the
//      per-pair definitions.  SH coefficients enter linearly.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared (no -march flag,
// so no FMA is ever formed in the structural module).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Method constants (thresholds taken from the prior-art rasterizer that the
// paper builds on, Sec. 4 "Implementation").
// ---------------------------------------------------------------------------
// Defaults of the three thresholds; every call takes them as options.
constexpr double kAlphaMin = 1.0 / 255.0;  // skip a pair below this contribution
constexpr double kAlphaMax = 0.99;         // clamp a contribution at this value
constexpr double kTMin = 1e-4;             // stop before T falls below this

struct Scene32 {
  const float *means, *scales, *rots, *opac, *sh;
  const uint8_t *types;
  int64_t n;
  int sh_degree;
};

struct Scene64 {
  const double *means, *scales, *rots, *opac, *sh;
};

// Camera as passed in: viewmat[16] row-major world->camera, fx, fy, cx, cy,
// width, height, znear  (packed as 23 floats: 16 + 4 + W + H + znear).
struct Cam {
  float V[16];
  float fx, fy, cx, cy;
  int W, H;
  float znear;
};

Cam load_cam(const float *c) {
  Cam k;
  for (int i = 0; i < 16; ++i) k.V[i] = c[i];
  k.fx = c[16]; k.fy = c[17]; k.cx = c[18]; k.cy = c[19];
  k.W = (int)c[20]; k.H = (int)c[21]; k.znear = c[22];
  return k;
}

struct Opts {
  double bg[3];
  float dilation;
  double lambda_z, theta_z, temp_z;
  double pix_off[2];  // offset of every pixel sample (0 for rendering; finite-difference pins)
  double amin, amax, tmin;  // skip, clamp and stop thresholds
};

Opts load_opts(const double *o) {
  Opts p;
  p.bg[0] = o[0]; p.bg[1] = o[1]; p.bg[2] = o[2];
  p.dilation = (float)o[3];
  p.lambda_z = o[4]; p.theta_z = o[5]; p.temp_z = o[6];
  p.pix_off[0] = o[7]; p.pix_off[1] = o[8];
  p.amin = o[9]; p.amax = o[10]; p.tmin = o[11];
  return p;
}

// ===========================================================================
// 1. Structural module (binary32, fixed order, no FMA).
// ===========================================================================
struct Struct {
  uint8_t valid;
  int32_t px0, py0, px1, py1;  // inclusive pixel rectangle
  uint32_t tiles;              // tiles touched
  uint32_t zbits;              // depth key: bit pattern of camera z
  uint8_t flip;                // 1 if the normal is negated to face the camera
};

constexpr float kPad = 1.00390625f;  // 1 + 2^-8

// Inputs of the structural decisions besides the scene and camera.
struct StructCfg {
  float delta;  // screen-space dilation of 3D splats
  float amin;   // skip threshold, binary32
  float rr0;    // smallest binary32 >= 2 ln(1 / amin): radius^2 of the alpha = 1 support
};

StructCfg struct_cfg(float delta, double amin) {
  StructCfg c;
  c.delta = delta;
  c.amin = (float)amin;
  const double r = 2.0 * std::log(1.0 / (double)c.amin);
  float f = (float)r;
  if ((double)f < r) f = std::nextafter(f, INFINITY);
  c.rr0 = f;
  return c;
}

Struct structural(const Scene32 &s, int64_t g, const Cam &c, const StructCfg &cfg) {
  Struct o{};
  o.valid = 0;
  const float *V = c.V;
  const float mx = s.means[3 * g], my = s.means[3 * g + 1], mz = s.means[3 * g + 2];
  const float sx = s.scales[3 * g], sy = s.scales[3 * g + 1], sz = s.scales[3 * g + 2];
  const float rw = s.rots[4 * g], rx = s.rots[4 * g + 1], ry = s.rots[4 * g + 2],
              rz = s.rots[4 * g + 3];
  const float al = s.opac[g];
  const bool is2d = s.types[g] == 0;

  // Camera-space centre.
  const float xc = ((V[0] * mx + V[1] * my) + V[2] * mz) + V[3];
  const float yc = ((V[4] * mx + V[5] * my) + V[6] * mz) + V[7];
  const float zc = ((V[8] * mx + V[9] * my) + V[10] * mz) + V[11];
  if (!(zc > c.znear)) return o;
  if (!(al >= cfg.amin)) return o;

  // Rotation from the (not necessarily unit) quaternion (w, x, y, z).
  const float n2 = ((rw * rw + rx * rx) + ry * ry) + rz * rz;
  if (!(n2 > 0.0f)) return o;
  const float k2 = 2.0f / n2;
  float R[3][3];
  R[0][0] = 1.0f - k2 * (ry * ry + rz * rz);
  R[0][1] = k2 * (rx * ry - rw * rz);
  R[0][2] = k2 * (rx * rz + rw * ry);
  R[1][0] = k2 * (rx * ry + rw * rz);
  R[1][1] = 1.0f - k2 * (rx * rx + rz * rz);
  R[1][2] = k2 * (ry * rz - rw * rx);
  R[2][0] = k2 * (rx * rz - rw * ry);
  R[2][1] = k2 * (ry * rz + rw * rx);
  R[2][2] = 1.0f - k2 * (rx * rx + ry * ry);

  // Support radius^2 from the unmodulated opacity (a Pade bound on
  // 2 ln(alpha / amin), never below it for alpha <= 1).
  const float rr = cfg.rr0 + 4.0f * ((al - 1.0f) / (al + 1.0f));

  const float sc[3] = {sx, sy, sz};
  // Camera-space scaled axes: C[i][j] = (R_v (R e_j s_j))_i.
  float C[3][3];
  for (int j = 0; j < 3; ++j) {
    const float w0 = R[0][j] * sc[j], w1 = R[1][j] * sc[j], w2 = R[2][j] * sc[j];
    for (int i = 0; i < 3; ++i)
      C[i][j] = (V[4 * i] * w0 + V[4 * i + 1] * w1) + V[4 * i + 2] * w2;
  }

  const float Wm1 = (float)(c.W - 1), Hm1 = (float)(c.H - 1);
  float xlo, xhi, ylo, yhi;
  int k;  // axis that carries the normal
  if (!is2d) {
    const float iz = 1.0f / zc;
    const float u = xc * iz, v = yc * iz;
    const float a0 = c.fx * iz, a1 = c.fy * iz;
    float A0[3], A1[3];
    for (int j = 0; j < 3; ++j) {
      A0[j] = a0 * (C[0][j] - u * C[2][j]);
      A1[j] = a1 * (C[1][j] - v * C[2][j]);
    }
    const float S00 = ((A0[0] * A0[0] + A0[1] * A0[1]) + A0[2] * A0[2]) + cfg.delta;
    const float S01 = (A0[0] * A1[0] + A0[1] * A1[1]) + A0[2] * A1[2];
    const float S11 = ((A1[0] * A1[0] + A1[1] * A1[1]) + A1[2] * A1[2]) + cfg.delta;
    const float det = S00 * S11 - S01 * S01;
    if (!(det > 0.0f)) return o;
    const float mu_x = c.fx * u + c.cx, mu_y = c.fy * v + c.cy;
    const float hx = sqrtf(rr * S00) * kPad, hy = sqrtf(rr * S11) * kPad;
    xlo = (mu_x - hx) - 0.5f; xhi = (mu_x + hx) - 0.5f;
    ylo = (mu_y - hy) - 0.5f; yhi = (mu_y + hy) - 0.5f;
    k = (sz <= sx && sz <= sy) ? 2 : (sy <= sx ? 1 : 0);
  } else {
    if (!(sx > 0.0f) || !(sy > 0.0f)) return o;
    // The whole support disc must lie in front of z_near.
    const float q = C[2][0] * C[2][0] + C[2][1] * C[2][1];
    const float e = sqrtf(rr * q);
    if (!(zc - e > c.znear)) return o;
    // Dual conic of the support disc in camera coordinates,
    // E = C diag(rr, rr, -1) C^T with C = [C_0 | C_1 | p_c]; its minors give
    // the screen-space bounding box without cancellation.
    const float E22 = rr * q - zc * zc;
    if (!(E22 < 0.0f)) return o;
    const float pc[3] = {xc, yc, zc};
    float lo[2], hi[2];
    const float f[2] = {c.fx, c.fy}, cc[2] = {c.cx, c.cy};
    for (int a = 0; a < 2; ++a) {
      const float Ea2 = rr * (C[a][0] * C[2][0] + C[a][1] * C[2][1]) - pc[a] * zc;
      const float n01 = C[a][0] * C[2][1] - C[a][1] * C[2][0];
      const float n02 = C[a][0] * zc - pc[a] * C[2][0];
      const float n12 = C[a][1] * zc - pc[a] * C[2][1];
      float disc = rr * (n02 * n02 + n12 * n12) - (rr * rr) * (n01 * n01);
      if (!(disc >= 0.0f)) disc = 0.0f;
      const float cen = cc[a] + f[a] * (Ea2 / E22);
      const float h = (f[a] * (sqrtf(disc) / (-E22))) * kPad;
      lo[a] = (cen - h) - 0.5f;
      hi[a] = (cen + h) - 0.5f;
    }
    xlo = lo[0]; xhi = hi[0]; ylo = lo[1]; yhi = hi[1];
    k = 2;
  }
  if (!(xhi >= 0.0f) || !(xlo <= Wm1) || !(yhi >= 0.0f) || !(ylo <= Hm1)) return o;
  const int px0 = (xlo <= 0.0f) ? 0 : (int)ceilf(xlo);
  const int px1 = (xhi >= Wm1) ? c.W - 1 : (int)floorf(xhi);
  const int py0 = (ylo <= 0.0f) ? 0 : (int)ceilf(ylo);
  const int py1 = (yhi >= Hm1) ? c.H - 1 : (int)floorf(yhi);
  if (px0 > px1 || py0 > py1) return o;

  // Normal orientation: camera-space axis k of R_v R, negated when it points
  // away from the camera (n . p_c > 0).
  const float nc0 = (V[0] * R[0][k] + V[1] * R[1][k]) + V[2] * R[2][k];
  const float nc1 = (V[4] * R[0][k] + V[5] * R[1][k]) + V[6] * R[2][k];
  const float nc2 = (V[8] * R[0][k] + V[9] * R[1][k]) + V[10] * R[2][k];
  const float dot = (nc0 * xc + nc1 * yc) + nc2 * zc;

  o.valid = 1;
  o.px0 = px0; o.px1 = px1; o.py0 = py0; o.py1 = py1;
  o.tiles = (uint32_t)(((px1 >> 4) - (px0 >> 4) + 1) * ((py1 >> 4) - (py0 >> 4) + 1));
  std::memcpy(&o.zbits, &zc, 4);
  o.flip = dot > 0.0f ? 1 : 0;
  return o;
}

// ===========================================================================
// Forward-mode dual numbers over the 11 per-splat parameters
// (mu 0..2, s 3..5, q 6..9, alpha 10).
// ===========================================================================
constexpr int NP = 11;

struct Dual {
  double v;
  double d[NP];
  Dual() : v(0) { for (int i = 0; i < NP; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < NP; ++i) d[i] = 0; }
  static Dual var(double x, int i) { Dual r(x); r.d[i] = 1.0; return r; }
};
inline Dual operator+(const Dual &a, const Dual &b) { Dual r(a.v + b.v); for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual &a, const Dual &b) { Dual r(a.v - b.v); for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual &a) { Dual r(-a.v); for (int i = 0; i < NP; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual &a, const Dual &b) { Dual r(a.v * b.v); for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual &a, const Dual &b) {
  Dual r(a.v / b.v);
  for (int i = 0; i < NP; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual &a, double b) { Dual r = a; r.v += b; return r; }
inline Dual operator+(double b, const Dual &a) { return a + b; }
inline Dual operator-(const Dual &a, double b) { Dual r = a; r.v -= b; return r; }
inline Dual operator-(double b, const Dual &a) { return (-a) + b; }
inline Dual operator*(const Dual &a, double b) { Dual r(a.v * b); for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] * b; return r; }
inline Dual operator*(double b, const Dual &a) { return a * b; }
inline Dual operator/(const Dual &a, double b) { return a * (1.0 / b); }
inline Dual dsqrt(const Dual &a) { double s = std::sqrt(a.v); Dual r(s); for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] / (2.0 * s); return r; }
inline Dual dexp(const Dual &a) { double e = std::exp(a.v); Dual r(e); for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] * e; return r; }
inline double sigmoid_v(double z) {
  return z >= 0 ? 1.0 / (1.0 + std::exp(-z)) : std::exp(z) / (1.0 + std::exp(z));
}
inline double dsigmoid(double z) { return sigmoid_v(z); }
inline Dual dsigmoid(const Dual &z) {
  const double s = sigmoid_v(z.v);
  Dual r(s);
  for (int i = 0; i < NP; ++i) r.d[i] = z.d[i] * s * (1.0 - s);
  return r;
}
inline double val(const Dual &a) { return a.v; }
inline double val(double a) { return a; }
inline double dsqrt(double a) { return std::sqrt(a); }
inline double dexp(double a) { return std::exp(a); }

// ===========================================================================
// Real spherical harmonics, built from the textbook definition:
//   Y_l^0 = K_l^0 P_l(z),
//   Y_l^m = sqrt2 K_l^m P_l^m(z) cos(m phi)   (m > 0),
//   Y_l^-m = sqrt2 K_l^m P_l^m(z) sin(m phi)  (m > 0),
// with P_l^m = (-1)^m (1 - z^2)^{m/2} d^m/dz^m P_l (Condon-Shortley phase)
// and K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  On the unit sphere
// (1 - z^2)^{m/2} cos(m phi) = Re (x + i y)^m and likewise Im for sin, so
// every Y is a polynomial in the direction and dual numbers pass through it.
// Coefficient j = l^2 + l + m.
// ===========================================================================
struct Legendre {
  // coef[l][m][p] : coefficient of z^p in d^m/dz^m P_l(z)
  double coef[4][4][4];
  double K[4][4];
  Legendre() {
    double P[4][4] = {{0}};
    P[0][0] = 1.0;          // P_0 = 1
    P[1][1] = 1.0;          // P_1 = z
    for (int l = 1; l < 3; ++l)  // Bonnet: (l+1) P_{l+1} = (2l+1) z P_l - l P_{l-1}
      for (int p = 0; p < 4; ++p)
        P[l + 1][p] = ((2 * l + 1) * (p > 0 ? P[l][p - 1] : 0.0) - l * P[l - 1][p]) / (l + 1);
    for (int l = 0; l < 4; ++l) {
      double cur[4];
      for (int p = 0; p < 4; ++p) cur[p] = P[l][p];
      for (int m = 0; m < 4; ++m) {
        for (int p = 0; p < 4; ++p) coef[l][m][p] = cur[p];
        double nxt[4] = {0, 0, 0, 0};
        for (int p = 1; p < 4; ++p) nxt[p - 1] = p * cur[p];
        for (int p = 0; p < 4; ++p) cur[p] = nxt[p];
      }
      for (int m = 0; m <= l; ++m) {
        double r = 1.0;
        for (int t = l - m + 1; t <= l + m; ++t) r /= t;  // (l-m)!/(l+m)!
        K[l][m] = std::sqrt((2 * l + 1) / (4.0 * M_PI) * r);
      }
    }
  }
};
const Legendre &legendre() { static Legendre L; return L; }

template <class S>
void sh_basis(int degree, const S dir[3], S *Y) {
  const Legendre &L = legendre();
  const S &x = dir[0], &y = dir[1], &z = dir[2];
  // (x + i y)^m
  S re[4], im[4];
  re[0] = S(1.0); im[0] = S(0.0);
  for (int m = 1; m < 4; ++m) {
    re[m] = re[m - 1] * x - im[m - 1] * y;
    im[m] = re[m - 1] * y + im[m - 1] * x;
  }
  for (int l = 0; l <= degree; ++l) {
    for (int m = 0; m <= l; ++m) {
      S poly(0.0), zp(1.0);
      for (int p = 0; p + m <= l; ++p) { poly = poly + L.coef[l][m][p] * zp; zp = zp * z; }
      const double sign = (m % 2) ? -1.0 : 1.0;
      if (m == 0) {
        Y[l * l + l] = L.K[l][0] * poly;
      } else {
        const double k = std::sqrt(2.0) * L.K[l][m] * sign;
        Y[l * l + l + m] = k * (poly * re[m]);
        Y[l * l + l - m] = k * (poly * im[m]);
      }
    }
  }
}

// ===========================================================================
// 2. Per-splat and per-pair definitions (templated on double / Dual).
// ===========================================================================
template <class S>
struct Splat {
  bool is2d;
  S alpha_eff;
  S pc[3];          // camera-space centre
  S nrm[3];         // camera-space normal, oriented by the structural sign
  S color[3];
  bool clamped[3];  // colour channel clamped at 0
  double Y[16];
  S Yd[16];
  // 3D
  S mu2[2], conic[3];  // conic = Sigma'^{-1} = [[c0 c1][c1 c2]]
  // 2D (camera frame)
  S tu[3], tv[3], sx, sy;
};

struct CamD {
  double R[3][3], t[3], o[3];  // world->camera rotation, translation, camera centre
  double fx, fy, cx, cy;
};

CamD cam_d(const Cam &c) {
  CamD k;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) k.R[i][j] = c.V[4 * i + j];
    k.t[i] = c.V[4 * i + 3];
  }
  // camera centre: the world point that maps to the camera origin, -R^{-1} t
  const double(*R)[3] = k.R;
  const double det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) -
                     R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
                     R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
  double Ri[3][3];
  Ri[0][0] = (R[1][1] * R[2][2] - R[1][2] * R[2][1]) / det;
  Ri[0][1] = (R[0][2] * R[2][1] - R[0][1] * R[2][2]) / det;
  Ri[0][2] = (R[0][1] * R[1][2] - R[0][2] * R[1][1]) / det;
  Ri[1][0] = (R[1][2] * R[2][0] - R[1][0] * R[2][2]) / det;
  Ri[1][1] = (R[0][0] * R[2][2] - R[0][2] * R[2][0]) / det;
  Ri[1][2] = (R[0][2] * R[1][0] - R[0][0] * R[1][2]) / det;
  Ri[2][0] = (R[1][0] * R[2][1] - R[1][1] * R[2][0]) / det;
  Ri[2][1] = (R[0][1] * R[2][0] - R[0][0] * R[2][1]) / det;
  Ri[2][2] = (R[0][0] * R[1][1] - R[0][1] * R[1][0]) / det;
  for (int i = 0; i < 3; ++i) k.o[i] = -(Ri[i][0] * k.t[0] + Ri[i][1] * k.t[1] + Ri[i][2] * k.t[2]);
  k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy;
  return k;
}

template <class S>
S param(const Scene64 &p, int64_t g, int idx);

template <>
double param<double>(const Scene64 &p, int64_t g, int idx) {
  if (idx < 3) return p.means[3 * g + idx];
  if (idx < 6) return p.scales[3 * g + idx - 3];
  if (idx < 10) return p.rots[4 * g + idx - 6];
  return p.opac[g];
}
template <>
Dual param<Dual>(const Scene64 &p, int64_t g, int idx) {
  return Dual::var(param<double>(p, g, idx), idx);
}

// Sec. 3.1: Sigma = R S S^T R^T with R from the normalised quaternion; the
// appendix on rasterization: Sigma' = J W Sigma W^T J^T, J the Jacobian of
// the pinhole map at the centre.  Sec. 3.2, Eq. 6-7 for the 2D opacity.
template <class S>
void setup_splat(const Scene32 &s32, const Scene64 &p, int64_t g, const CamD &c,
                 const Opts &opt, const Struct &st, Splat<S> &o) {
  S mu[3], sc[3], q[4];
  for (int i = 0; i < 3; ++i) mu[i] = param<S>(p, g, i);
  for (int i = 0; i < 3; ++i) sc[i] = param<S>(p, g, 3 + i);
  for (int i = 0; i < 4; ++i) q[i] = param<S>(p, g, 6 + i);
  S al = param<S>(p, g, 10);
  o.is2d = s32.types[g] == 0;

  // unit quaternion -> rotation matrix
  S qn = dsqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  S w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  S R[3][3];
  R[0][0] = 1.0 - 2.0 * (y * y + z * z); R[0][1] = 2.0 * (x * y - w * z); R[0][2] = 2.0 * (x * z + w * y);
  R[1][0] = 2.0 * (x * y + w * z); R[1][1] = 1.0 - 2.0 * (x * x + z * z); R[1][2] = 2.0 * (y * z - w * x);
  R[2][0] = 2.0 * (x * z - w * y); R[2][1] = 2.0 * (y * z + w * x); R[2][2] = 1.0 - 2.0 * (x * x + y * y);

  // world -> camera
  for (int i = 0; i < 3; ++i)
    o.pc[i] = c.R[i][0] * mu[0] + c.R[i][1] * mu[1] + c.R[i][2] * mu[2] + c.t[i];
  S RvR[3][3];  // R_v R
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      RvR[i][j] = c.R[i][0] * R[0][j] + c.R[i][1] * R[1][j] + c.R[i][2] * R[2][j];

  // opacity (2D: scale modulation)
  if (o.is2d) {
    S zt = (sc[2] - opt.theta_z) / opt.temp_z;
    S sig = dsigmoid(zt);
    S szs = sig * sc[2];
    o.alpha_eff = al * dexp(-opt.lambda_z * szs);
  } else {
    o.alpha_eff = al;
  }

  // normal: axis of the smallest scale for 3D (z axis on ties, then y),
  // the third tangent axis for 2D; sign fixed by the structural decision
  int k = 2;
  if (!o.is2d) {
    const float fsx = s32.scales[3 * g], fsy = s32.scales[3 * g + 1], fsz = s32.scales[3 * g + 2];
    k = (fsz <= fsx && fsz <= fsy) ? 2 : (fsy <= fsx ? 1 : 0);
  }
  const double sgn = st.flip ? -1.0 : 1.0;
  for (int i = 0; i < 3; ++i) o.nrm[i] = sgn * RvR[i][k];

  // colour: direction from the camera centre to the mean (world frame)
  S dv[3];
  for (int i = 0; i < 3; ++i) dv[i] = mu[i] - c.o[i];
  S dn = dsqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  S dir[3] = {dv[0] / dn, dv[1] / dn, dv[2] / dn};
  const int K = (s32.sh_degree + 1) * (s32.sh_degree + 1);
  sh_basis<S>(s32.sh_degree, dir, o.Yd);
  for (int j = 0; j < K; ++j) o.Y[j] = val(o.Yd[j]);
  for (int ch = 0; ch < 3; ++ch) {
    S acc(0.5);
    for (int j = 0; j < K; ++j) acc = acc + p.sh[(g * K + j) * 3 + ch] * o.Yd[j];
    o.clamped[ch] = !(val(acc) > 0.0);
    o.color[ch] = o.clamped[ch] ? S(0.0) : acc;
  }

  if (!o.is2d) {
    // Sigma = R diag(s^2) R^T, camera covariance, EWA projection
    S Sig[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        Sig[i][j] = R[i][0] * sc[0] * sc[0] * R[j][0] + R[i][1] * sc[1] * sc[1] * R[j][1] +
                    R[i][2] * sc[2] * sc[2] * R[j][2];
    S Sc[3][3], tmp[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        tmp[i][j] = c.R[i][0] * Sig[0][j] + c.R[i][1] * Sig[1][j] + c.R[i][2] * Sig[2][j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        Sc[i][j] = tmp[i][0] * c.R[j][0] + tmp[i][1] * c.R[j][1] + tmp[i][2] * c.R[j][2];
    const S &X = o.pc[0], &Yv = o.pc[1], &Z = o.pc[2];
    S J[2][3];
    J[0][0] = c.fx / Z; J[0][1] = S(0.0); J[0][2] = -c.fx * X / (Z * Z);
    J[1][0] = S(0.0); J[1][1] = c.fy / Z; J[1][2] = -c.fy * Yv / (Z * Z);
    S JS[2][3];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j)
        JS[i][j] = J[i][0] * Sc[0][j] + J[i][1] * Sc[1][j] + J[i][2] * Sc[2][j];
    S P00 = JS[0][0] * J[0][0] + JS[0][1] * J[0][1] + JS[0][2] * J[0][2] + (double)opt.dilation;
    S P01 = JS[0][0] * J[1][0] + JS[0][1] * J[1][1] + JS[0][2] * J[1][2];
    S P11 = JS[1][0] * J[1][0] + JS[1][1] * J[1][1] + JS[1][2] * J[1][2] + (double)opt.dilation;
    S det = P00 * P11 - P01 * P01;
    o.conic[0] = P11 / det;
    o.conic[1] = -P01 / det;
    o.conic[2] = P00 / det;
    o.mu2[0] = c.fx * X / Z + c.cx;
    o.mu2[1] = c.fy * Yv / Z + c.cy;
  } else {
    for (int i = 0; i < 3; ++i) {
      o.tu[i] = RvR[i][0];
      o.tv[i] = RvR[i][1];
    }
    o.sx = sc[0];
    o.sy = sc[1];
  }
}

// Intersection of the pixel ray kappa * omega (camera frame, omega =
// K^{-1} (px, py, 1)) with the surfel plane written in the surfel's own
// parameters, p_c + u s_x t_u + v s_y t_v: a 3x3 linear system in
// (u, v, kappa), solved by Cramer's rule.  This is the same point the paper's
// homogeneous form (Eq. uv) describes.
template <class S>
void surfel_hit(const Splat<S> &sp, const double om[3], S &u, S &v, S &kap) {
  S a[3], b[3], mo[3], rhs[3];
  for (int i = 0; i < 3; ++i) {
    a[i] = sp.sx * sp.tu[i];
    b[i] = sp.sy * sp.tv[i];
    mo[i] = S(-om[i]);
    rhs[i] = -sp.pc[i];
  }
  auto det3 = [](const S *c0, const S *c1, const S *c2) {
    return c0[0] * (c1[1] * c2[2] - c1[2] * c2[1]) - c0[1] * (c1[0] * c2[2] - c1[2] * c2[0]) +
           c0[2] * (c1[0] * c2[1] - c1[1] * c2[0]);
  };
  const S D = det3(a, b, mo);
  u = det3(rhs, b, mo) / D;
  v = det3(a, rhs, mo) / D;
  kap = det3(a, b, rhs) / D;
}

// Eq. 1 at pixel sample (px, py); also the pair's depth.
template <class S>
void eval_pair(const Splat<S> &sp, const CamD &c, double px, double py, S &d, S &depth) {
  if (!sp.is2d) {
    S dx = px - sp.mu2[0], dy = py - sp.mu2[1];
    d = sp.conic[0] * dx * dx + 2.0 * sp.conic[1] * dx * dy + sp.conic[2] * dy * dy;
    depth = sp.pc[2];
  } else {
    const double om[3] = {(px - c.cx) / c.fx, (py - c.cy) / c.fy, 1.0};
    S u, v, kap;
    surfel_hit(sp, om, u, v, kap);
    d = u * u + v * v;
    depth = kap;  // camera z of the hit point (omega_z = 1)
  }
}

// A decision taken within rounding of its threshold ("tie") may go either way
// in a binary32 evaluation, and both outcomes are correct results of the
// method.  The margins say how close counts as a tie.
struct Margins {
  double alpha_rel;  // activity tie if |raw - amin| <= alpha_rel * amin
  double t_rel;      // stop tie if |T' - tmin| <= t_rel * tmin
  double clamp_rel;  // clamp tie (gradient only) if |raw - amax| <= clamp_rel * amax
};

// Per-view binning of splats by tile (candidate lookup only; the order of
// blending is decided per pixel below).
struct Bins {
  int tiles_x, tiles_y;
  std::vector<std::vector<int64_t>> list;        // unsorted, index order
  std::vector<std::vector<uint64_t>> sorted_keys;  // (zbits << 32 | local idx) sorted
};

struct Work {
  const Scene32 *s32;
  const Scene64 *s64;
  std::vector<Cam> cams;
  std::vector<CamD> camd;
  Opts opt;
  std::vector<Struct> st;  // [V*N]
  std::vector<Bins> bins;  // [V]
  bool brute;
};

void build(Work &w, const float *cams, int V, bool brute) {
  const int64_t N = w.s32->n;
  w.cams.resize(V);
  w.camd.resize(V);
  w.st.resize((size_t)V * N);
  w.bins.resize(V);
  w.brute = brute;
  for (int v = 0; v < V; ++v) {
    w.cams[v] = load_cam(cams + 23 * v);
    w.camd[v] = cam_d(w.cams[v]);
    const StructCfg cfg = struct_cfg(w.opt.dilation, w.opt.amin);
    for (int64_t g = 0; g < N; ++g) w.st[(size_t)v * N + g] = structural(*w.s32, g, w.cams[v], cfg);
    Bins &b = w.bins[v];
    b.tiles_x = (w.cams[v].W + 15) / 16;
    b.tiles_y = (w.cams[v].H + 15) / 16;
    b.list.assign((size_t)b.tiles_x * b.tiles_y, {});
    for (int64_t g = 0; g < N; ++g) {
      const Struct &s = w.st[(size_t)v * N + g];
      if (!s.valid) continue;
      for (int ty = s.py0 >> 4; ty <= (s.py1 >> 4); ++ty)
        for (int tx = s.px0 >> 4; tx <= (s.px1 >> 4); ++tx)
          b.list[(size_t)ty * b.tiles_x + tx].push_back(g);
    }
    b.sorted_keys.resize(b.list.size());
    for (size_t t = 0; t < b.list.size(); ++t) {
      auto &sk = b.sorted_keys[t];
      sk.clear();
      for (int64_t g : b.list[t]) sk.push_back(((uint64_t)w.st[(size_t)v * N + g].zbits << 32) | (uint64_t)g);
      std::sort(sk.begin(), sk.end());
    }
  }
}

template <class F>
void parallel_for(int64_t n, int threads, F f) {
  if (threads <= 1 || n < 64) {
    f(0, 0, n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    const int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=, &f] { f(t, a, b); });
  }
  for (auto &x : th) x.join();
}

struct PairRec {
  uint32_t zbits;
  int64_t g;
  double raw;    // alpha_eff exp(-d/2) before the clamp
  double alpha;  // clamped contribution
  bool clamped;
};

struct PixelOut {
  double rgb[3], depth, nrm[3], T;
  int n_contrib, last;
  uint8_t tie;
  int nflags;  // activity and stop ties met along the way
  int64_t wcount[2];
};

// Per-splat binary64 set-up, memoised per (view, splat) when the scene is
// small enough; otherwise recomputed for each candidate.  Same arithmetic
// either way.
struct SplatCache {
  std::vector<Splat<double>> sp;
  std::vector<uint8_t> have;
};

void build_cache(const Work &w, SplatCache &c, int threads) {
  const int64_t N = w.s32->n, V = (int64_t)w.cams.size();
  if (V * N > 4000000) return;
  c.sp.resize((size_t)(V * N));
  c.have.assign((size_t)(V * N), 0);
  parallel_for(V * N, threads, [&](int, int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      const int v = (int)(i / N);
      const int64_t g = i % N;
      if (!w.st[(size_t)i].valid) continue;
      setup_splat<double>(*w.s32, *w.s64, g, w.camd[v], w.opt, w.st[(size_t)i], c.sp[(size_t)i]);
      c.have[(size_t)i] = 1;
    }
  });
}

const Splat<double> &get_splat(const Work &w, const SplatCache &c, int v, int64_t g,
                               Splat<double> &tmp) {
  const size_t i = (size_t)v * w.s32->n + g;
  if (!c.have.empty() && c.have[i]) return c.sp[i];
  setup_splat<double>(*w.s32, *w.s64, g, w.camd[v], w.opt, w.st[i], tmp);
  return tmp;
}

// One pixel (Eq. 2): gather the candidates, order them by (depth key, index),
// skip inactive pairs, composite front to back until the transmittance would
// fall below the floor.  The blended pairs are returned through `seq`.
// Activity and stop decisions that fall within the tie margins are numbered
// in the order they are met; bit k of `flip` takes the other outcome of tie
// k (a branch of the composite that a binary32 evaluation may legitimately
// follow).  flip = 0 is the binary64 decision everywhere.
void render_pixel(const Work &w, const SplatCache &cache, int v, int x, int y,
                  const Margins &mg, uint32_t flip, PixelOut &po, std::vector<PairRec> &seq) {
  const int64_t N = w.s32->n;
  const CamD &cd = w.camd[v];
  const double amin = w.opt.amin, amax = w.opt.amax, tmin = w.opt.tmin;
  const double px = x + 0.5 + w.opt.pix_off[0], py = y + 0.5 + w.opt.pix_off[1];
  std::vector<PairRec> cand;
  Splat<double> tmp;
  auto consider = [&](int64_t g) {
    const Struct &st = w.st[(size_t)v * N + g];
    if (!st.valid) return;
    if (!w.brute && (x < st.px0 || x > st.px1 || y < st.py0 || y > st.py1)) return;
    const Splat<double> &sp = get_splat(w, cache, v, g, tmp);
    double d, dep;
    eval_pair<double>(sp, cd, px, py, d, dep);
    const double raw = sp.alpha_eff * std::exp(-0.5 * d);
    cand.push_back(PairRec{st.zbits, g, raw, std::min(amax, raw), raw > amax});
  };
  if (w.brute) {
    for (int64_t g = 0; g < N; ++g) consider(g);
  } else {
    const Bins &b = w.bins[v];
    for (int64_t g : b.list[(size_t)(y >> 4) * b.tiles_x + (x >> 4)]) consider(g);
  }
  std::sort(cand.begin(), cand.end(), [](const PairRec &a, const PairRec &b) {
    return a.zbits != b.zbits ? a.zbits < b.zbits : a.g < b.g;
  });
  double T = 1.0;
  po.tie = 0;
  po.nflags = 0;
  po.rgb[0] = po.rgb[1] = po.rgb[2] = 0.0;
  po.depth = 0.0;
  po.nrm[0] = po.nrm[1] = po.nrm[2] = 0.0;
  po.n_contrib = 0;
  po.wcount[0] = po.wcount[1] = 0;
  int64_t last_g = -1;
  seq.clear();
  auto decide = [&](bool outcome, bool tie, uint8_t bit) {
    if (!tie) return outcome;
    po.tie |= bit;
    const bool flipped = po.nflags < 32 && ((flip >> po.nflags) & 1u);
    po.nflags += 1;
    return flipped ? !outcome : outcome;
  };
  for (const PairRec &pr : cand) {
    // active iff raw >= amin (false for NaN; std::min would hide it)
    const bool active = decide(pr.raw >= amin, std::fabs(pr.raw - amin) <= mg.alpha_rel * amin, 1);
    if (!active) continue;
    po.wcount[w.s32->types[pr.g] == 0 ? 0 : 1] += 1;
    const double Tn = T * (1.0 - pr.alpha);
    if (decide(Tn < tmin, std::fabs(Tn - tmin) <= mg.t_rel * tmin, 2)) break;
    if (std::fabs(pr.raw - amax) <= mg.clamp_rel * amax) po.tie |= 4;
    const Splat<double> &sp = get_splat(w, cache, v, pr.g, tmp);
    double d, dep;
    eval_pair<double>(sp, cd, px, py, d, dep);
    const double wgt = pr.alpha * T;
    for (int ch = 0; ch < 3; ++ch) po.rgb[ch] += wgt * sp.color[ch];
    po.depth += wgt * dep;
    for (int i = 0; i < 3; ++i) po.nrm[i] += wgt * sp.nrm[i];
    T = Tn;
    po.n_contrib += 1;
    last_g = pr.g;
    seq.push_back(pr);
  }
  for (int ch = 0; ch < 3; ++ch) po.rgb[ch] += T * w.opt.bg[ch];
  po.T = T;
  po.last = 0;
  if (last_g >= 0) {
    // 1 + position of the last blended splat in its tile's (key, index) order
    const Bins &b = w.bins[v];
    const auto &sk = b.sorted_keys[(size_t)(y >> 4) * b.tiles_x + (x >> 4)];
    const uint64_t key = ((uint64_t)w.st[(size_t)v * N + last_g].zbits << 32) | (uint64_t)last_g;
    po.last = (int)(std::lower_bound(sk.begin(), sk.end(), key) - sk.begin()) + 1;
  }
}

}  // namespace

// ===========================================================================
// C entry points (ctypes).
// ===========================================================================
extern "C" {

// Structural decisions for every (view, splat).
int oracle_structural(const float *means, const float *scales, const float *rots,
                      const float *opac, const uint8_t *types, int64_t n,
                      const float *cams, int V, float dilation, double alpha_min,
                      uint8_t *valid, int32_t *rect, uint32_t *tiles, uint32_t *zbits,
                      uint8_t *flip) {
  Scene32 s{means, scales, rots, opac, nullptr, types, n, 0};
  const StructCfg cfg = struct_cfg(dilation, alpha_min);
  for (int v = 0; v < V; ++v) {
    Cam c = load_cam(cams + 23 * v);
    for (int64_t g = 0; g < n; ++g) {
      Struct st = structural(s, g, c, cfg);
      const size_t i = (size_t)v * n + g;
      valid[i] = st.valid;
      rect[4 * i] = st.px0; rect[4 * i + 1] = st.py0; rect[4 * i + 2] = st.px1; rect[4 * i + 3] = st.py1;
      tiles[i] = st.valid ? st.tiles : 0;
      zbits[i] = st.valid ? st.zbits : 0;
      flip[i] = st.flip;
    }
  }
  return 0;
}

// Key/value list: every valid (view, splat) emits one pair per tile of its
// rectangle, in index order, key = (global tile << 32) | depth bits, value =
// view * n + splat; then a stable sort by key and the tile ranges.
int64_t oracle_sorted_pairs(const uint8_t *valid, const int32_t *rect, const uint32_t *zbits,
                            int64_t n, const int32_t *wh, int V, uint64_t *keys_out,
                            uint32_t *vals_out, int64_t cap, uint32_t *ranges, int64_t n_tiles_total) {
  std::vector<std::pair<uint64_t, uint32_t>> pairs;
  int64_t tile_base = 0;
  for (int v = 0; v < V; ++v) {
    const int tx = (wh[2 * v] + 15) / 16, ty = (wh[2 * v + 1] + 15) / 16;
    for (int64_t g = 0; g < n; ++g) {
      const size_t i = (size_t)v * n + g;
      if (!valid[i]) continue;
      for (int y = rect[4 * i + 1] >> 4; y <= (rect[4 * i + 3] >> 4); ++y)
        for (int x = rect[4 * i] >> 4; x <= (rect[4 * i + 2] >> 4); ++x) {
          const uint64_t tile = (uint64_t)(tile_base + (int64_t)y * tx + x);
          pairs.emplace_back((tile << 32) | zbits[i], (uint32_t)i);
        }
    }
    tile_base += (int64_t)tx * ty;
  }
  std::stable_sort(pairs.begin(), pairs.end(),
                   [](const auto &a, const auto &b) { return a.first < b.first; });
  const int64_t D = (int64_t)pairs.size();
  if (D > cap) return D;
  for (int64_t i = 0; i < D; ++i) { keys_out[i] = pairs[i].first; vals_out[i] = pairs[i].second; }
  for (int64_t t = 0; t < 2 * n_tiles_total; ++t) ranges[t] = 0;
  for (int64_t i = 0; i < D; ++i) {
    const int64_t t = (int64_t)(pairs[i].first >> 32);
    if (i == 0 || (int64_t)(pairs[i - 1].first >> 32) != t) ranges[2 * t] = (uint32_t)i;
    if (i == D - 1 || (int64_t)(pairs[i + 1].first >> 32) != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
  }
  return D;
}

// Forward at a list of pixels.  pix = [P,3] (view, y, x).  out8 = [P,8]
// (r, g, b, alpha, depth, nx, ny, nz); tfin = [P]; counts = [P,2]
// (n_contrib, last); tie = [P]; wcount = [2] summed over pixels.
// opts = [bg r, g, b, dilation, lambda_z, theta_z, temp_z, pixel offset x, y,
// alpha_min, alpha_max, t_min]; margins = [alpha_rel, t_rel, clamp_rel].
// flip = [P] tie branches (see render_pixel) or NULL; nflags = [P] number of
// activity / stop ties met, or NULL.
int oracle_forward(const float *m32, const float *s32, const float *r32, const float *o32,
                   const float *sh32, const uint8_t *types, int64_t n, int sh_degree,
                   const double *m64, const double *s64, const double *r64, const double *o64,
                   const double *sh64, const float *cams, int V, const double *opts,
                   const double *margins, const int32_t *pix, int64_t P, const uint32_t *flip,
                   int brute, int threads, double *out8, double *tfin, int32_t *counts,
                   uint8_t *tie, int32_t *nflags, int64_t *wcount) {
  Scene32 sc32{m32, s32, r32, o32, sh32, types, n, sh_degree};
  Scene64 sc64{m64, s64, r64, o64, sh64};
  Work w;
  w.s32 = &sc32;
  w.s64 = &sc64;
  w.opt = load_opts(opts);
  build(w, cams, V, brute != 0);
  const Margins mg{margins[0], margins[1], margins[2]};
  SplatCache cache;
  if (4 * P >= n) build_cache(w, cache, threads);
  std::vector<int64_t> wc(2 * std::max(1, threads), 0);
  parallel_for(P, threads, [&](int t, int64_t a, int64_t b) {
    std::vector<PairRec> seq;
    for (int64_t i = a; i < b; ++i) {
      PixelOut po;
      render_pixel(w, cache, pix[3 * i], pix[3 * i + 2], pix[3 * i + 1], mg, flip ? flip[i] : 0u,
                   po, seq);
      double *o = out8 + 8 * i;
      o[0] = po.rgb[0]; o[1] = po.rgb[1]; o[2] = po.rgb[2];
      o[3] = 1.0 - po.T;
      o[4] = po.depth;
      o[5] = po.nrm[0]; o[6] = po.nrm[1]; o[7] = po.nrm[2];
      tfin[i] = po.T;
      counts[2 * i] = po.n_contrib;
      counts[2 * i + 1] = po.last;
      tie[i] = po.tie;
      if (nflags) nflags[i] = po.nflags;
      wc[2 * t] += po.wcount[0];
      wc[2 * t + 1] += po.wcount[1];
    }
  });
  wcount[0] = wcount[1] = 0;
  for (size_t t = 0; t < wc.size() / 2; ++t) { wcount[0] += wc[2 * t]; wcount[1] += wc[2 * t + 1]; }
  return 0;
}

// Backward of L = sum over listed pixels of <G, out> (G = [P,8] in the
// order of out8), on the branch of each pixel selected by flip (NULL: the
// binary64 decisions; margins as in oracle_forward).  Outputs dL/d(params)
// in binary64, plus tolerance scales of the same shapes:
//   a_params, a_sh  sums of the absolute per-pair terms;
//   c_params        a bound on the rounding of a binary32 evaluation of the
//                   dL/dalpha~ path, in units of the binary32 unit roundoff
//                   (see below);
//   x_params        per element, the sum over clamp ties (pairs whose
//                   contribution is within the clamp margin of alpha_max)
//                   of |dL/dalpha~ d(alpha_eff e^{-d/2})/dtheta|: the
//                   difference between the clamped and the unclamped
//                   branch, either of which a binary32 evaluation may take.
//
// The rounding bound.  A binary32 reverse pass forms dL/dalpha~_i =
// T_i (f_i - S_i) from T_i recovered by dividing the final transmittance by
// (1 - alpha~_j) for j >= i, and from the suffix S accumulated over the
// pairs behind i.  Each of the m forward products, the m - i divisions and
// the m - i accumulation steps contributes a relative rounding of a few
// units of the largest magnitude it carries, and an error da_j in a
// contribution moves (1 - alpha~_j) by da_j / (1 - alpha~_j), with
// da_j / alpha~_j a few units times (1 + the exponent's magnitude).  So per
// pair
//   c_i = T_i (F_i + Shat_i) n_eff |d alpha~_i / d theta|_mag,
//   n_eff = m + 2 + sum over unclamped blended j of alpha~_j (1 + e_j) / (1 - alpha~_j),
// where F_i is the sum of |terms| of f_i, Shat_i the largest |S_j| and F_j
// behind i (the background term included), e_j the exponent's magnitude in
// log2 units, and |d alpha~/d theta|_mag the derivative of alpha~ with the
// exponent's terms taken by magnitude (3D: the entrywise conic and offset
// magnitudes; 2D: |d alpha~/d theta|).  A test multiplies c by a few units
// of binary32 roundoff.  The other per-pair terms are products, bounded
// relative to a_params.
int oracle_backward(const float *m32, const float *s32, const float *r32, const float *o32,
                    const float *sh32, const uint8_t *types, int64_t n, int sh_degree,
                    const double *m64, const double *s64, const double *r64, const double *o64,
                    const double *sh64, const float *cams, int V, const double *opts,
                    const double *margins, const int32_t *pix, int64_t P, const uint32_t *flip,
                    const double *G, int threads,
                    double *g_params /* [n,11] */, double *g_sh /* [n,K,3] */,
                    double *a_params, double *a_sh, double *c_params, double *x_params) {
  Scene32 sc32{m32, s32, r32, o32, sh32, types, n, sh_degree};
  Scene64 sc64{m64, s64, r64, o64, sh64};
  Work w;
  w.s32 = &sc32;
  w.s64 = &sc64;
  w.opt = load_opts(opts);
  build(w, cams, V, false);
  const Margins mg{margins[0], margins[1], margins[2]};
  SplatCache cache;
  if (4 * P >= n) build_cache(w, cache, threads);
  const int K = (sh_degree + 1) * (sh_degree + 1);
  const int nt = std::max(1, threads);
  const double amax = w.opt.amax;
  // Per-thread sparse accumulators: splat -> slot of [NP params | NP abs |
  // NP cond | NP clamp-tie | 3K sh | 3K sh abs].  Merged in thread order
  // (deterministic).
  const size_t slot = (size_t)4 * NP + (size_t)6 * K;
  std::vector<std::unordered_map<int64_t, size_t>> where(nt);
  std::vector<std::vector<double>> acc(nt);
  parallel_for(P, threads, [&](int t, int64_t a, int64_t b) {
    std::vector<PairRec> seq;
    auto cell = [&](int64_t g) -> double * {
      auto it = where[t].find(g);
      if (it == where[t].end()) {
        it = where[t].emplace(g, acc[t].size()).first;
        acc[t].resize(acc[t].size() + slot, 0.0);
      }
      return acc[t].data() + it->second;
    };
    for (int64_t i = a; i < b; ++i) {
      const int v = pix[3 * i], y = pix[3 * i + 1], x = pix[3 * i + 2];
      PixelOut po;
      render_pixel(w, cache, v, x, y, mg, flip ? flip[i] : 0u, po, seq);
      const double *Gp = G + 8 * i;
      const double px = x + 0.5 + w.opt.pix_off[0], py = y + 0.5 + w.opt.pix_off[1];
      const int m = (int)seq.size();
      // forward transmittances and per-pair scalar f_i
      std::vector<Splat<Dual>> sps(m);
      std::vector<Dual> dd(m), dep(m), aa(m);
      std::vector<double> T(m + 1), f(m), Fa(m);
      T[0] = 1.0;
      double n_eff = m + 2.0;
      for (int j = 0; j < m; ++j) {
        const int64_t g = seq[j].g;
        const Struct &st = w.st[(size_t)v * n + g];
        setup_splat<Dual>(sc32, sc64, g, w.camd[v], w.opt, st, sps[j]);
        eval_pair<Dual>(sps[j], w.camd[v], px, py, dd[j], dep[j]);
        aa[j] = seq[j].clamped ? Dual(amax) : sps[j].alpha_eff * dexp(-0.5 * dd[j]);
        T[j + 1] = T[j] * (1.0 - seq[j].alpha);
        const double terms[7] = {Gp[0] * val(sps[j].color[0]), Gp[1] * val(sps[j].color[1]),
                                 Gp[2] * val(sps[j].color[2]), Gp[4] * val(dep[j]),
                                 Gp[5] * val(sps[j].nrm[0]), Gp[6] * val(sps[j].nrm[1]),
                                 Gp[7] * val(sps[j].nrm[2])};
        f[j] = 0.0;
        Fa[j] = 0.0;
        for (int k = 0; k < 7; ++k) {
          f[j] += terms[k];
          Fa[j] += std::fabs(terms[k]);
        }
        if (!seq[j].clamped) {
          const double e_mag = 0.5 * std::fabs(dd[j].v) / std::log(2.0);
          n_eff += seq[j].alpha * (1.0 + e_mag) / (1.0 - seq[j].alpha);
        }
      }
      // alpha = 1 - T_final and rgb += T_final * bg: background term
      const double fbg = Gp[0] * w.opt.bg[0] + Gp[1] * w.opt.bg[1] + Gp[2] * w.opt.bg[2] - Gp[3];
      double Ssuf = fbg;  // S_m
      double Shat = std::fabs(Gp[0] * w.opt.bg[0]) + std::fabs(Gp[1] * w.opt.bg[1]) +
                    std::fabs(Gp[2] * w.opt.bg[2]) + std::fabs(Gp[3]);
      for (int j = m - 1; j >= 0; --j) {
        const int64_t g = seq[j].g;
        const double al = seq[j].alpha;
        const double dLda = T[j] * (f[j] - Ssuf);
        Ssuf = f[j] * al + (1.0 - al) * Ssuf;
        const double wgt = al * T[j];
        const Splat<Dual> &sp = sps[j];
        double *c = cell(g);
        double *gg = c, *ga = c + NP, *gcnd = c + 2 * NP, *gx = c + 3 * NP, *gs = c + 4 * NP,
               *as = c + 4 * NP + 3 * K;
        const double cond_a = T[j] * (Fa[j] + Shat) * n_eff;
        Shat = std::max(Shat, std::max(std::fabs(Ssuf), Fa[j]));
        const bool clamp_tie = std::fabs(seq[j].raw - amax) <= mg.clamp_rel * amax;
        Dual unc;
        if (clamp_tie) unc = sp.alpha_eff * dexp(-0.5 * dd[j]);
        // 3D: d(alpha~)/d(theta) goes through the screen-space quantities of
        // Eq. 1 (offset D = p - mu', conic Q); its magnitude form takes
        // sum_ab |D_a D_b| |dQ_ab| + 2 sum_a |(Q D)_a| |dmu'_a|.
        double D0 = 0, D1 = 0, QD0 = 0, QD1 = 0, gexp = 0;
        if (!sp.is2d) {
          D0 = px - sp.mu2[0].v;
          D1 = py - sp.mu2[1].v;
          QD0 = sp.conic[0].v * D0 + sp.conic[1].v * D1;
          QD1 = sp.conic[1].v * D0 + sp.conic[2].v * D1;
          gexp = std::exp(-0.5 * dd[j].v);
        }
        for (int q = 0; q < NP; ++q) {
          double terms[8];
          terms[0] = dLda * aa[j].d[q];
          terms[1] = wgt * Gp[4] * dep[j].d[q];
          for (int k = 0; k < 3; ++k) terms[2 + k] = wgt * Gp[5 + k] * sp.nrm[k].d[q];
          for (int k = 0; k < 3; ++k) terms[5 + k] = wgt * Gp[k] * sp.color[k].d[q];
          for (int k = 0; k < 8; ++k) { gg[q] += terms[k]; ga[q] += std::fabs(terms[k]); }
          double da = std::fabs(aa[j].d[q]);
          if (!sp.is2d && !seq[j].clamped) {
            const double cd = D0 * D0 * std::fabs(sp.conic[0].d[q]) +
                              2.0 * std::fabs(D0 * D1) * std::fabs(sp.conic[1].d[q]) +
                              D1 * D1 * std::fabs(sp.conic[2].d[q]) +
                              2.0 * (std::fabs(QD0) * std::fabs(sp.mu2[0].d[q]) +
                                     std::fabs(QD1) * std::fabs(sp.mu2[1].d[q]));
            da = std::fabs(sp.alpha_eff.d[q]) * gexp + al * 0.5 * cd;
          }
          gcnd[q] += cond_a * da;
          if (clamp_tie) gx[q] += std::fabs(dLda * unc.d[q]);
        }
        for (int ch = 0; ch < 3; ++ch) {
          if (sp.clamped[ch]) continue;
          const double dc = wgt * Gp[ch];
          for (int jj = 0; jj < K; ++jj) {
            gs[jj * 3 + ch] += dc * sp.Y[jj];
            as[jj * 3 + ch] += std::fabs(dc * sp.Y[jj]);
          }
        }
      }
    }
  });
  std::memset(g_params, 0, sizeof(double) * n * NP);
  std::memset(a_params, 0, sizeof(double) * n * NP);
  std::memset(c_params, 0, sizeof(double) * n * NP);
  std::memset(x_params, 0, sizeof(double) * n * NP);
  std::memset(g_sh, 0, sizeof(double) * n * K * 3);
  std::memset(a_sh, 0, sizeof(double) * n * K * 3);
  for (int t = 0; t < nt; ++t) {
    std::vector<std::pair<int64_t, size_t>> order(where[t].begin(), where[t].end());
    std::sort(order.begin(), order.end());
    for (const auto &e : order) {
      const double *c = acc[t].data() + e.second;
      const int64_t g = e.first;
      for (int q = 0; q < NP; ++q) {
        g_params[g * NP + q] += c[q];
        a_params[g * NP + q] += c[NP + q];
        c_params[g * NP + q] += c[2 * NP + q];
        x_params[g * NP + q] += c[3 * NP + q];
      }
      for (int j = 0; j < 3 * K; ++j) {
        g_sh[g * 3 * K + j] += c[4 * NP + j];
        a_sh[g * 3 * K + j] += c[4 * NP + 3 * K + j];
      }
    }
  }
  return 0;
}

// Screen-space translation gradient of every (view, splat) for
// L = sum over the listed pixels of <G, out>.  Translating splat (v, g)'s
// screen footprint by delta means evaluating it at p - delta, so
//   dL/d delta = - sum_p [dL/dalpha~ d alpha~/dp + dL/ddepth d depth/dp]
// over the splat's blended pairs (alpha~ = alpha_eff exp(-d/2) unless it is
// clamped, where it does not move).  3D: d = D^T Q D with D = p - mu', so
// dd/dp = 2 Q D, and the depth is fixed.  2D: (u, v, kappa) solve
// M (u, v, kappa) = -p_c with M = [s_x t_u | s_y t_v | -omega],
// omega = ((px - cx)/fx, (py - cy)/fy, 1); differentiating M x = r in
// omega_k gives d(u, v, kappa)/d omega_k = kappa M^{-1} e_k; d = u^2 + v^2,
// depth = kappa.  Tie branches as in oracle_backward.  out: [V*n, 2],
// binary64.
int oracle_screen_grad(const float *m32, const float *s32, const float *r32, const float *o32,
                       const float *sh32, const uint8_t *types, int64_t n, int sh_degree,
                       const double *m64, const double *s64, const double *r64,
                       const double *o64, const double *sh64, const float *cams, int V,
                       const double *opts, const double *margins, const int32_t *pix, int64_t P,
                       const uint32_t *flip, const double *G, int threads, double *out) {
  Scene32 sc32{m32, s32, r32, o32, sh32, types, n, sh_degree};
  Scene64 sc64{m64, s64, r64, o64, sh64};
  Work w;
  w.s32 = &sc32;
  w.s64 = &sc64;
  w.opt = load_opts(opts);
  build(w, cams, V, false);
  const Margins mg{margins[0], margins[1], margins[2]};
  SplatCache cache;
  if (4 * P >= n) build_cache(w, cache, threads);
  const int nt = std::max(1, threads);
  std::vector<std::unordered_map<int64_t, std::array<double, 2>>> acc(nt);
  parallel_for(P, threads, [&](int t, int64_t a, int64_t b) {
    std::vector<PairRec> seq;
    Splat<double> tmp;
    for (int64_t i = a; i < b; ++i) {
      const int v = pix[3 * i], y = pix[3 * i + 1], x = pix[3 * i + 2];
      PixelOut po;
      render_pixel(w, cache, v, x, y, mg, flip ? flip[i] : 0u, po, seq);
      const double *Gp = G + 8 * i;
      const CamD &cd = w.camd[v];
      const double px = x + 0.5 + w.opt.pix_off[0], py = y + 0.5 + w.opt.pix_off[1];
      const int m = (int)seq.size();
      std::vector<double> T(m + 1), f(m), dgx(m), dgy(m), ddx(m), ddy(m);
      T[0] = 1.0;
      for (int j = 0; j < m; ++j) {
        const Splat<double> &sp = get_splat(w, cache, v, seq[j].g, tmp);
        double d, dep;
        eval_pair<double>(sp, cd, px, py, d, dep);
        T[j + 1] = T[j] * (1.0 - seq[j].alpha);
        f[j] = Gp[0] * sp.color[0] + Gp[1] * sp.color[1] + Gp[2] * sp.color[2] + Gp[4] * dep +
               Gp[5] * sp.nrm[0] + Gp[6] * sp.nrm[1] + Gp[7] * sp.nrm[2];
        // d(d)/dp and d(depth)/dp
        if (!sp.is2d) {
          const double D0 = px - sp.mu2[0], D1 = py - sp.mu2[1];
          ddx[j] = 2.0 * (sp.conic[0] * D0 + sp.conic[1] * D1);
          ddy[j] = 2.0 * (sp.conic[1] * D0 + sp.conic[2] * D1);
          dgx[j] = dgy[j] = 0.0;
        } else {
          const double om[3] = {(px - cd.cx) / cd.fx, (py - cd.cy) / cd.fy, 1.0};
          double u, vv, kap;
          surfel_hit<double>(sp, om, u, vv, kap);
          double A[3], B[3], Mo[3];
          for (int k = 0; k < 3; ++k) {
            A[k] = sp.sx * sp.tu[k];
            B[k] = sp.sy * sp.tv[k];
            Mo[k] = -om[k];
          }
          auto det3 = [](const double *c0, const double *c1, const double *c2) {
            return c0[0] * (c1[1] * c2[2] - c1[2] * c2[1]) -
                   c0[1] * (c1[0] * c2[2] - c1[2] * c2[0]) +
                   c0[2] * (c1[0] * c2[1] - c1[1] * c2[0]);
          };
          const double Dm = det3(A, B, Mo);
          double dx3[2][3];  // d(u, v, kappa)/d(px), d(py)
          for (int k = 0; k < 2; ++k) {
            double e[3] = {0, 0, 0};
            e[k] = 1.0;
            const double sc = kap / (k == 0 ? cd.fx : cd.fy);
            dx3[k][0] = sc * det3(e, B, Mo) / Dm;
            dx3[k][1] = sc * det3(A, e, Mo) / Dm;
            dx3[k][2] = sc * det3(A, B, e) / Dm;
          }
          ddx[j] = 2.0 * u * dx3[0][0] + 2.0 * vv * dx3[0][1];
          ddy[j] = 2.0 * u * dx3[1][0] + 2.0 * vv * dx3[1][1];
          dgx[j] = dx3[0][2];
          dgy[j] = dx3[1][2];
        }
      }
      double Ssuf = Gp[0] * w.opt.bg[0] + Gp[1] * w.opt.bg[1] + Gp[2] * w.opt.bg[2] - Gp[3];
      for (int j = m - 1; j >= 0; --j) {
        const double al = seq[j].alpha;
        const double dLda = T[j] * (f[j] - Ssuf);
        Ssuf = f[j] * al + (1.0 - al) * Ssuf;
        const double wgt = al * T[j];
        const double da = seq[j].clamped ? 0.0 : -0.5 * seq[j].raw;  // d alpha~ / d d
        const double gx = dLda * da * ddx[j] + Gp[4] * wgt * dgx[j];
        const double gy = dLda * da * ddy[j] + Gp[4] * wgt * dgy[j];
        auto &c = acc[t][(int64_t)v * n + seq[j].g];
        c[0] -= gx;
        c[1] -= gy;
      }
    }
  });
  std::memset(out, 0, sizeof(double) * (size_t)V * n * 2);
  for (int t = 0; t < nt; ++t) {
    std::vector<std::pair<int64_t, std::array<double, 2>>> order(acc[t].begin(), acc[t].end());
    std::sort(order.begin(), order.end(),
              [](const auto &a, const auto &b) { return a.first < b.first; });
    for (const auto &e : order) {
      out[2 * e.first] += e.second[0];
      out[2 * e.first + 1] += e.second[1];
    }
  }
  return 0;
}

// Real SH basis at unit directions (for the basis pins): dirs [P,3] -> Y [P,K].
int oracle_sh_basis(int degree, const double *dirs, int64_t P, double *Y) {
  const int K = (degree + 1) * (degree + 1);
  for (int64_t i = 0; i < P; ++i) {
    double d[3] = {dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
    double y[16];
    sh_basis<double>(degree, d, y);
    for (int j = 0; j < K; ++j) Y[i * K + j] = y[j];
  }
  return 0;
}

// 2D ray-plane coordinates (u, v) and hit depth of one surfel at a list of
// pixel samples, for the pins of Eq. uv.  params = mu[3], s[3], q[4].
int oracle_surfel_uv(const double *params, const float *cam, const double *pxy, int64_t P,
                     double *uvz) {
  Cam c = load_cam(cam);
  CamD cd = cam_d(c);
  float m32[3], s32f[3], r32[4], o32 = 0.5f;
  uint8_t t = 0;
  for (int i = 0; i < 3; ++i) { m32[i] = (float)params[i]; s32f[i] = (float)params[3 + i]; }
  for (int i = 0; i < 4; ++i) r32[i] = (float)params[6 + i];
  double o64 = 0.5, sh[3] = {0.0, 0.0, 0.0};
  Scene32 s{m32, s32f, r32, &o32, nullptr, &t, 1, 0};
  Scene64 p{params, params + 3, params + 6, &o64, sh};
  Opts opt{{0, 0, 0}, 0.0f, 1.0, 1.05, 0.001, {0.0, 0.0}, kAlphaMin, kAlphaMax, kTMin};
  Struct st{};
  Splat<double> sp;
  setup_splat<double>(s, p, 0, cd, opt, st, sp);
  for (int64_t i = 0; i < P; ++i) {
    const double px = pxy[2 * i], py = pxy[2 * i + 1];
    const double om[3] = {(px - cd.cx) / cd.fx, (py - cd.cy) / cd.fy, 1.0};
    double u, v, kap;
    surfel_hit<double>(sp, om, u, v, kap);
    uvz[3 * i] = u;
    uvz[3 * i + 1] = v;
    uvz[3 * i + 2] = kap;
  }
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adaptive Type Exchange (Sec. 3.2 and the appendix "Effective Rank and Type
// Switch").  Per primitive, in binary64 from the binary32 inputs:
//   erank = exp(-sum_i p_i log p_i), p = q / |q|_1, q = (s_x^2, s_y^2, s_z^2)
//   (Eq. 3; 0 log 0 = 0; all-zero scales: erank = 0, no switch).
//   3D (t != 0) with erank < theta_e: the least significant scale is moved to
//   z by S* = P S P^T and R* = R P^T, with P = P_x when s_x is the least and
//   P = P_y when s_y is (z before y before x on ties, so nothing moves when
//   s_z is a least); the type becomes 2D.  The quaternion of R* is taken
//   from the matrix (largest-diagonal branch), unit length, w >= 0.
//   2D with erank > theta_e: the type becomes 3D, parameters unchanged.
// Outputs: types_out u8[n], scales_out f32[n,3] (a permutation of the input
// scales), quats_out f64[n,4] (unit; the input quaternion normalised when
// the rotation is kept), erank f64[n], moved i32[n] (0 none, 1 P_x, 2 P_y).
static void quat_to_mat(const double q[4], double R[9]) {
  const double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void mat_to_quat(const double R[9], double q[4]) {
  const double tr = R[0] + R[4] + R[8];
  double w, x, y, z;
  if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
    const double r = std::sqrt(1.0 + tr);
    w = 0.5 * r;
    x = (R[7] - R[5]) / (2 * r);
    y = (R[2] - R[6]) / (2 * r);
    z = (R[3] - R[1]) / (2 * r);
  } else if (R[0] >= R[4] && R[0] >= R[8]) {
    const double r = std::sqrt(1.0 + R[0] - R[4] - R[8]);
    x = 0.5 * r;
    w = (R[7] - R[5]) / (2 * r);
    y = (R[1] + R[3]) / (2 * r);
    z = (R[2] + R[6]) / (2 * r);
  } else if (R[4] >= R[8]) {
    const double r = std::sqrt(1.0 - R[0] + R[4] - R[8]);
    y = 0.5 * r;
    w = (R[2] - R[6]) / (2 * r);
    x = (R[1] + R[3]) / (2 * r);
    z = (R[5] + R[7]) / (2 * r);
  } else {
    const double r = std::sqrt(1.0 - R[0] - R[4] + R[8]);
    z = 0.5 * r;
    w = (R[3] - R[1]) / (2 * r);
    x = (R[2] + R[6]) / (2 * r);
    y = (R[5] + R[7]) / (2 * r);
  }
  const double n = std::sqrt(w * w + x * x + y * y + z * z) * (w < 0 ? -1.0 : 1.0);
  q[0] = w / n; q[1] = x / n; q[2] = y / n; q[3] = z / n;
}

extern "C" double oracle_erank(double sx, double sy, double sz) {
  const double q[3] = {sx * sx, sy * sy, sz * sz};
  const double sum = q[0] + q[1] + q[2];
  if (!(sum > 0.0)) return 0.0;
  double h = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double p = q[i] / sum;
    if (p > 0.0) h -= p * std::log(p);
  }
  return std::exp(h);
}

extern "C" int oracle_type_exchange(const float *scales, const float *rots, const uint8_t *types,
                                    int64_t n, double theta, uint8_t *types_out,
                                    float *scales_out, double *quats_out, double *erank,
                                    int32_t *moved) {
  // P_x and P_y as row-major matrices (the appendix's definitions)
  static const double Px[9] = {0, 1, 0, 0, 0, 1, 1, 0, 0};
  static const double Py[9] = {0, 0, 1, 1, 0, 0, 0, 1, 0};
  for (int64_t i = 0; i < n; ++i) {
    const float *s = scales + 3 * i;
    const double e = oracle_erank(s[0], s[1], s[2]);
    erank[i] = e;
    double q[4] = {rots[4 * i], rots[4 * i + 1], rots[4 * i + 2], rots[4 * i + 3]};
    const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) quats_out[4 * i + k] = q[k] / qn;
    for (int k = 0; k < 3; ++k) scales_out[3 * i + k] = s[k];
    moved[i] = 0;
    const bool is3d = types[i] != 0;
    types_out[i] = is3d ? 1 : 0;
    if (is3d && e > 0.0 && e < theta) {
      types_out[i] = 0;
      const double *P = nullptr;
      if (s[2] <= s[0] && s[2] <= s[1]) {
        P = nullptr;
      } else if (s[1] <= s[0]) {
        P = Py;
        moved[i] = 2;
      } else {
        P = Px;
        moved[i] = 1;
      }
      if (P) {
        // S* = P S P^T: diagonal entries (P S P^T)_ii = s_j where P_ij = 1
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c)
            if (P[3 * r + c] != 0.0) scales_out[3 * i + r] = s[c];
        // R* = R P^T
        double R[9], Rs[9];
        quat_to_mat(q, R);
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += R[3 * r + k] * P[3 * c + k];  // (P^T)_kc = P_ck
            Rs[3 * r + c] = acc;
          }
        mat_to_quat(Rs, quats_out + 4 * i);
      }
    } else if (!is3d && e > theta) {
      types_out[i] = 1;
    }
  }
  return 0;
}
