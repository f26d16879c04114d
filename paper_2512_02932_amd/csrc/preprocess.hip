// Preprocess (forward and backward) of the hybrid rasterizer, gfx950.
//
// One thread per (view, primitive).  Forward:
//   * structural decisions in binary32 with a fixed operation order and no
//     contraction: cull, conservative pixel rectangle, tiles touched, depth
//     key, normal orientation.  The test suite checks these bit for bit.
//   * continuous per-splat quantities in binary64 (CDNA runs FP64 vector
//     code at the FP32 rate, and this kernel is memory-bound), rounded once
//     into an 80-byte record in a splat-local pixel frame:
//       3D (Sec. 3.1 + appendix "affine projection"): Sigma = R S S^T R^T,
//          Sigma' = J W Sigma W^T J^T + delta I, conic = Sigma'^{-1},
//          mu' = projected centre.
//       2D (appendix "ray-splat intersection", Eq. uv): the map from the
//          surfel plane (u, v, 1) to homogeneous pixels is M = K [s_x t_u |
//          s_y t_v | p_c]; its inverse takes a pixel to (u, v, 1)/z, which
//          is the homogeneous-plane solution of Eq. uv in matrix form.
//       colour from real SH (degree <= 3) at the view direction; opacity of
//       2D surfels through Eq. 6-7; camera-space normal.
// Backward: the chain rule from the per-splat accumulators written by the
// raster backward to mu, s, q, alpha (and s_z via Eq. 6-7) and SH, summed
// over views, in binary64.

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr float kRR0 = 11.0825272f;     // smallest binary32 >= 2 ln 255
constexpr float kPad = 1.00390625f;     // 1 + 2^-8
constexpr double kLog2e = 1.4426950408889634;

struct Structural {
  int valid;
  int px0, py0, px1, py1;
  uint32_t tiles;
  uint32_t zbits;
  int flip;
  int axis;
};

// ---------------------------------------------------------------------------
// Structural decisions, binary32.  The operation order below is the
// specification; no fused multiply-add may be formed.
// ---------------------------------------------------------------------------
__host__ __device__ Structural structural_f32(const float *m, const float *sc, const float *q,
                                              float al, bool is2d, const DevCam &c,
                                              float delta) {
#pragma clang fp contract(off)
  Structural o;
  o.valid = 0;
  o.px0 = o.py0 = o.px1 = o.py1 = 0;
  o.tiles = 0;
  o.zbits = 0;
  o.flip = 0;
  o.axis = 2;
  const float *V = c.V;
  const float xc = ((V[0] * m[0] + V[1] * m[1]) + V[2] * m[2]) + V[3];
  const float yc = ((V[4] * m[0] + V[5] * m[1]) + V[6] * m[2]) + V[7];
  const float zc = ((V[8] * m[0] + V[9] * m[1]) + V[10] * m[2]) + V[11];
  if (!(zc > c.znear)) return o;
  if (!(al >= kAlphaMin)) return o;

  const float qw = q[0], qx = q[1], qy = q[2], qz = q[3];
  const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  if (!(n2 > 0.0f)) return o;
  const float k2 = 2.0f / n2;
  float R[9];
  R[0] = 1.0f - k2 * (qy * qy + qz * qz);
  R[1] = k2 * (qx * qy - qw * qz);
  R[2] = k2 * (qx * qz + qw * qy);
  R[3] = k2 * (qx * qy + qw * qz);
  R[4] = 1.0f - k2 * (qx * qx + qz * qz);
  R[5] = k2 * (qy * qz - qw * qx);
  R[6] = k2 * (qx * qz - qw * qy);
  R[7] = k2 * (qy * qz + qw * qx);
  R[8] = 1.0f - k2 * (qx * qx + qy * qy);

  const float rr = kRR0 + 4.0f * ((al - 1.0f) / (al + 1.0f));

  // camera-space scaled axes, column j = R_v (R e_j s_j)
  float C[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float w0 = R[j] * sc[j], w1 = R[3 + j] * sc[j], w2 = R[6 + j] * sc[j];
#pragma unroll
    for (int i = 0; i < 3; ++i) C[3 * i + j] = (V[4 * i] * w0 + V[4 * i + 1] * w1) + V[4 * i + 2] * w2;
  }

  const float Wm1 = (float)(c.W - 1), Hm1 = (float)(c.H - 1);
  float xlo, xhi, ylo, yhi;
  int k;
  if (!is2d) {
    const float iz = 1.0f / zc;
    const float u = xc * iz, v = yc * iz;
    const float a0 = c.fx * iz, a1 = c.fy * iz;
    float A0[3], A1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      A0[j] = a0 * (C[j] - u * C[6 + j]);
      A1[j] = a1 * (C[3 + j] - v * C[6 + j]);
    }
    const float S00 = ((A0[0] * A0[0] + A0[1] * A0[1]) + A0[2] * A0[2]) + delta;
    const float S01 = (A0[0] * A1[0] + A0[1] * A1[1]) + A0[2] * A1[2];
    const float S11 = ((A1[0] * A1[0] + A1[1] * A1[1]) + A1[2] * A1[2]) + delta;
    const float det = S00 * S11 - S01 * S01;
    if (!(det > 0.0f)) return o;
    const float mux = c.fx * u + c.cx, muy = c.fy * v + c.cy;
    const float hx = sqrtf(rr * S00) * kPad, hy = sqrtf(rr * S11) * kPad;
    xlo = (mux - hx) - 0.5f;
    xhi = (mux + hx) - 0.5f;
    ylo = (muy - hy) - 0.5f;
    yhi = (muy + hy) - 0.5f;
    k = (sc[2] <= sc[0] && sc[2] <= sc[1]) ? 2 : (sc[1] <= sc[0] ? 1 : 0);
  } else {
    if (!(sc[0] > 0.0f) || !(sc[1] > 0.0f)) return o;
    const float qq = C[6] * C[6] + C[7] * C[7];
    const float e = sqrtf(rr * qq);
    if (!(zc - e > c.znear)) return o;
    const float E22 = rr * qq - zc * zc;
    if (!(E22 < 0.0f)) return o;
    const float pcv[2] = {xc, yc};
    const float fv[2] = {c.fx, c.fy}, cv[2] = {c.cx, c.cy};
    float lo[2], hi[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const float ca0 = C[3 * a], ca1 = C[3 * a + 1];
      const float Ea2 = rr * (ca0 * C[6] + ca1 * C[7]) - pcv[a] * zc;
      const float n01 = ca0 * C[7] - ca1 * C[6];
      const float n02 = ca0 * zc - pcv[a] * C[6];
      const float n12 = ca1 * zc - pcv[a] * C[7];
      float disc = rr * (n02 * n02 + n12 * n12) - (rr * rr) * (n01 * n01);
      if (!(disc >= 0.0f)) disc = 0.0f;
      const float cen = cv[a] + fv[a] * (Ea2 / E22);
      const float h = (fv[a] * (sqrtf(disc) / (-E22))) * kPad;
      lo[a] = (cen - h) - 0.5f;
      hi[a] = (cen + h) - 0.5f;
    }
    xlo = lo[0];
    xhi = hi[0];
    ylo = lo[1];
    yhi = hi[1];
    k = 2;
  }
  if (!(xhi >= 0.0f) || !(xlo <= Wm1) || !(yhi >= 0.0f) || !(ylo <= Hm1)) return o;
  const int px0 = (xlo <= 0.0f) ? 0 : (int)ceilf(xlo);
  const int px1 = (xhi >= Wm1) ? c.W - 1 : (int)floorf(xhi);
  const int py0 = (ylo <= 0.0f) ? 0 : (int)ceilf(ylo);
  const int py1 = (yhi >= Hm1) ? c.H - 1 : (int)floorf(yhi);
  if (px0 > px1 || py0 > py1) return o;

  const float nc0 = (V[0] * R[k] + V[1] * R[3 + k]) + V[2] * R[6 + k];
  const float nc1 = (V[4] * R[k] + V[5] * R[3 + k]) + V[6] * R[6 + k];
  const float nc2 = (V[8] * R[k] + V[9] * R[3 + k]) + V[10] * R[6 + k];
  const float dot = (nc0 * xc + nc1 * yc) + nc2 * zc;

  o.valid = 1;
  o.px0 = px0;
  o.px1 = px1;
  o.py0 = py0;
  o.py1 = py1;
  o.tiles = (uint32_t)(((px1 >> 4) - (px0 >> 4) + 1) * ((py1 >> 4) - (py0 >> 4) + 1));
  uint32_t zb;
  __builtin_memcpy(&zb, &zc, 4);
  o.zbits = zb;
  o.flip = dot > 0.0f ? 1 : 0;
  o.axis = k;
  return o;
}

// ---------------------------------------------------------------------------
// Real spherical harmonics up to degree 3 (Condon-Shortley phase), as
// polynomials of the unit direction, and their gradient.
// Coefficient j = l^2 + l + m.
// ---------------------------------------------------------------------------
constexpr double kY0 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
constexpr double kY1 = 0.48860251190291992;   // sqrt(3 / (4 pi))
constexpr double kY2a = 1.0925484305920792;   // sqrt(15 / (4 pi))
constexpr double kY2b = 0.31539156525252005;  // sqrt(5 / (16 pi))
constexpr double kY2c = 0.54627421529603959;  // sqrt(15 / (16 pi))
constexpr double kY3a = 0.59004358992664352;  // sqrt(35 / (32 pi))
constexpr double kY3b = 2.8906114426405538;   // sqrt(105 / (4 pi))
constexpr double kY3c = 0.45704579946446572;  // sqrt(21 / (32 pi))
constexpr double kY3d = 0.37317633259011546;  // sqrt(7 / (16 pi))
constexpr double kY3e = 1.4453057213202769;   // sqrt(105 / (16 pi))

__device__ inline void sh_basis(int deg, double x, double y, double z, double *Y,
                                double (*dY)[3]) {
  Y[0] = kY0;
  dY[0][0] = dY[0][1] = dY[0][2] = 0.0;
  if (deg < 1) return;
  Y[1] = -kY1 * y;  dY[1][0] = 0;        dY[1][1] = -kY1;     dY[1][2] = 0;
  Y[2] = kY1 * z;   dY[2][0] = 0;        dY[2][1] = 0;        dY[2][2] = kY1;
  Y[3] = -kY1 * x;  dY[3][0] = -kY1;     dY[3][1] = 0;        dY[3][2] = 0;
  if (deg < 2) return;
  Y[4] = kY2a * x * y;
  dY[4][0] = kY2a * y; dY[4][1] = kY2a * x; dY[4][2] = 0;
  Y[5] = -kY2a * y * z;
  dY[5][0] = 0; dY[5][1] = -kY2a * z; dY[5][2] = -kY2a * y;
  Y[6] = kY2b * (3.0 * z * z - 1.0);
  dY[6][0] = 0; dY[6][1] = 0; dY[6][2] = 6.0 * kY2b * z;
  Y[7] = -kY2a * x * z;
  dY[7][0] = -kY2a * z; dY[7][1] = 0; dY[7][2] = -kY2a * x;
  Y[8] = kY2c * (x * x - y * y);
  dY[8][0] = 2.0 * kY2c * x; dY[8][1] = -2.0 * kY2c * y; dY[8][2] = 0;
  if (deg < 3) return;
  Y[9] = -kY3a * y * (3.0 * x * x - y * y);
  dY[9][0] = -kY3a * 6.0 * x * y; dY[9][1] = -kY3a * (3.0 * x * x - 3.0 * y * y); dY[9][2] = 0;
  Y[10] = kY3b * x * y * z;
  dY[10][0] = kY3b * y * z; dY[10][1] = kY3b * x * z; dY[10][2] = kY3b * x * y;
  Y[11] = -kY3c * y * (5.0 * z * z - 1.0);
  dY[11][0] = 0; dY[11][1] = -kY3c * (5.0 * z * z - 1.0); dY[11][2] = -kY3c * 10.0 * y * z;
  Y[12] = kY3d * z * (5.0 * z * z - 3.0);
  dY[12][0] = 0; dY[12][1] = 0; dY[12][2] = kY3d * (15.0 * z * z - 3.0);
  Y[13] = -kY3c * x * (5.0 * z * z - 1.0);
  dY[13][0] = -kY3c * (5.0 * z * z - 1.0); dY[13][1] = 0; dY[13][2] = -kY3c * 10.0 * x * z;
  Y[14] = kY3e * z * (x * x - y * y);
  dY[14][0] = kY3e * 2.0 * x * z; dY[14][1] = -kY3e * 2.0 * y * z; dY[14][2] = kY3e * (x * x - y * y);
  Y[15] = -kY3a * x * (x * x - 3.0 * y * y);
  dY[15][0] = -kY3a * (3.0 * x * x - 3.0 * y * y); dY[15][1] = kY3a * 6.0 * x * y; dY[15][2] = 0;
}

// ---------------------------------------------------------------------------
// Continuous per-(view, splat) quantities, binary64.
// ---------------------------------------------------------------------------
struct Geo {
  double q[4], qn;      // normalised quaternion and |r|
  double R[9];          // rotation (row-major)
  double s[3];
  double pc[3];         // camera-space centre
  double RvR[9];        // R_v R
  double dir[3], dist;  // unit direction camera centre -> mean, distance
  double alpha_eff, gate_sig, gate_arg;
  double color[3];
  int clamped[3];
  double Y[16];
  double dY[16][3];
  double nrm[3];        // oriented camera-space normal
  double ox, oy;        // local pixel frame origin (integers)
  // 3D
  double A[6];          // 2x3, Sigma' = A A^T + delta I
  double Sp[3];         // Sigma' (00, 01, 11)
  double conic[3];
  double mu2[2];
  // 2D
  double M[9];          // plane -> pixel map in the local frame
  double Hi[9];         // M^{-1}
};

__device__ inline double frame_origin(double v) {
  double f = floor(v);
  if (!(f > -1.0e6)) f = -1.0e6;  // also catches NaN
  if (f > 1.0e6) f = 1.0e6;
  return f;
}

__device__ void geo_setup(const SceneDev &sc, int64_t g, const DevCam &c, const DevOpts &opt,
                          const Structural &st, bool is2d, Geo &o) {
  const float *mf = sc.means + 3 * g;
  const float *sf = sc.scales + 3 * g;
  const float *qf = sc.rots + 4 * g;
  const double mu[3] = {mf[0], mf[1], mf[2]};
  for (int i = 0; i < 3; ++i) o.s[i] = sf[i];
  const double r[4] = {qf[0], qf[1], qf[2], qf[3]};
  o.qn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
  for (int i = 0; i < 4; ++i) o.q[i] = r[i] / o.qn;
  const double w = o.q[0], x = o.q[1], y = o.q[2], z = o.q[3];
  o.R[0] = 1.0 - 2.0 * (y * y + z * z);
  o.R[1] = 2.0 * (x * y - w * z);
  o.R[2] = 2.0 * (x * z + w * y);
  o.R[3] = 2.0 * (x * y + w * z);
  o.R[4] = 1.0 - 2.0 * (x * x + z * z);
  o.R[5] = 2.0 * (y * z - w * x);
  o.R[6] = 2.0 * (x * z - w * y);
  o.R[7] = 2.0 * (y * z + w * x);
  o.R[8] = 1.0 - 2.0 * (x * x + y * y);
  const double *Vd = c.Vd;
  for (int i = 0; i < 3; ++i)
    o.pc[i] = Vd[4 * i] * mu[0] + Vd[4 * i + 1] * mu[1] + Vd[4 * i + 2] * mu[2] + Vd[4 * i + 3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      o.RvR[3 * i + j] = Vd[4 * i] * o.R[j] + Vd[4 * i + 1] * o.R[3 + j] + Vd[4 * i + 2] * o.R[6 + j];

  // opacity; 2D: alpha* = alpha exp(-lambda_z sigmoid((s_z - theta_z)/T_z) s_z)
  const double al = sc.opac[g];
  if (is2d) {
    o.gate_arg = (o.s[2] - (double)opt.theta_z) / (double)opt.temp_z;
    const double za = o.gate_arg;
    o.gate_sig = za >= 0 ? 1.0 / (1.0 + exp(-za)) : exp(za) / (1.0 + exp(za));
    o.alpha_eff = al * exp(-(double)opt.lambda_z * o.gate_sig * o.s[2]);
  } else {
    o.gate_arg = 0.0;
    o.gate_sig = 0.0;
    o.alpha_eff = al;
  }

  // colour
  double dv[3];
  for (int i = 0; i < 3; ++i) dv[i] = mu[i] - c.o[i];
  o.dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int i = 0; i < 3; ++i) o.dir[i] = dv[i] / o.dist;
  const int deg = sc.sh_degree;
  const int K = (deg + 1) * (deg + 1);
  sh_basis(deg, o.dir[0], o.dir[1], o.dir[2], o.Y, o.dY);
  const float *shp = sc.sh + (size_t)g * K * 3;
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.5;
    for (int j = 0; j < K; ++j) acc += (double)shp[3 * j + ch] * o.Y[j];
    o.clamped[ch] = !(acc > 0.0);
    o.color[ch] = o.clamped[ch] ? 0.0 : acc;
  }

  // normal
  const double sg = st.flip ? -1.0 : 1.0;
  for (int i = 0; i < 3; ++i) o.nrm[i] = sg * o.RvR[3 * i + st.axis];

  const double X = o.pc[0], Yc = o.pc[1], Z = o.pc[2];
  const double fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy;
  if (!is2d) {
    // A = J R_v R S (2x3): Sigma' = A A^T + delta I
    const double J00 = fx / Z, J02 = -fx * X / (Z * Z), J11 = fy / Z, J12 = -fy * Yc / (Z * Z);
    for (int j = 0; j < 3; ++j) {
      const double c0 = o.RvR[j] * o.s[j], c1 = o.RvR[3 + j] * o.s[j], c2 = o.RvR[6 + j] * o.s[j];
      o.A[j] = J00 * c0 + J02 * c2;
      o.A[3 + j] = J11 * c1 + J12 * c2;
    }
    o.Sp[0] = o.A[0] * o.A[0] + o.A[1] * o.A[1] + o.A[2] * o.A[2] + (double)opt.dilation;
    o.Sp[1] = o.A[0] * o.A[3] + o.A[1] * o.A[4] + o.A[2] * o.A[5];
    o.Sp[2] = o.A[3] * o.A[3] + o.A[4] * o.A[4] + o.A[5] * o.A[5] + (double)opt.dilation;
    const double det = o.Sp[0] * o.Sp[2] - o.Sp[1] * o.Sp[1];
    o.conic[0] = o.Sp[2] / det;
    o.conic[1] = -o.Sp[1] / det;
    o.conic[2] = o.Sp[0] / det;
    o.mu2[0] = fx * X / Z + cx;
    o.mu2[1] = fy * Yc / Z + cy;
    o.ox = frame_origin(o.mu2[0]);
    o.oy = frame_origin(o.mu2[1]);
  } else {
    o.ox = frame_origin(fx * X / Z + cx);
    o.oy = frame_origin(fy * Yc / Z + cy);
    const double cxl = cx - o.ox, cyl = cy - o.oy;
    double Cm[9];  // columns s_x t_u, s_y t_v, p_c (camera frame)
    for (int i = 0; i < 3; ++i) {
      Cm[3 * i] = o.s[0] * o.RvR[3 * i];
      Cm[3 * i + 1] = o.s[1] * o.RvR[3 * i + 1];
      Cm[3 * i + 2] = o.pc[i];
    }
    for (int j = 0; j < 3; ++j) {
      o.M[j] = fx * Cm[j] + cxl * Cm[6 + j];
      o.M[3 + j] = fy * Cm[3 + j] + cyl * Cm[6 + j];
      o.M[6 + j] = Cm[6 + j];
    }
    const double *M = o.M;
    const double a00 = M[4] * M[8] - M[5] * M[7];
    const double a01 = M[2] * M[7] - M[1] * M[8];
    const double a02 = M[1] * M[5] - M[2] * M[4];
    const double det = M[0] * a00 + M[3] * a01 + M[6] * a02;
    const double id = 1.0 / det;
    o.Hi[0] = a00 * id;
    o.Hi[1] = a01 * id;
    o.Hi[2] = a02 * id;
    o.Hi[3] = (M[5] * M[6] - M[3] * M[8]) * id;
    o.Hi[4] = (M[0] * M[8] - M[2] * M[6]) * id;
    o.Hi[5] = (M[2] * M[3] - M[0] * M[5]) * id;
    o.Hi[6] = (M[3] * M[7] - M[4] * M[6]) * id;
    o.Hi[7] = (M[1] * M[6] - M[0] * M[7]) * id;
    o.Hi[8] = (M[0] * M[4] - M[1] * M[3]) * id;
  }
}

__global__ void __launch_bounds__(256)
preprocess_kernel(SceneDev sc, const DevCam *__restrict__ cams, int V, DevOpts opt,
                  Record *__restrict__ rec, uint32_t *__restrict__ tiles,
                  uint32_t *__restrict__ zbits, int4 *__restrict__ rect) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)V * sc.n;
  if (i >= total) return;
  const int v = (int)(i / sc.n);
  const int64_t g = i - (int64_t)v * sc.n;
  const DevCam &c = cams[v];
  const bool is2d = sc.types[g] == 0;
  const float m[3] = {sc.means[3 * g], sc.means[3 * g + 1], sc.means[3 * g + 2]};
  const float s[3] = {sc.scales[3 * g], sc.scales[3 * g + 1], sc.scales[3 * g + 2]};
  const float q[4] = {sc.rots[4 * g], sc.rots[4 * g + 1], sc.rots[4 * g + 2], sc.rots[4 * g + 3]};
  const Structural st = structural_f32(m, s, q, sc.opac[g], is2d, c, opt.dilation);
  tiles[i] = st.valid ? st.tiles : 0u;
  zbits[i] = st.zbits;
  rect[i] = make_int4(st.px0, st.py0, st.px1, st.py1);
  if (!st.valid) return;

  Geo o;
  geo_setup(sc, g, c, opt, st, is2d, o);
  Record r;
  const double k2 = sqrt(0.5 * kLog2e);
  float aeff = (float)o.alpha_eff;
  if (!is2d) {
    const float mx = (float)(o.mu2[0] - o.ox), my = (float)(o.mu2[1] - o.oy);
    const float A = (float)(0.5 * kLog2e * o.conic[0]);
    const float B = (float)(kLog2e * o.conic[1]);
    const float C = (float)(0.5 * kLog2e * o.conic[2]);
    if (!(isfinite(mx) && isfinite(my) && isfinite(A) && isfinite(B) && isfinite(C))) aeff = 0.0f;
    r.r[0] = make_float4(1.0f, (float)o.ox, (float)o.oy, aeff);
    r.r[1] = make_float4(mx, my, A, B);
    r.r[2] = make_float4(C, 0.0f, 0.0f, 0.0f);
    r.r[3] = make_float4(0.0f, (float)o.color[0], (float)o.color[1], (float)o.color[2]);
    r.r[4] = make_float4((float)o.nrm[0], (float)o.nrm[1], (float)o.nrm[2], (float)o.pc[2]);
  } else {
    float h[9];
    bool fin = true;
    for (int j = 0; j < 9; ++j) {
      h[j] = (float)(j < 6 ? k2 * o.Hi[j] : o.Hi[j]);
      fin = fin && isfinite(h[j]);
    }
    if (!fin) aeff = 0.0f;  // edge-on: every ray misses; never active
    r.r[0] = make_float4(0.0f, (float)o.ox, (float)o.oy, aeff);
    r.r[1] = make_float4(h[0], h[1], h[2], h[3]);
    r.r[2] = make_float4(h[4], h[5], h[6], h[7]);
    r.r[3] = make_float4(h[8], (float)o.color[0], (float)o.color[1], (float)o.color[2]);
    r.r[4] = make_float4((float)o.nrm[0], (float)o.nrm[1], (float)o.nrm[2], 0.0f);
  }
  Record *dst = rec + i;
#pragma unroll
  for (int k = 0; k < 5; ++k) dst->r[k] = r.r[k];
}

// ---------------------------------------------------------------------------
// Backward.  accum[(v*N + g)*16 + k] holds dL/d(record quantity):
//   3D: 0 mx, 1 my, 2 A, 3 B, 4 C, 5 depth z, 9 alpha_eff, 10-12 rgb, 13-15 n
//   2D: 0-8 H (stored, scaled) entries, 9 alpha_eff, 10-12 rgb, 13-15 n
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(128)
preprocess_bwd_kernel(SceneDev sc, const DevCam *__restrict__ cams, int V, DevOpts opt,
                      const uint32_t *__restrict__ tiles, const float *__restrict__ accum,
                      float *g_means, float *g_scales, float *g_rots, float *g_opac,
                      float *g_sh, int accumulate) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= sc.n) return;
  const bool is2d = sc.types[g] == 0;
  const int deg = sc.sh_degree;
  const int K = (deg + 1) * (deg + 1);
  const float m[3] = {sc.means[3 * g], sc.means[3 * g + 1], sc.means[3 * g + 2]};
  const float s[3] = {sc.scales[3 * g], sc.scales[3 * g + 1], sc.scales[3 * g + 2]};
  const float q[4] = {sc.rots[4 * g], sc.rots[4 * g + 1], sc.rots[4 * g + 2], sc.rots[4 * g + 3]};

  double gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gal = 0.0;
  double gsh[48];
  for (int j = 0; j < 3 * K; ++j) gsh[j] = 0.0;
  const double k2 = sqrt(0.5 * kLog2e);

  for (int v = 0; v < V; ++v) {
    const int64_t i = (int64_t)v * sc.n + g;
    if (tiles[i] == 0) continue;
    float a[kGradSlots];
    bool any = false;
    const float4 *ap = reinterpret_cast<const float4 *>(accum + i * kGradSlots);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 t = ap[k];
      a[4 * k] = t.x; a[4 * k + 1] = t.y; a[4 * k + 2] = t.z; a[4 * k + 3] = t.w;
    }
#pragma unroll
    for (int k = 0; k < kGradSlots; ++k) any = any || (a[k] != 0.0f);
    if (!any) continue;
    const DevCam &c = cams[v];
    const Structural st = structural_f32(m, s, q, sc.opac[g], is2d, c, opt.dilation);
    Geo o;
    geo_setup(sc, g, c, opt, st, is2d, o);

    double gpc[3] = {0, 0, 0};   // dL/d p_c
    double gRvR[9];              // dL/d (R_v R)
    for (int j = 0; j < 9; ++j) gRvR[j] = 0.0;
    double gsv[3] = {0, 0, 0};   // dL/d s (this view)

    // normal: n = sign * (R_v R)[:, axis]
    const double sg = st.flip ? -1.0 : 1.0;
    for (int r = 0; r < 3; ++r) gRvR[3 * r + st.axis] += sg * (double)a[13 + r];

    const double X = o.pc[0], Yc = o.pc[1], Z = o.pc[2];
    const double fx = c.fx, fy = c.fy;
    if (!is2d) {
      // conic entries (A, B, C stored = k c00, 2k c01, k c11 with k = log2e/2)
      const double kk = 0.5 * kLog2e;
      const double ga = kk * a[2], gb = 2.0 * kk * a[3], gc = kk * a[4];
      // dL/dSigma' = -Q G Q with G = [[ga, gb/2], [gb/2, gc]]
      const double *Q = o.conic;  // (q00, q01, q11)
      const double G00 = ga, G01 = 0.5 * gb, G11 = gc;
      // QG
      const double t00 = Q[0] * G00 + Q[1] * G01, t01 = Q[0] * G01 + Q[1] * G11;
      const double t10 = Q[1] * G00 + Q[2] * G01, t11 = Q[1] * G01 + Q[2] * G11;
      const double S00 = -(t00 * Q[0] + t01 * Q[1]);
      const double S01 = -(t00 * Q[1] + t01 * Q[2]);
      const double S11 = -(t10 * Q[1] + t11 * Q[2]);
      // Sigma' = A A^T: dL/dA = 2 S A (S symmetric)
      double gA[6];
      for (int j = 0; j < 3; ++j) {
        gA[j] = 2.0 * (S00 * o.A[j] + S01 * o.A[3 + j]);
        gA[3 + j] = 2.0 * (S01 * o.A[j] + S11 * o.A[3 + j]);
      }
      // A = J Cm with Cm = R_v R S (3x3), J = [[J00,0,J02],[0,J11,J12]]
      const double J00 = fx / Z, J02 = -fx * X / (Z * Z), J11 = fy / Z, J12 = -fy * Yc / (Z * Z);
      double gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
      for (int j = 0; j < 3; ++j) {
        const double c0 = o.RvR[j] * o.s[j], c1 = o.RvR[3 + j] * o.s[j], c2 = o.RvR[6 + j] * o.s[j];
        gJ00 += gA[j] * c0;
        gJ02 += gA[j] * c2;
        gJ11 += gA[3 + j] * c1;
        gJ12 += gA[3 + j] * c2;
        const double gc0 = gA[j] * J00, gc1 = gA[3 + j] * J11, gc2 = gA[j] * J02 + gA[3 + j] * J12;
        // Cm[:, j] = RvR[:, j] * s_j
        gRvR[j] += gc0 * o.s[j];
        gRvR[3 + j] += gc1 * o.s[j];
        gRvR[6 + j] += gc2 * o.s[j];
        gsv[j] += gc0 * o.RvR[j] + gc1 * o.RvR[3 + j] + gc2 * o.RvR[6 + j];
      }
      const double iz = 1.0 / Z, iz2 = iz * iz, iz3 = iz2 * iz;
      gpc[0] += gJ02 * (-fx * iz2);
      gpc[1] += gJ12 * (-fy * iz2);
      gpc[2] += gJ00 * (-fx * iz2) + gJ02 * (2.0 * fx * X * iz3) + gJ11 * (-fy * iz2) +
                gJ12 * (2.0 * fy * Yc * iz3);
      // projected centre
      const double gmx = a[0], gmy = a[1];
      gpc[0] += gmx * fx * iz;
      gpc[1] += gmy * fy * iz;
      gpc[2] += -gmx * fx * X * iz2 - gmy * fy * Yc * iz2;
      // depth = z
      gpc[2] += a[5];
      gal += (double)a[9];
    } else {
      // stored h = D Hi (rows 0, 1 scaled by k2); Hi = M^{-1}
      double gH[9];
      for (int j = 0; j < 9; ++j) gH[j] = (double)a[j] * (j < 6 ? k2 : 1.0);
      // dL/dM = -Hi^T gH Hi^T
      double T1[9];  // Hi^T gH
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc)
          T1[3 * r + cc] = o.Hi[r] * gH[cc] + o.Hi[3 + r] * gH[3 + cc] + o.Hi[6 + r] * gH[6 + cc];
      double gM[9];
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc)
          gM[3 * r + cc] = -(T1[3 * r] * o.Hi[3 * cc] + T1[3 * r + 1] * o.Hi[3 * cc + 1] +
                             T1[3 * r + 2] * o.Hi[3 * cc + 2]);
      // M = K' Cm, K' = [[fx, 0, cxl], [0, fy, cyl], [0, 0, 1]]: dL/dCm = K'^T gM
      const double cxl = c.cx - o.ox, cyl = c.cy - o.oy;
      double gC[9];
      for (int j = 0; j < 3; ++j) {
        gC[j] = fx * gM[j];
        gC[3 + j] = fy * gM[3 + j];
        gC[6 + j] = cxl * gM[j] + cyl * gM[3 + j] + gM[6 + j];
      }
      // Cm = [s_x RvR[:,0] | s_y RvR[:,1] | p_c]
      for (int r = 0; r < 3; ++r) {
        gRvR[3 * r] += gC[3 * r] * o.s[0];
        gRvR[3 * r + 1] += gC[3 * r + 1] * o.s[1];
        gpc[r] += gC[3 * r + 2];
      }
      gsv[0] += gC[0] * o.RvR[0] + gC[3] * o.RvR[3] + gC[6] * o.RvR[6];
      gsv[1] += gC[1] * o.RvR[1] + gC[4] * o.RvR[4] + gC[7] * o.RvR[7];
      // opacity: alpha_eff = alpha exp(-lambda sig s_z)
      const double al = sc.opac[g];
      const double ga_eff = (double)a[9];
      gal += ga_eff * (o.alpha_eff / al);
      const double lam = opt.lambda_z;
      const double dsz = o.gate_sig + o.s[2] * o.gate_sig * (1.0 - o.gate_sig) / (double)opt.temp_z;
      gsv[2] += ga_eff * o.alpha_eff * (-lam) * dsz;
    }

    // colour: c_ch = max(0, 1/2 + sum_j f_j,ch Y_j(dir))
    const float *shp = sc.sh + (size_t)g * K * 3;
    double gdir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
      if (o.clamped[ch]) continue;
      const double gcol = (double)a[10 + ch];
      for (int j = 0; j < K; ++j) {
        gsh[3 * j + ch] += gcol * o.Y[j];
        const double f = shp[3 * j + ch];
        gdir[0] += gcol * f * o.dY[j][0];
        gdir[1] += gcol * f * o.dY[j][1];
        gdir[2] += gcol * f * o.dY[j][2];
      }
    }
    // dir = (mu - o) / |mu - o|
    const double dd = o.dir[0] * gdir[0] + o.dir[1] * gdir[1] + o.dir[2] * gdir[2];
    for (int k = 0; k < 3; ++k) gmu[k] += (gdir[k] - o.dir[k] * dd) / o.dist;

    // p_c = V mu + t
    const double *Vd = c.Vd;
    for (int k = 0; k < 3; ++k) gmu[k] += Vd[k] * gpc[0] + Vd[4 + k] * gpc[1] + Vd[8 + k] * gpc[2];
    // RvR = V R: dL/dR = V^T gRvR
    double gR[9];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc)
        gR[3 * r + cc] = Vd[r] * gRvR[cc] + Vd[4 + r] * gRvR[3 + cc] + Vd[8 + r] * gRvR[6 + cc];
    // R(q) for a unit quaternion q = (w, x, y, z)
    const double w = o.q[0], x = o.q[1], y = o.q[2], z = o.q[3];
    const double gw = 2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    const double gx = 2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] +
                             z * gR[6] + w * gR[7] - 2.0 * x * gR[8]);
    const double gy = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] -
                             w * gR[6] + z * gR[7] - 2.0 * y * gR[8]);
    const double gz = 2.0 * (-2.0 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] -
                             2.0 * z * gR[4] + y * gR[5] + x * gR[6] + y * gR[7]);
    const double gqn[4] = {gw, gx, gy, gz};
    // q = r / |r|
    const double dq = gqn[0] * o.q[0] + gqn[1] * o.q[1] + gqn[2] * o.q[2] + gqn[3] * o.q[3];
    for (int k = 0; k < 4; ++k) gq[k] += (gqn[k] - o.q[k] * dq) / o.qn;
    for (int k = 0; k < 3; ++k) gs[k] += gsv[k];
  }

  auto put = [&](float *dst, int64_t idx, double val) {
    if (!dst) return;
    if (accumulate) dst[idx] += (float)val;
    else dst[idx] = (float)val;
  };
  for (int k = 0; k < 3; ++k) put(g_means, 3 * g + k, gmu[k]);
  for (int k = 0; k < 3; ++k) put(g_scales, 3 * g + k, gs[k]);
  for (int k = 0; k < 4; ++k) put(g_rots, 4 * g + k, gq[k]);
  put(g_opac, g, gal);
  for (int j = 0; j < 3 * K; ++j) put(g_sh, (int64_t)g * 3 * K + j, gsh[j]);
}

}  // namespace

void launch_preprocess(const SceneDev &sc, const DevCam *cams, int V, DevOpts opt, Record *rec,
                       uint32_t *tiles, uint32_t *zbits, int4 *rect, hipStream_t s) {
  const int64_t total = (int64_t)V * sc.n;
  if (total == 0) return;
  const int bs = 256;
  const int64_t nb = (total + bs - 1) / bs;
  hipLaunchKernelGGL(preprocess_kernel, dim3((unsigned)nb), dim3(bs), 0, s, sc, cams, V, opt, rec,
                     tiles, zbits, rect);
}

void launch_preprocess_bwd(const SceneDev &sc, const DevCam *cams, int V, DevOpts opt,
                           const uint32_t *tiles, const float *accum, float *g_means,
                           float *g_scales, float *g_rots, float *g_opac, float *g_sh,
                           int accumulate, hipStream_t s) {
  if (sc.n == 0) return;
  const int bs = 128;
  const int64_t nb = (sc.n + bs - 1) / bs;
  hipLaunchKernelGGL(preprocess_bwd_kernel, dim3((unsigned)nb), dim3(bs), 0, s, sc, cams, V, opt,
                     tiles, accum, g_means, g_scales, g_rots, g_opac, g_sh, accumulate);
}

}  // namespace hgs
