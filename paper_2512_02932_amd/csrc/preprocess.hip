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
                                              float delta, float amin, float rr0) {
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
  if (!(al >= amin)) return o;

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

  const float rr = rr0 + 4.0f * ((al - 1.0f) / (al + 1.0f));

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

  // column k of R, selected without dynamic register indexing
  const float rk0 = k == 0 ? R[0] : (k == 1 ? R[1] : R[2]);
  const float rk1 = k == 0 ? R[3] : (k == 1 ? R[4] : R[5]);
  const float rk2 = k == 0 ? R[6] : (k == 1 ? R[7] : R[8]);
  const float nc0 = (V[0] * rk0 + V[1] * rk1) + V[2] * rk2;
  const float nc1 = (V[4] * rk0 + V[5] * rk1) + V[6] * rk2;
  const float nc2 = (V[8] * rk0 + V[9] * rk1) + V[10] * rk2;
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
// polynomials of the unit direction, and (backward only) their gradient.
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

template <int D>
__device__ __forceinline__ void sh_basis(double x, double y, double z, double *Y) {
  Y[0] = kY0;
  if constexpr (D >= 1) {
    Y[1] = -kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = -kY1 * x;
  }
  if constexpr (D >= 2) {
    Y[4] = kY2a * x * y;
    Y[5] = -kY2a * y * z;
    Y[6] = kY2b * (3.0 * z * z - 1.0);
    Y[7] = -kY2a * x * z;
    Y[8] = kY2c * (x * x - y * y);
  }
  if constexpr (D >= 3) {
    Y[9] = -kY3a * y * (3.0 * x * x - y * y);
    Y[10] = kY3b * x * y * z;
    Y[11] = -kY3c * y * (5.0 * z * z - 1.0);
    Y[12] = kY3d * z * (5.0 * z * z - 3.0);
    Y[13] = -kY3c * x * (5.0 * z * z - 1.0);
    Y[14] = kY3e * z * (x * x - y * y);
    Y[15] = -kY3a * x * (x * x - 3.0 * y * y);
  }
}

// sum_j w_j dY_j/d(x, y, z) for weights w (one per coefficient)
template <int D>
__device__ __forceinline__ void sh_grad_dot(double x, double y, double z, const double *w,
                                            double *g) {
  g[0] = g[1] = g[2] = 0.0;
  if constexpr (D >= 1) {
    g[1] += -kY1 * w[1];
    g[2] += kY1 * w[2];
    g[0] += -kY1 * w[3];
  }
  if constexpr (D >= 2) {
    g[0] += kY2a * y * w[4];
    g[1] += kY2a * x * w[4];
    g[1] += -kY2a * z * w[5];
    g[2] += -kY2a * y * w[5];
    g[2] += 6.0 * kY2b * z * w[6];
    g[0] += -kY2a * z * w[7];
    g[2] += -kY2a * x * w[7];
    g[0] += 2.0 * kY2c * x * w[8];
    g[1] += -2.0 * kY2c * y * w[8];
  }
  if constexpr (D >= 3) {
    g[0] += -kY3a * 6.0 * x * y * w[9];
    g[1] += -kY3a * (3.0 * x * x - 3.0 * y * y) * w[9];
    g[0] += kY3b * y * z * w[10];
    g[1] += kY3b * x * z * w[10];
    g[2] += kY3b * x * y * w[10];
    g[1] += -kY3c * (5.0 * z * z - 1.0) * w[11];
    g[2] += -kY3c * 10.0 * y * z * w[11];
    g[2] += kY3d * (15.0 * z * z - 3.0) * w[12];
    g[0] += -kY3c * (5.0 * z * z - 1.0) * w[13];
    g[2] += -kY3c * 10.0 * x * z * w[13];
    g[0] += kY3e * 2.0 * x * z * w[14];
    g[1] += -kY3e * 2.0 * y * z * w[14];
    g[2] += kY3e * (x * x - y * y) * w[14];
    g[0] += -kY3a * (3.0 * x * x - 3.0 * y * y) * w[15];
    g[1] += kY3a * 6.0 * x * y * w[15];
  }
}

// SH coefficients of one splat, [K][3] floats.
template <int K>
__device__ __forceinline__ void load_sh(const float *__restrict__ sh, int64_t g, float *f) {
  const float *p = sh + (size_t)g * (3 * K);
  if constexpr ((3 * K) % 4 == 0) {
    const float4 *p4 = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int i = 0; i < (3 * K) / 4; ++i) {
      const float4 t = p4[i];
      f[4 * i] = t.x;
      f[4 * i + 1] = t.y;
      f[4 * i + 2] = t.z;
      f[4 * i + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) f[i] = p[i];
  }
}

// SH rows of a block in LDS.  A splat's 3K coefficients are contiguous in
// memory, so a thread reading or writing its own splat's row touches a
// different cache line per lane on every access; the block instead moves
// the rows of its splats [g0, g0 + nb) between memory and LDS with
// consecutive lanes on consecutive 16-byte words, and each thread then works
// on its own row at rows + t * kRow.  kRow pads 3K so that the rows of eight
// consecutive lanes start on different LDS banks for 16-byte accesses (or is
// odd for 4-byte ones).
template <int K>
struct ShRows {
  static constexpr int kN = 3 * K;
  static constexpr int kRow = (kN % 2) ? kN : (kN % 32 == 16 ? kN + 4 : kN);
};

template <int K, int NT>
__device__ __forceinline__ void sh_rows_load(const float *__restrict__ sh, int64_t g0, int nb,
                                             float *rows) {
  constexpr int N = ShRows<K>::kN, R = ShRows<K>::kRow;
  const float *src = sh + g0 * N;
  const int total = nb * N;
  int done = 0;
  if ((((uintptr_t)src) & 15) == 0) {
    const int n4 = total >> 2;
    for (int e4 = threadIdx.x; e4 < n4; e4 += NT) {
      const float4 t = reinterpret_cast<const float4 *>(src)[e4];
      if constexpr (N % 4 == 0) {
        const int r = (4 * e4) / N;
        *reinterpret_cast<float4 *>(rows + r * R + (4 * e4 - r * N)) = t;
      } else {
        const float v[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = 4 * e4 + u;
          const int r = e / N;
          rows[r * R + (e - r * N)] = v[u];
        }
      }
    }
    done = 4 * n4;
  }
  for (int e = done + threadIdx.x; e < total; e += NT) {
    const int r = e / N;
    rows[r * R + (e - r * N)] = src[e];
  }
}

// The rows back to memory (dst = rows, or dst + rows with accumulate).
template <int K, int NT>
__device__ __forceinline__ void sh_rows_store(float *__restrict__ dst_sh, int64_t g0, int nb,
                                              const float *rows, int accumulate) {
  constexpr int N = ShRows<K>::kN, R = ShRows<K>::kRow;
  float *dst = dst_sh + g0 * N;
  const int total = nb * N;
  int done = 0;
  if constexpr (N % 4 == 0) {
    if ((((uintptr_t)dst) & 15) == 0) {
      const int n4 = total >> 2;
      for (int e4 = threadIdx.x; e4 < n4; e4 += NT) {
        const int r = (4 * e4) / N;
        float4 t = *reinterpret_cast<const float4 *>(rows + r * R + (4 * e4 - r * N));
        float4 *d = reinterpret_cast<float4 *>(dst) + e4;
        if (accumulate) {
          const float4 o = *d;
          t.x = o.x + t.x;
          t.y = o.y + t.y;
          t.z = o.z + t.z;
          t.w = o.w + t.w;
        }
        *d = t;
      }
      done = 4 * n4;
    }
  }
  for (int e = done + threadIdx.x; e < total; e += NT) {
    const int r = e / N;
    const float v = rows[r * R + (e - r * N)];
    dst[e] = accumulate ? dst[e] + v : v;
  }
}

// A thread's row into registers.
template <int K>
__device__ __forceinline__ void sh_row_read(const float *row, float *f) {
  constexpr int N = ShRows<K>::kN;
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const float4 t = reinterpret_cast<const float4 *>(row)[i];
      f[4 * i] = t.x;
      f[4 * i + 1] = t.y;
      f[4 * i + 2] = t.z;
      f[4 * i + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) f[i] = row[i];
  }
}

// ---------------------------------------------------------------------------
// Continuous per-(view, splat) quantities, binary64.
// ---------------------------------------------------------------------------
struct Geo {
  double q[4], qn;      // normalised quaternion and |r|
  double s[3];
  double pc[3];         // camera-space centre
  double RvR[9];        // R_v R (row-major)
  double alpha_eff, gate_sig;
  double ox, oy;        // local pixel frame origin: the rectangle's corner
  // 3D
  double A[6];          // 2x3, Sigma' = A A^T + delta I
  double conic[3];
  double mu2[2];
  // 2D
  double Hi[9];         // inverse of the plane -> pixel map in the local frame
};

__device__ __forceinline__ void geo_setup(const float *mf, const float *sf, const float *qf,
                                          float opac, bool is2d, const DevCam &c,
                                          const DevOpts &opt, double ox, double oy, Geo &o) {
  const double mu[3] = {mf[0], mf[1], mf[2]};
  for (int i = 0; i < 3; ++i) o.s[i] = sf[i];
  const double r[4] = {qf[0], qf[1], qf[2], qf[3]};
  o.qn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
  // one binary64 division per divisor, then products (a division is a
  // long dependent sequence on the GPU; the results stay within binary64
  // rounding of the quotients)
  const double iqn = 1.0 / o.qn;
  for (int i = 0; i < 4; ++i) o.q[i] = r[i] * iqn;
  const double w = o.q[0], x = o.q[1], y = o.q[2], z = o.q[3];
  double R[9];
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
  const double *Vd = c.Vd;
  for (int i = 0; i < 3; ++i)
    o.pc[i] = Vd[4 * i] * mu[0] + Vd[4 * i + 1] * mu[1] + Vd[4 * i + 2] * mu[2] + Vd[4 * i + 3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      o.RvR[3 * i + j] = Vd[4 * i] * R[j] + Vd[4 * i + 1] * R[3 + j] + Vd[4 * i + 2] * R[6 + j];

  // opacity; 2D: alpha* = alpha exp(-lambda_z sigmoid((s_z - theta_z)/T_z) s_z)
  const double al = opac;
  if (is2d) {
    const double za = (o.s[2] - (double)opt.theta_z) / (double)opt.temp_z;
    o.gate_sig = za >= 0 ? 1.0 / (1.0 + exp(-za)) : exp(za) / (1.0 + exp(za));
    o.alpha_eff = al * exp(-(double)opt.lambda_z * o.gate_sig * o.s[2]);
  } else {
    o.gate_sig = 0.0;
    o.alpha_eff = al;
  }

  o.ox = ox;
  o.oy = oy;
  const double X = o.pc[0], Yc = o.pc[1], Z = o.pc[2];
  const double fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy;
  if (!is2d) {
    // A = J R_v R S (2x3): Sigma' = A A^T + delta I
    const double iz = 1.0 / Z;
    const double J00 = fx * iz, J02 = -fx * X * (iz * iz), J11 = fy * iz,
                 J12 = -fy * Yc * (iz * iz);
    for (int j = 0; j < 3; ++j) {
      const double c0 = o.RvR[j] * o.s[j], c1 = o.RvR[3 + j] * o.s[j], c2 = o.RvR[6 + j] * o.s[j];
      o.A[j] = J00 * c0 + J02 * c2;
      o.A[3 + j] = J11 * c1 + J12 * c2;
    }
    const double S0 = o.A[0] * o.A[0] + o.A[1] * o.A[1] + o.A[2] * o.A[2] + (double)opt.dilation;
    const double S1 = o.A[0] * o.A[3] + o.A[1] * o.A[4] + o.A[2] * o.A[5];
    const double S2 = o.A[3] * o.A[3] + o.A[4] * o.A[4] + o.A[5] * o.A[5] + (double)opt.dilation;
    const double det = S0 * S2 - S1 * S1;
    const double idet = 1.0 / det;
    o.conic[0] = S2 * idet;
    o.conic[1] = -S1 * idet;
    o.conic[2] = S0 * idet;
    o.mu2[0] = fx * X * iz + cx;
    o.mu2[1] = fy * Yc * iz + cy;
  } else {
    // plane (u, v, 1) -> homogeneous pixel in the local frame:
    // M = K' [s_x t_u | s_y t_v | p_c], K' = K shifted by the frame origin
    const double cxl = cx - ox, cyl = cy - oy;
    double M[9];
    for (int j = 0; j < 3; ++j) {
      const double sj = j < 2 ? o.s[j] : 1.0;
      const double c0 = j < 2 ? sj * o.RvR[j] : o.pc[0];
      const double c1 = j < 2 ? sj * o.RvR[3 + j] : o.pc[1];
      const double c2 = j < 2 ? sj * o.RvR[6 + j] : o.pc[2];
      M[j] = fx * c0 + cxl * c2;
      M[3 + j] = fy * c1 + cyl * c2;
      M[6 + j] = c2;
    }
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

// Unit view direction (camera centre -> mean) and the distance.
__device__ __forceinline__ void view_dir(const float *mf, const DevCam &c, double *dir,
                                         double &dist) {
  double dv[3];
  for (int i = 0; i < 3; ++i) dv[i] = (double)mf[i] - c.o[i];
  dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  const double idist = 1.0 / dist;
  for (int i = 0; i < 3; ++i) dir[i] = dv[i] * idist;
}

__device__ __forceinline__ double col_of(const double *M9, int row, int axis) {
  return axis == 0 ? M9[3 * row] : (axis == 1 ? M9[3 * row + 1] : M9[3 * row + 2]);
}

// flags per (view, splat): bit 0 valid, bit 1 normal negated, bits 2-3 axis
constexpr uint8_t kValid = 1, kFlip = 2;

__device__ __forceinline__ int4 rect_of(const Structural &st) {
  return make_int4(st.px0, st.py0, st.px1, st.py1);
}

// Splat g of scene sc seen by camera c, written as instance i.
template <int DEG>
__device__ __forceinline__ void preprocess_one(const SceneDev &sc, const DevCam &c, int64_t g,
                                               int64_t i, const DevOpts &opt,
                                               Record *__restrict__ rec,
                                               uint32_t *__restrict__ tiles,
                                               uint32_t *__restrict__ zbits,
                                               int4 *__restrict__ rect,
                                               uint8_t *__restrict__ flags,
                                               uint32_t *__restrict__ prect = nullptr) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const bool is2d = sc.types[g] == 0;
  const float m[3] = {sc.means[3 * g], sc.means[3 * g + 1], sc.means[3 * g + 2]};
  const float s[3] = {sc.scales[3 * g], sc.scales[3 * g + 1], sc.scales[3 * g + 2]};
  const float4 q4 = reinterpret_cast<const float4 *>(sc.rots)[g];
  const float q[4] = {q4.x, q4.y, q4.z, q4.w};
  const float al = sc.opac[g];
  const Structural st = structural_f32(m, s, q, al, is2d, c, opt.dilation, opt.alpha_min, opt.rr0);
  tiles[i] = st.valid ? st.tiles : 0u;
  zbits[i] = st.zbits;
  rect[i] = make_int4(st.px0, st.py0, st.px1, st.py1);
  if (prect) {
    const int4 r = rect_of(st);
    prect[i] = !st.valid ? kNoTiles : (tile_rect_packs(r) ? pack_tile_rect(r) : kWideRect);
  }
  flags[i] = (uint8_t)((st.valid ? kValid : 0) | (st.flip ? kFlip : 0) | (st.axis << 2));
  if (!st.valid) return;

  Geo o;
  geo_setup(m, s, q, al, is2d, c, opt, (double)st.px0, (double)st.py0, o);
  double dir[3], dist;
  view_dir(m, c, dir, dist);
  double Y[K];
  sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
  float f[3 * K];
  load_sh<K>(sc.sh, g, f);
  float col[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.5;
#pragma unroll
    for (int j = 0; j < K; ++j) acc += (double)f[3 * j + ch] * Y[j];
    col[ch] = (acc > 0.0 && acc < 3.0e38) ? (float)acc : 0.0f;  // NaN, <= 0: 0
  }
  const double sg = st.flip ? -1.0 : 1.0;
  float nx = (float)(sg * col_of(o.RvR, 0, st.axis)),
        ny = (float)(sg * col_of(o.RvR, 1, st.axis)),
        nz = (float)(sg * col_of(o.RvR, 2, st.axis));
  const double k2 = sqrt(0.5 * kLog2e);
  float aeff = (float)o.alpha_eff;
  // the raster accumulates colour and normal with weight 0 for inactive
  // pairs, so a record's values must be finite; a non-finite one is never
  // active
  if (!(isfinite(nx) && isfinite(ny) && isfinite(nz) && isfinite(aeff))) {
    aeff = 0.0f;
    nx = ny = nz = 0.0f;
  }
  Record r;
  r.r[0] = make_float4((float)st.px0, (float)st.py0, (float)st.px1, (float)st.py1);
  if (!is2d) {
    const float mx = (float)(o.mu2[0] - o.ox), my = (float)(o.mu2[1] - o.oy);
    const float A = (float)(0.5 * kLog2e * o.conic[0]);
    const float B = (float)(kLog2e * o.conic[1]);
    const float C = (float)(0.5 * kLog2e * o.conic[2]);
    if (!(isfinite(mx) && isfinite(my) && isfinite(A) && isfinite(B) && isfinite(C))) aeff = 0.0f;
    r.r[1] = make_float4(mx, my, A, B);
    r.r[2] = make_float4(C, (float)o.pc[2], 0.0f, 0.0f);
    r.r[3] = make_float4(0.0f, col[0], col[1], col[2]);
    r.r[4] = make_float4(nx, ny, nz, aeff);
  } else {
    float h[9];
    bool fin = true;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      h[j] = (float)(j < 6 ? k2 * o.Hi[j] : o.Hi[j]);
      fin = fin && isfinite(h[j]);
    }
    if (!fin) aeff = 0.0f;  // edge-on: every ray misses; never active
    r.r[1] = make_float4(h[0], h[1], h[2], h[3]);
    r.r[2] = make_float4(h[4], h[5], h[6], h[7]);
    r.r[3] = make_float4(h[8], col[0], col[1], col[2]);
    r.r[4] = make_float4(nx, ny, nz, -aeff);  // negative sign marks a surfel
  }
  Record *dst = rec + i;
#pragma unroll
  for (int k = 0; k < 5; ++k) dst->r[k] = r.r[k];
}

// V views of one scene: instance i = v * N + g.
template <int DEG>
__global__ void __launch_bounds__(256)
preprocess_kernel(SceneDev sc, const DevCam *__restrict__ cams, int V, DevOpts opt,
                  Record *__restrict__ rec, uint32_t *__restrict__ tiles,
                  uint32_t *__restrict__ zbits, int4 *__restrict__ rect,
                  uint8_t *__restrict__ flags, uint32_t *__restrict__ prect) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)V * sc.n;
  if (i >= total) return;
  const int v = (int)(i / sc.n);
  const int64_t g = i - (int64_t)v * sc.n;
  preprocess_one<DEG>(sc, cams[v], g, i, opt, rec, tiles, zbits, rect, flags, prect);
}

// A batch of requests (scene, camera): instance i < *n_inst belongs to the
// slot whose range [inst_base, inst_base + scene.n) holds it.
__global__ void __launch_bounds__(256)
preprocess_slots_kernel(const Slot *__restrict__ slots, const int *__restrict__ n_slots,
                        const uint64_t *__restrict__ n_inst, DevOpts opt, int64_t inst_cap,
                        Record *__restrict__ rec, uint32_t *__restrict__ tiles,
                        uint32_t *__restrict__ zbits, int4 *__restrict__ rect,
                        uint8_t *__restrict__ flags, uint32_t *__restrict__ prect) {
  const int ns = *n_slots;
  const uint64_t cnt = *n_inst < (uint64_t)inst_cap ? *n_inst : (uint64_t)inst_cap;
  if (ns <= 0) return;
  // grid-stride: the grid is sized for a typical batch, not the capacity
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; (uint64_t)i < cnt;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Slot &sl = slots[slot_of_instance(slots, ns, i)];
    const int64_t g = i - sl.inst_base;
    switch (sl.scene.sh_degree) {
      case 0: preprocess_one<0>(sl.scene, sl.cam, g, i, opt, rec, tiles, zbits, rect, flags, prect); break;
      case 1: preprocess_one<1>(sl.scene, sl.cam, g, i, opt, rec, tiles, zbits, rect, flags, prect); break;
      case 2: preprocess_one<2>(sl.scene, sl.cam, g, i, opt, rec, tiles, zbits, rect, flags, prect); break;
      default: preprocess_one<3>(sl.scene, sl.cam, g, i, opt, rec, tiles, zbits, rect, flags, prect); break;
    }
  }
}

// ---------------------------------------------------------------------------
// Backward.  accum[(v*N + g)*16 + k] holds dL/d(record quantity):
//   3D: 0 mx, 1 my, 2 A, 3 B, 4 C, 5 depth z, 9 alpha_eff, 10-12 rgb, 13-15 n
//   2D: 0-8 H (stored, scaled) entries, 9 alpha_eff, 10-12 rgb, 13-15 n
// ---------------------------------------------------------------------------
// One view's geometric chain: the record slots a -> dL/d mu (through the
// camera-space centre), dL/d s, dL/d q (raw quaternion) and dL/d opacity,
// added to gmu, gs, gq, gal.  Linear in a.
template <typename T>
__device__ __forceinline__ void geo_chain(const Geo &o, const DevCam &c, const DevOpts &opt,
                                          const T (&a)[kGradSlots], uint8_t fl, bool is2d,
                                          float al32, double *gmu, double *gs, double *gq,
                                          double &gal) {
  const double k2 = sqrt(0.5 * kLog2e);
  const int axis = (fl >> 2) & 3;

  double gpc[3] = {0, 0, 0};  // dL/d p_c
  double gRvR[9];             // dL/d (R_v R)
#pragma unroll
  for (int j = 0; j < 9; ++j) gRvR[j] = 0.0;
  double gsv[3] = {0, 0, 0};  // dL/d s (this view)

  // normal: n = sign * (R_v R)[:, axis]
  const double sg = (fl & kFlip) ? -1.0 : 1.0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double gn = sg * (double)a[13 + r];
    gRvR[3 * r] += axis == 0 ? gn : 0.0;
    gRvR[3 * r + 1] += axis == 1 ? gn : 0.0;
    gRvR[3 * r + 2] += axis == 2 ? gn : 0.0;
  }

  const double X = o.pc[0], Yc = o.pc[1], Z = o.pc[2];
  const double fx = c.fx, fy = c.fy;
  if (!is2d) {
    // conic entries (A, B, C stored = k c00, 2k c01, k c11 with k = log2e/2)
    const double kk = 0.5 * kLog2e;
    const double G00 = kk * a[2], G01 = kk * a[3], G11 = kk * a[4];
    // dL/dSigma' = -Q G Q, G = [[G00, G01], [G01, G11]]
    const double *Q = o.conic;
    const double t00 = Q[0] * G00 + Q[1] * G01, t01 = Q[0] * G01 + Q[1] * G11;
    const double t10 = Q[1] * G00 + Q[2] * G01, t11 = Q[1] * G01 + Q[2] * G11;
    const double S00 = -(t00 * Q[0] + t01 * Q[1]);
    const double S01 = -(t00 * Q[1] + t01 * Q[2]);
    const double S11 = -(t10 * Q[1] + t11 * Q[2]);
    const double iz = 1.0 / Z, iz2 = iz * iz, iz3 = iz2 * iz;
    const double J00 = fx * iz, J02 = -fx * X * iz2, J11 = fy * iz, J12 = -fy * Yc * iz2;
    double gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      // Sigma' = A A^T: dL/dA = 2 S A
      const double gA0 = 2.0 * (S00 * o.A[j] + S01 * o.A[3 + j]);
      const double gA1 = 2.0 * (S01 * o.A[j] + S11 * o.A[3 + j]);
      const double c0 = o.RvR[j] * o.s[j], c1 = o.RvR[3 + j] * o.s[j], c2 = o.RvR[6 + j] * o.s[j];
      gJ00 += gA0 * c0;
      gJ02 += gA0 * c2;
      gJ11 += gA1 * c1;
      gJ12 += gA1 * c2;
      const double gc0 = gA0 * J00, gc1 = gA1 * J11, gc2 = gA0 * J02 + gA1 * J12;
      gRvR[j] += gc0 * o.s[j];
      gRvR[3 + j] += gc1 * o.s[j];
      gRvR[6 + j] += gc2 * o.s[j];
      gsv[j] += gc0 * o.RvR[j] + gc1 * o.RvR[3 + j] + gc2 * o.RvR[6 + j];
    }
    const double gmx = a[0], gmy = a[1];
    gpc[0] += gJ02 * (-fx * iz2) + gmx * fx * iz;
    gpc[1] += gJ12 * (-fy * iz2) + gmy * fy * iz;
    gpc[2] += gJ00 * (-fx * iz2) + gJ02 * (2.0 * fx * X * iz3) + gJ11 * (-fy * iz2) +
              gJ12 * (2.0 * fy * Yc * iz3) - gmx * fx * X * iz2 - gmy * fy * Yc * iz2 +
              (double)a[5];
    gal += (double)a[9];
  } else {
    // stored h = D Hi (rows 0, 1 scaled by k2); Hi = M^{-1}; dL/dM = -Hi^T gH Hi^T
    double gH[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) gH[j] = (double)a[j] * (j < 6 ? k2 : 1.0);
    double T1[9];  // Hi^T gH
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        T1[3 * r + cc] = o.Hi[r] * gH[cc] + o.Hi[3 + r] * gH[3 + cc] + o.Hi[6 + r] * gH[6 + cc];
    // M = K' Cm: dL/dCm = K'^T gM with gM = -T1 Hi^T
    const double cxl = c.cx - o.ox, cyl = c.cy - o.oy;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double gM0 = -(T1[0] * o.Hi[3 * j] + T1[1] * o.Hi[3 * j + 1] + T1[2] * o.Hi[3 * j + 2]);
      const double gM1 = -(T1[3] * o.Hi[3 * j] + T1[4] * o.Hi[3 * j + 1] + T1[5] * o.Hi[3 * j + 2]);
      const double gM2 = -(T1[6] * o.Hi[3 * j] + T1[7] * o.Hi[3 * j + 1] + T1[8] * o.Hi[3 * j + 2]);
      const double gC0 = fx * gM0, gC1 = fy * gM1;
      const double gC2 = cxl * gM0 + cyl * gM1 + gM2;
      if (j < 2) {  // Cm[:, j] = s_j (R_v R)[:, j]
        gRvR[j] += gC0 * o.s[j];
        gRvR[3 + j] += gC1 * o.s[j];
        gRvR[6 + j] += gC2 * o.s[j];
        gsv[j] += gC0 * o.RvR[j] + gC1 * o.RvR[3 + j] + gC2 * o.RvR[6 + j];
      } else {  // Cm[:, 2] = p_c
        gpc[0] += gC0;
        gpc[1] += gC1;
        gpc[2] += gC2;
      }
    }
    const double ga_eff = (double)a[9];
    gal += ga_eff * (o.alpha_eff / (double)al32);
    const double dsz =
        o.gate_sig + o.s[2] * o.gate_sig * (1.0 - o.gate_sig) / (double)opt.temp_z;
    gsv[2] += ga_eff * o.alpha_eff * (-(double)opt.lambda_z) * dsz;
  }

  // p_c = V mu + t
  const double *Vd = c.Vd;
#pragma unroll
  for (int k = 0; k < 3; ++k) gmu[k] += Vd[k] * gpc[0] + Vd[4 + k] * gpc[1] + Vd[8 + k] * gpc[2];
  // RvR = V R: dL/dR = V^T gRvR
  double gR[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      gR[3 * r + cc] = Vd[r] * gRvR[cc] + Vd[4 + r] * gRvR[3 + cc] + Vd[8 + r] * gRvR[6 + cc];
  // R(q) for a unit quaternion q = (w, x, y, z)
  const double w = o.q[0], x = o.q[1], y = o.q[2], z = o.q[3];
  const double gqn[4] = {
      2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]),
      2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] + z * gR[6] +
             w * gR[7] - 2.0 * x * gR[8]),
      2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
             z * gR[7] - 2.0 * y * gR[8]),
      2.0 * (-2.0 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * z * gR[4] +
             y * gR[5] + x * gR[6] + y * gR[7])};
  // q = r / |r|
  const double dq = gqn[0] * o.q[0] + gqn[1] * o.q[1] + gqn[2] * o.q[2] + gqn[3] * o.q[3];
  const double iqn = 1.0 / o.qn;
#pragma unroll
  for (int k = 0; k < 4; ++k) gq[k] += (gqn[k] - o.q[k] * dq) * iqn;
#pragma unroll
  for (int k = 0; k < 3; ++k) gs[k] += gsv[k];
}

// Channels whose colour 1/2 + sum_j f_j,ch Y_j is not clamped at zero.
template <int K>
__device__ __forceinline__ void colour_live(const float *f, const double *Y, bool (&live)[3]) {
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.5;
#pragma unroll
    for (int j = 0; j < K; ++j) acc += (double)f[3 * j + ch] * Y[j];
    live[ch] = acc > 0.0;
  }
}

// One view's colour chain: dL/dc -> gy (dL/dc where unclamped; dL/d f_j,ch
// is gy_ch Y_j) and dL/d mu through the view direction, added to gmu.
// Linear in gcol.
template <int DEG, typename T>
__device__ __forceinline__ void colour_chain(const float *f, const double *Y, const double *dir,
                                             double dist, const bool (&live)[3],
                                             const T (&gcol)[3], T (&gy)[3], double *gmu) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  double wj[K];
#pragma unroll
  for (int j = 0; j < K; ++j) wj[j] = 0.0;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    gy[ch] = live[ch] ? gcol[ch] : T(0);
    if (!live[ch]) continue;
#pragma unroll
    for (int j = 0; j < K; ++j) wj[j] += (double)gcol[ch] * (double)f[3 * j + ch];
  }
  double gdir[3];
  sh_grad_dot<DEG>(dir[0], dir[1], dir[2], wj, gdir);
  // dir = (mu - o) / |mu - o|
  const double dd = dir[0] * gdir[0] + dir[1] * gdir[1] + dir[2] * gdir[2];
  const double idist = 1.0 / dist;
#pragma unroll
  for (int k = 0; k < 3; ++k) gmu[k] += (gdir[k] - dir[k] * dd) * idist;
}

// Modes of the kernel:
//   kBwdPlain  one slot plane -> gradients;
//   kBwdFdo    FDO with one view: the colour, low and high planes at accum,
//              accum + plane, accum + 2 plane.  The thread first forms its
//              primitive's Alg. 1 weights (w_low, w_high) from g_low and
//              g_high (fdo_weights), then runs the chain once on the slots
//              c + w_low l + w_high h: the chain is linear in the slots, so
//              that is the update g_c + w_l g_l + w_h g_h.
constexpr int kBwdPlain = 0, kBwdFdo = 1;

// One plane's 16 slots of (view, splat) i.
__device__ __forceinline__ void load_plane(const float *__restrict__ p, int64_t i,
                                           float (&a)[kGradSlots]) {
  const float4 *p0 = reinterpret_cast<const float4 *>(p + i * kGradSlots);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float4 t = p0[k];
    a[4 * k] = t.x;
    a[4 * k + 1] = t.y;
    a[4 * k + 2] = t.z;
    a[4 * k + 3] = t.w;
  }
}

// The slots the chain takes: one plane (plain), or the FDO planes combined
// in binary64 with the weights w.
template <int MODE, typename T>
__device__ __forceinline__ void load_slots(const float *__restrict__ accum, int64_t plane,
                                           int64_t i, double2 w, T (&a)[kGradSlots]) {
  float c[kGradSlots];
  load_plane(accum, i, c);
#pragma unroll
  for (int k = 0; k < kGradSlots; ++k) a[k] = c[k];
  if constexpr (MODE == kBwdFdo) {
    const float4 *p1 = reinterpret_cast<const float4 *>(accum + plane + i * kGradSlots);
    const float4 *p2 = reinterpret_cast<const float4 *>(accum + 2 * plane + i * kGradSlots);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 u = p1[k], v = p2[k];
      a[4 * k] += w.x * (double)u.x + w.y * (double)v.x;
      a[4 * k + 1] += w.x * (double)u.y + w.y * (double)v.y;
      a[4 * k + 2] += w.x * (double)u.z + w.y * (double)v.z;
      a[4 * k + 3] += w.x * (double)u.w + w.y * (double)v.w;
    }
  }
}

// Alg. 1's weights for a primitive seen in one view, from the low and high
// slot planes (accum + plane, accum + 2 plane).  g_low and g_high are formed
// as the plain backward forms them and rounded to binary32 as stored
// gradients are; d = g_low . g_high, |g_low|^2 and |g_high|^2 are summed in
// binary64 over means, scales, rotations, opacity and SH.  If d < 0 a 2D
// primitive (type 0) takes w_low = 1 - d / |g_low|^2 (Eq. 9: g_high loses
// its component along g_low), a 3D one w_high = 1 - d / |g_high|^2 (Eq. 10);
// otherwise both are 1.  Sets w = (w_low, w_high); returns d < 0.
template <int DEG>
__device__ __forceinline__ bool fdo_weights(const SceneDev &sc, const DevCam *__restrict__ cams,
                                              const DevOpts &opt, const uint8_t *__restrict__ flags,
                                              const int4 *__restrict__ rect,
                                              const float *__restrict__ accum, int64_t plane,
                                              int64_t g, const float *shrow, double2 &w) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  double d = 0.0, nl = 0.0, nh = 0.0;
  const uint8_t fl = flags[g];
  if (fl & kValid) {
    float al[kGradSlots], ah[kGradSlots];
    load_plane(accum + plane, g, al);
    load_plane(accum + 2 * plane, g, ah);
    bool anyl = false, anyh = false;
#pragma unroll
    for (int k = 0; k < kGradSlots; ++k) {
      anyl = anyl || (al[k] != 0.0f);
      anyh = anyh || (ah[k] != 0.0f);
    }
    if (anyl || anyh) {
      const bool is2d = sc.types[g] == 0;
      const float m[3] = {sc.means[3 * g], sc.means[3 * g + 1], sc.means[3 * g + 2]};
      const float s[3] = {sc.scales[3 * g], sc.scales[3 * g + 1], sc.scales[3 * g + 2]};
      const float4 q4 = reinterpret_cast<const float4 *>(sc.rots)[g];
      const float q[4] = {q4.x, q4.y, q4.z, q4.w};
      const float al32 = sc.opac[g];
      const DevCam &c = cams[0];
      double lmu[3] = {0, 0, 0}, ls[3] = {0, 0, 0}, lq[4] = {0, 0, 0, 0}, lo = 0.0;
      double hmu[3] = {0, 0, 0}, hs[3] = {0, 0, 0}, hq[4] = {0, 0, 0, 0}, ho = 0.0;
      {
        const int4 rc = rect[g];
        Geo o;
        geo_setup(m, s, q, al32, is2d, c, opt, (double)rc.x, (double)rc.y, o);
        if (anyl) geo_chain(o, c, opt, al, fl, is2d, al32, lmu, ls, lq, lo);
        if (anyh) geo_chain(o, c, opt, ah, fl, is2d, al32, hmu, hs, hq, ho);
      }
      const float gcl[3] = {al[10], al[11], al[12]}, gch[3] = {ah[10], ah[11], ah[12]};
      const bool coll = gcl[0] != 0.0f || gcl[1] != 0.0f || gcl[2] != 0.0f;
      const bool colh = gch[0] != 0.0f || gch[1] != 0.0f || gch[2] != 0.0f;
      if (coll || colh) {
        double dir[3], dist;
        view_dir(m, c, dir, dist);
        double Y[K];
        sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
        float f[3 * K];
        sh_row_read<K>(shrow, f);
        bool live[3];
        colour_live<K>(f, Y, live);
        float gyl[3] = {0.0f, 0.0f, 0.0f}, gyh[3] = {0.0f, 0.0f, 0.0f};
        if (coll) colour_chain<DEG>(f, Y, dir, dist, live, gcl, gyl, lmu);
        if (colh) colour_chain<DEG>(f, Y, dir, dist, live, gch, gyh, hmu);
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            const double x = (float)((double)gyl[ch] * Y[j]);
            const double y = (float)((double)gyh[ch] * Y[j]);
            d = fma(x, y, d);
            nl = fma(x, x, nl);
            nh = fma(y, y, nh);
          }
      }
      auto dot = [&](double lv, double hv) {
        const double x = (float)lv, y = (float)hv;
        d = fma(x, y, d);
        nl = fma(x, x, nl);
        nh = fma(y, y, nh);
      };
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        dot(lmu[k], hmu[k]);
        dot(ls[k], hs[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) dot(lq[k], hq[k]);
      dot(lo, ho);
    }
  }
  double wl = 1.0, wh = 1.0;
  const bool conflict = d < 0.0;
  if (conflict) {
    if (sc.types[g] == 0)
      wl = 1.0 - d / nl;
    else
      wh = 1.0 - d / nh;
  }
  w = make_double2(wl, wh);
  return conflict;
}

// The chain of splat g; its SH coefficients are read from, and dL/dSH
// written to, its LDS row.
template <int DEG, int MODE>
__device__ __forceinline__ void preprocess_bwd_one(
    const SceneDev &sc, const DevCam *__restrict__ cams, int V, const DevOpts &opt,
    const uint8_t *__restrict__ flags, const int4 *__restrict__ rect,
    const float *__restrict__ accum, int64_t plane, double2 wgt, int64_t g, float *row,
    float *g_means, float *g_scales, float *g_rots, float *g_opac, bool want_sh,
    int accumulate) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  // the combined slots are formed and kept in binary64
  using Slot = typename std::conditional<MODE == kBwdFdo, double, float>::type;
  const bool is2d = sc.types[g] == 0;
  const float m[3] = {sc.means[3 * g], sc.means[3 * g + 1], sc.means[3 * g + 2]};
  const float s[3] = {sc.scales[3 * g], sc.scales[3 * g + 1], sc.scales[3 * g + 2]};
  const float4 q4 = reinterpret_cast<const float4 *>(sc.rots)[g];
  const float q[4] = {q4.x, q4.y, q4.z, q4.w};
  const float al32 = sc.opac[g];

  double gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gal = 0.0;

  // ---- pass 1: geometry (record geometry, opacity, normal) ----
  for (int v = 0; v < V; ++v) {
    const int64_t i = (int64_t)v * sc.n + g;
    const uint8_t fl = flags[i];
    if (!(fl & kValid)) continue;
    Slot a[kGradSlots];
    load_slots<MODE>(accum, plane, i, wgt, a);
    bool any = false;
#pragma unroll
    for (int k = 0; k < kGradSlots; ++k) any = any || (a[k] != 0.0f);
    if (!any) continue;
    const DevCam &c = cams[v];
    const int4 rc = rect[i];
    Geo o;
    geo_setup(m, s, q, al32, is2d, c, opt, (double)rc.x, (double)rc.y, o);
    geo_chain(o, c, opt, a, fl, is2d, al32, gmu, gs, gq, gal);
  }

  auto put = [&](float *dst, int64_t idx, double val) {
    if (!dst) return;
    if (accumulate) dst[idx] += (float)val;
    else dst[idx] = (float)val;
  };
  for (int k = 0; k < 3; ++k) put(g_scales, 3 * g + k, gs[k]);
  if (g_rots) {
    float4 *dst = reinterpret_cast<float4 *>(g_rots) + g;
    float4 val = make_float4((float)gq[0], (float)gq[1], (float)gq[2], (float)gq[3]);
    if (accumulate) {
      const float4 old = *dst;
      val.x += old.x;
      val.y += old.y;
      val.z += old.z;
      val.w += old.w;
    }
    *dst = val;
  }
  put(g_opac, g, gal);

  // ---- pass 2: colour, c_ch = max(0, 1/2 + sum_j f_j,ch Y_j(dir)) ----
  // dL/dSH is summed over the views in the row, in place of the SH values
  float f[3 * K];
  sh_row_read<K>(row, f);
#pragma unroll
  for (int j = 0; j < 3 * K; ++j) row[j] = 0.0f;
  for (int v = 0; v < V; ++v) {
    const int64_t i = (int64_t)v * sc.n + g;
    if (!(flags[i] & kValid)) continue;
    const float *ap = accum + i * kGradSlots;
    Slot gcol[3] = {ap[10], ap[11], ap[12]};
    if constexpr (MODE == kBwdFdo) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch)
        gcol[ch] += wgt.x * (double)ap[plane + 10 + ch] + wgt.y * (double)ap[2 * plane + 10 + ch];
    }
    if (gcol[0] == Slot(0) && gcol[1] == Slot(0) && gcol[2] == Slot(0)) continue;
    double dir[3], dist;
    view_dir(m, cams[v], dir, dist);
    double Y[K];
    sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
    bool live[3];
    colour_live<K>(f, Y, live);
    Slot gy[3];
    colour_chain<DEG>(f, Y, dir, dist, live, gcol, gy, gmu);
    if (want_sh) {
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) row[3 * j + ch] += (float)((double)gy[ch] * Y[j]);
    }
  }
  for (int k = 0; k < 3; ++k) put(g_means, 3 * g + k, gmu[k]);
}


constexpr int kBwdThreads = 128;

template <int DEG, int MODE>
__device__ __forceinline__ void preprocess_bwd_body(
    const SceneDev &sc, const DevCam *__restrict__ cams, int V, const DevOpts &opt,
    const uint8_t *__restrict__ flags, const int4 *__restrict__ rect,
    const float *__restrict__ accum, int64_t plane, uint32_t *__restrict__ n_conflict,
    float *g_means, float *g_scales, float *g_rots,
    float *g_opac, float *g_sh, int accumulate) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ float s_rows[kBwdThreads * ShRows<K>::kRow];
  const int64_t g0 = (int64_t)blockIdx.x * kBwdThreads;
  const int64_t g = g0 + threadIdx.x;
  const int nb = (int)(sc.n - g0 < kBwdThreads ? sc.n - g0 : kBwdThreads);
  sh_rows_load<K, kBwdThreads>(sc.sh, g0, nb, s_rows);
  __syncthreads();
  float *row = s_rows + threadIdx.x * ShRows<K>::kRow;
  double2 wgt = make_double2(0.0, 0.0);
  if constexpr (MODE == kBwdFdo) {
    // conflicts of this block, added once per block
    __shared__ uint32_t blk_conf;
    if (threadIdx.x == 0) blk_conf = 0;
    __syncthreads();
    bool conf = false;
    if (g < sc.n) conf = fdo_weights<DEG>(sc, cams, opt, flags, rect, accum, plane, g, row, wgt);
    const uint64_t m = __ballot(conf);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&blk_conf, (uint32_t)__popcll(m));
    __syncthreads();
    if (threadIdx.x == 0 && blk_conf && n_conflict) atomicAdd(n_conflict, blk_conf);
  }
  if (g < sc.n) preprocess_bwd_one<DEG, MODE>(sc, cams, V, opt, flags, rect, accum, plane, wgt,
                                             g, row, g_means, g_scales, g_rots, g_opac,
                                             g_sh != nullptr, accumulate);
  if (g_sh) {
    __syncthreads();
    sh_rows_store<K, kBwdThreads>(g_sh, g0, nb, s_rows, accumulate);
  }
}

template <int DEG>
__global__ void __launch_bounds__(kBwdThreads)
preprocess_bwd_kernel(SceneDev sc, const DevCam *__restrict__ cams, int V, DevOpts opt,
                      const uint8_t *__restrict__ flags, const int4 *__restrict__ rect,
                      const float *__restrict__ accum, float *g_means, float *g_scales,
                      float *g_rots, float *g_opac, float *g_sh, int accumulate) {
  preprocess_bwd_body<DEG, kBwdPlain>(sc, cams, V, opt, flags, rect, accum, 0, nullptr, g_means,
                                      g_scales, g_rots, g_opac, g_sh, accumulate);
}

template <int DEG>
__global__ void __launch_bounds__(kBwdThreads)
fdo_fused_bwd_kernel(SceneDev sc, const DevCam *__restrict__ cams, DevOpts opt,
                     const uint8_t *__restrict__ flags, const int4 *__restrict__ rect,
                     const float *__restrict__ accum, int64_t plane,
                     uint32_t *__restrict__ n_conflict, float *g_means, float *g_scales,
                     float *g_rots, float *g_opac, float *g_sh, int accumulate) {
  preprocess_bwd_body<DEG, kBwdFdo>(sc, cams, 1, opt, flags, rect, accum, plane, n_conflict,
                                    g_means, g_scales, g_rots, g_opac, g_sh, accumulate);
}
}  // namespace

void launch_preprocess(const SceneDev &sc, const DevCam *cams, int V, DevOpts opt, Record *rec,
                       uint32_t *tiles, uint32_t *zbits, int4 *rect, uint8_t *flags,
                       uint32_t *prect, hipStream_t s) {
  const int64_t total = (int64_t)V * sc.n;
  if (total == 0) return;
  const int bs = 256;
  const dim3 grid((unsigned)((total + bs - 1) / bs));
  switch (sc.sh_degree) {
    case 0: hipLaunchKernelGGL(preprocess_kernel<0>, grid, dim3(bs), 0, s, sc, cams, V, opt, rec, tiles, zbits, rect, flags, prect); break;
    case 1: hipLaunchKernelGGL(preprocess_kernel<1>, grid, dim3(bs), 0, s, sc, cams, V, opt, rec, tiles, zbits, rect, flags, prect); break;
    case 2: hipLaunchKernelGGL(preprocess_kernel<2>, grid, dim3(bs), 0, s, sc, cams, V, opt, rec, tiles, zbits, rect, flags, prect); break;
    default: hipLaunchKernelGGL(preprocess_kernel<3>, grid, dim3(bs), 0, s, sc, cams, V, opt, rec, tiles, zbits, rect, flags, prect); break;
  }
}

void launch_preprocess_slots(const Slot *slots, const int *n_slots, const uint64_t *n_inst,
                             DevOpts opt, int64_t inst_cap, Record *rec, uint32_t *tiles,
                             uint32_t *zbits, int4 *rect, uint8_t *flags, uint32_t *prect,
                             hipStream_t s) {
  if (inst_cap <= 0) return;
  const int64_t blocks = std::min<int64_t>((inst_cap + 255) / 256, 4096);
  hipLaunchKernelGGL(preprocess_slots_kernel, dim3((unsigned)blocks), dim3(256), 0, s, slots,
                     n_slots, n_inst, opt, inst_cap, rec, tiles, zbits, rect, flags, prect);
}

#define HGS_BY_DEGREE(deg, CALL) \
  switch (deg) {                   \
    case 0: CALL(0); break;        \
    case 1: CALL(1); break;        \
    case 2: CALL(2); break;        \
    default: CALL(3); break;       \
  }

void launch_preprocess_bwd(const SceneDev &sc, const DevCam *cams, int V, DevOpts opt,
                           const uint8_t *flags, const int4 *rect, const float *accum,
                           float *g_means, float *g_scales, float *g_rots, float *g_opac,
                           float *g_sh, int accumulate, hipStream_t s) {
  if (sc.n == 0) return;
  const dim3 grid((unsigned)((sc.n + kBwdThreads - 1) / kBwdThreads));
#define HGS_BWD(D)                                                                            \
  hipLaunchKernelGGL(preprocess_bwd_kernel<D>, grid, dim3(kBwdThreads), 0, s, sc, cams, V,    \
                     opt, flags, rect, accum, g_means, g_scales, g_rots, g_opac, g_sh,        \
                     accumulate)
  HGS_BY_DEGREE(sc.sh_degree, HGS_BWD)
#undef HGS_BWD
}

void launch_fdo_fused_bwd(const SceneDev &sc, const DevCam *cams, DevOpts opt,
                          const uint8_t *flags, const int4 *rect, const float *accum,
                          int64_t plane, uint32_t *n_conflict, float *g_means, float *g_scales,
                          float *g_rots, float *g_opac, float *g_sh, int accumulate,
                          hipStream_t s) {
  if (sc.n == 0) return;
  const dim3 grid((unsigned)((sc.n + kBwdThreads - 1) / kBwdThreads));
#define HGS_F(D)                                                                              \
  hipLaunchKernelGGL(fdo_fused_bwd_kernel<D>, grid, dim3(kBwdThreads), 0, s, sc, cams, opt, flags, rect, \
                     accum, plane, n_conflict, g_means, g_scales, g_rots, g_opac, g_sh,         \
                     accumulate)
  HGS_BY_DEGREE(sc.sh_degree, HGS_F)
#undef HGS_F
}
#undef HGS_BY_DEGREE

}  // namespace hgs
