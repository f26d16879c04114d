// Adaptive Type Exchange (Sec. 3.2, Eq. 3; appendix "Effective Rank and
// Type Switch"), gfx950, in place.
//
// erank = exp(H), H = -sum_i p_i log p_i, p = q / |q|_1, q = (s_x^2, s_y^2,
// s_z^2), decided in binary64 (0 log 0 = 0; all-zero scales give 0 and never
// switch).  A 3D primitive (type != 0) with erank < theta_e becomes 2D after
// its least significant scale is moved to z: S* = P S P^T and R* = R P^T with
//   P_x (s_x least): S* = diag(s_y, s_z, s_x), R* = R P_x^T
//   P_y (s_y least): S* = diag(s_z, s_x, s_y), R* = R P_y^T
// and nothing moved when s_z is a least (ties: z, then y).  P_x^T is the
// rotation by +120 degrees about (1,1,1)/sqrt(3), quaternion (1,1,1,1)/2,
// and P_y^T the rotation by -120 degrees, (1,-1,-1,-1)/2, so the stored
// quaternion becomes q (x) that quaternion: the same length as q, the same
// rotation as R P^T.  A 2D primitive with erank > theta_e becomes 3D with
// all parameters kept.
//
// The pass is HBM-bound only if the decision is cheap, and a binary64
// log/exp per primitive is not (several hundred lane operations).  So H is
// first evaluated in binary32 on the scales divided by their maximum (no
// overflow, q in [0,1]) and compared with ln theta_e; its error is below
// 1e-5, so a margin of 1e-4 settles every primitive outside the band, and
// the decision is then the binary64 one.  Primitives inside the band, and
// those with zero, subnormal, infinite or NaN scales (the binary32 value is
// then NaN or the scaling overflows), take the binary64 evaluation.
//
// Each thread takes groups of 4 consecutive primitives: 48 bytes of scales
// as three 16-byte loads and 4 type bytes as one word when the arrays are
// aligned for it, and reads a rotation only when it rewrites it.  Blocks of
// 1024 threads stride over the groups, one block per CU at most; the switch
// counts are summed per block and added with one atomic per counter per
// block (same-address device atomics serialise, one per wave costs more
// than the pass).

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kXBlock = 1024;
constexpr float kBand = 1.0e-4f;

__device__ __forceinline__ double erank64(float sx, float sy, float sz) {
  const double q0 = (double)sx * sx, q1 = (double)sy * sy, q2 = (double)sz * sz;
  const double sum = q0 + q1 + q2;
  if (!(sum > 0.0)) return 0.0;
  double h = 0.0;
  const double p0 = q0 / sum, p1 = q1 / sum, p2 = q2 / sum;
  if (p0 > 0.0) h -= p0 * log(p0);
  if (p1 > 0.0) h -= p1 * log(p1);
  if (p2 > 0.0) h -= p2 * log(p2);
  return exp(h);
}

__device__ __forceinline__ float plogp(float p) { return p > 0.0f ? p * __logf(p) : 0.0f; }

// The binary64 outcome of erank < theta (below), erank > theta (above) and
// erank == 0 (zero: all-zero or NaN scales, which never switch).
__device__ __forceinline__ void decide(float sx, float sy, float sz, float lnth, double theta,
                                       bool &below, bool &above, bool &zero) {
  const float ax = fabsf(sx), ay = fabsf(sy), az = fabsf(sz);
  const float m = fmaxf(fmaxf(ax, ay), az);  // fmaxf drops a NaN operand
  const float r = 1.0f / m;
  const float a = ax * r, b = ay * r, c = az * r;
  const float qa = a * a, qb = b * b, qc = c * c;
  const float sum = qa + qb + qc;  // in [1, 3] for finite, normal m; NaN if a scale is
  const float inv = 1.0f / sum;
  const float h = -(plogp(qa * inv) + plogp(qb * inv) + plogp(qc * inv));
  const bool plain = m >= 1.17549435e-38f && m <= 3.40282347e38f && sum >= 0.5f;
  if (plain && h < lnth - kBand) {
    below = true; above = false; zero = false;
  } else if (plain && h > lnth + kBand) {
    below = false; above = true; zero = false;
  } else {  // near the threshold, or zero, subnormal, infinite or NaN scales
    const double e = erank64(sx, sy, sz);
    zero = !(e > 0.0);
    below = e < theta;
    above = e > theta;
  }
}

// Applies the rule to primitive i; returns the new type byte.
__device__ __forceinline__ uint8_t exchange_one(int64_t i, float sx, float sy, float sz, uint8_t t,
                                                float lnth, double theta, float *__restrict__ scales,
                                                float4 *__restrict__ rots, int &c2, int &c3) {
  bool below, above, zero;
  decide(sx, sy, sz, lnth, theta, below, above, zero);
  if (t != 0) {
    if (!(below && !zero)) return t;
    ++c2;
    if (!(sz <= sx && sz <= sy)) {
      const float4 q = rots[i];
      float4 n;
      if (sy <= sx) {  // P_y: (s_z, s_x, s_y), q (x) (1,-1,-1,-1)/2
        scales[3 * i] = sz;
        scales[3 * i + 1] = sx;
        scales[3 * i + 2] = sy;
        n.x = 0.5f * (q.x + q.y + q.z + q.w);
        n.y = 0.5f * (-q.x + q.y - q.z + q.w);
        n.z = 0.5f * (-q.x + q.y + q.z - q.w);
        n.w = 0.5f * (-q.x - q.y + q.z + q.w);
      } else {  // P_x: (s_y, s_z, s_x), q (x) (1,1,1,1)/2
        scales[3 * i] = sy;
        scales[3 * i + 1] = sz;
        scales[3 * i + 2] = sx;
        n.x = 0.5f * (q.x - q.y - q.z - q.w);
        n.y = 0.5f * (q.x + q.y + q.z - q.w);
        n.z = 0.5f * (q.x - q.y + q.z + q.w);
        n.w = 0.5f * (q.x + q.y - q.z + q.w);
      }
      rots[i] = n;
    }
    return 0;
  }
  if (!above) return 0;
  ++c3;
  return 1;
}

template <bool VEC>
__global__ void __launch_bounds__(kXBlock)
type_exchange_kernel(int64_t n, float *__restrict__ scales, float4 *__restrict__ rots,
                     uint8_t *__restrict__ types, float lnth, double theta,
                     uint32_t *__restrict__ counts) {
  int c2 = 0, c3 = 0;
  const int64_t groups = (n + 3) >> 2;
  for (int64_t g = (int64_t)blockIdx.x * kXBlock + threadIdx.x; g < groups;
       g += (int64_t)gridDim.x * kXBlock) {
    const int64_t i0 = g << 2;
    if (VEC && i0 + 4 <= n) {
      const float4 *s4 = reinterpret_cast<const float4 *>(scales + 3 * i0);
      const float4 u = s4[0], v = s4[1], w = s4[2];
      const uint32_t tw = *reinterpret_cast<const uint32_t *>(types + i0);
      uint32_t nw = 0;
      nw |= (uint32_t)exchange_one(i0, u.x, u.y, u.z, (uint8_t)(tw & 0xff), lnth, theta, scales,
                                   rots, c2, c3);
      nw |= (uint32_t)exchange_one(i0 + 1, u.w, v.x, v.y, (uint8_t)((tw >> 8) & 0xff), lnth,
                                   theta, scales, rots, c2, c3) << 8;
      nw |= (uint32_t)exchange_one(i0 + 2, v.z, v.w, w.x, (uint8_t)((tw >> 16) & 0xff), lnth,
                                   theta, scales, rots, c2, c3) << 16;
      nw |= (uint32_t)exchange_one(i0 + 3, w.y, w.z, w.w, (uint8_t)(tw >> 24), lnth, theta,
                                   scales, rots, c2, c3) << 24;
      if (nw != tw) *reinterpret_cast<uint32_t *>(types + i0) = nw;
    } else {
      const int64_t end = i0 + 4 < n ? i0 + 4 : n;
      for (int64_t i = i0; i < end; ++i) {
        const float sx = scales[3 * i], sy = scales[3 * i + 1], sz = scales[3 * i + 2];
        const uint8_t t = types[i];
        const uint8_t nt = exchange_one(i, sx, sy, sz, t, lnth, theta, scales, rots, c2, c3);
        if (nt != t) types[i] = nt;
      }
    }
  }
  if (!counts) return;
  __shared__ int red[2][kXBlock / 64];
  for (int o = 32; o; o >>= 1) {
    c2 += __shfl_xor(c2, o);
    c3 += __shfl_xor(c3, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = c2;
    red[1][threadIdx.x >> 6] = c3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0, b = 0;
    for (int k = 0; k < kXBlock / 64; ++k) {
      a += red[0][k];
      b += red[1][k];
    }
    if (a) atomicAdd(counts, a);
    if (b) atomicAdd(counts + 1, b);
  }
}

}  // namespace

void launch_type_exchange(int64_t n, float *scales, float *rots, uint8_t *types, double theta,
                          uint32_t *counts, int n_cu, hipStream_t s) {
  if (n <= 0) return;
  const float lnth = theta > 0.0 ? (float)std::log(theta) : -INFINITY;
  const int64_t groups = (n + 3) >> 2;
  int64_t grid = (groups + kXBlock - 1) / kXBlock;
  if (grid > n_cu) grid = n_cu;
  const bool vec = (reinterpret_cast<uintptr_t>(scales) & 15u) == 0 &&
                   (reinterpret_cast<uintptr_t>(types) & 3u) == 0;
  if (vec)
    hipLaunchKernelGGL(type_exchange_kernel<true>, dim3((unsigned)grid), dim3(kXBlock), 0, s, n,
                       scales, reinterpret_cast<float4 *>(rots), types, lnth, theta, counts);
  else
    hipLaunchKernelGGL(type_exchange_kernel<false>, dim3((unsigned)grid), dim3(kXBlock), 0, s, n,
                       scales, reinterpret_cast<float4 *>(rots), types, lnth, theta, counts);
}

}  // namespace hgs
