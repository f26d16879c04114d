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
// first evaluated in binary32, in log2 units with the hardware reciprocal
// and log2, on the scales divided by their maximum (no overflow, q in
// [0,1]), and compared with log2 theta_e; its error is a few 1e-7, so a
// margin of 1e-4 (natural units) settles every primitive outside the band,
// and the decision is then the binary64 one.  Primitives inside the band,
// and those with zero, subnormal, infinite or NaN scales, take the binary64
// evaluation.
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
// Margin on H in log2 units (1e-4 in natural units).
constexpr float kBand2 = 1.4427e-4f;

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

// p log2 p with the hardware log2 (about 1 ulp for normal inputs); terms of
// p <= 1e-30 are below 1e-28 and taken as 0, which also keeps subnormal p
// away from the instruction.
__device__ __forceinline__ float plog2p(float p) {
  return p > 1.0e-30f ? p * __builtin_amdgcn_logf(p) : 0.0f;
}

// Binary32 pre-decision: -1 erank < theta, +1 erank > theta, 0 undecided
// (inside the margin, or zero, subnormal, infinite or NaN scales).  With
// the hardware reciprocal and log2 the error of H is a few 1e-7.
__device__ __forceinline__ int quick_side(float sx, float sy, float sz, float l2th) {
  const float ax = fabsf(sx), ay = fabsf(sy), az = fabsf(sz);
  const float m = fmaxf(fmaxf(ax, ay), az);  // fmaxf drops a NaN operand
  const float r = __builtin_amdgcn_rcpf(m);
  const float a = ax * r, b = ay * r, c = az * r;
  const float qa = a * a, qb = b * b, qc = c * c;
  const float sum = qa + qb + qc;  // in [1, 3] for finite, normal m; NaN if a scale is
  const float inv = __builtin_amdgcn_rcpf(sum);
  const float h2 = -(plog2p(qa * inv) + plog2p(qb * inv) + plog2p(qc * inv));
  const bool plain = m >= 1.17549435e-38f && m <= 3.40282347e38f && sum >= 0.5f;
  if (!plain) return 0;
  return h2 < l2th - kBand2 ? -1 : (h2 > l2th + kBand2 ? 1 : 0);
}

// Binary64 decision: the same three-way outcome, and 2 for erank == 0
// (all-zero or NaN scales, which never switch).
__device__ __forceinline__ int exact_side(float sx, float sy, float sz, double theta) {
  const double e = erank64(sx, sy, sz);
  if (!(e > 0.0)) return 2;
  return e < theta ? -1 : (e > theta ? 1 : 0);
}

// New type byte and reparameterisation (0 none, 1 P_x, 2 P_y) from the side.
__device__ __forceinline__ uint8_t rule(int side, uint8_t t, float sx, float sy, float sz, int &mv,
                                        int &c2, int &c3) {
  mv = 0;
  if (t != 0) {
    if (side != -1) return t;
    ++c2;
    if (!(sz <= sx && sz <= sy)) mv = sy <= sx ? 2 : 1;
    return 0;
  }
  if (side != 1) return 0;
  ++c3;
  return 1;
}

// Rewrites the rotation of primitive i and permutes its scales in registers.
__device__ __forceinline__ void reparameterise(int64_t i, int mv, float &sx, float &sy, float &sz,
                                               float4 q, float4 *__restrict__ rots) {
  float4 n;
  const float x = sx, y = sy, z = sz;
  if (mv == 2) {  // P_y: (s_z, s_x, s_y), q (x) (1,-1,-1,-1)/2
    sx = z;
    sy = x;
    sz = y;
    n.x = 0.5f * (q.x + q.y + q.z + q.w);
    n.y = 0.5f * (-q.x + q.y - q.z + q.w);
    n.z = 0.5f * (-q.x + q.y + q.z - q.w);
    n.w = 0.5f * (-q.x - q.y + q.z + q.w);
  } else {  // P_x: (s_y, s_z, s_x), q (x) (1,1,1,1)/2
    sx = y;
    sy = z;
    sz = x;
    n.x = 0.5f * (q.x - q.y - q.z - q.w);
    n.y = 0.5f * (q.x + q.y + q.z - q.w);
    n.z = 0.5f * (q.x - q.y + q.z + q.w);
    n.w = 0.5f * (q.x + q.y - q.z + q.w);
  }
  rots[i] = n;
}

// Up to 4 consecutive primitives i0 .. i0+k-1 whose scales and types are
// in registers: decide all, evaluate the undecided in binary64, then read
// the rotations to rewrite together.  Rotations are stored here; the new
// scales are left in sx, sy, sz (moved = bit j set when primitive j's
// changed) and the new type bytes returned.
__device__ __forceinline__ uint32_t exchange4(int64_t i0, int k, float (&sx)[4], float (&sy)[4],
                                              float (&sz)[4], uint32_t tw, float l2th,
                                              double theta, float4 *__restrict__ rots,
                                              unsigned &moved, int &c2, int &c3) {
  int side[4];
  bool undecided = false;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    side[j] = j < k ? quick_side(sx[j], sy[j], sz[j], l2th) : 1;
    undecided |= j < k && side[j] == 0;
  }
  if (undecided) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < k && side[j] == 0) side[j] = exact_side(sx[j], sy[j], sz[j], theta);
  }
  int mv[4];
  uint32_t nw = 0;
  moved = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint8_t t = (uint8_t)(tw >> (8 * j));
    nw |= (uint32_t)(j < k ? rule(side[j], t, sx[j], sy[j], sz[j], mv[j], c2, c3) : t) << (8 * j);
    if (j >= k) mv[j] = 0;
    moved |= (mv[j] != 0 ? 1u : 0u) << j;
  }
  if (moved) {
    float4 q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      q[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (mv[j]) q[j] = rots[i0 + j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (mv[j]) reparameterise(i0 + j, mv[j], sx[j], sy[j], sz[j], q[j], rots);
  }
  return nw;
}

template <bool VEC>
__global__ void __launch_bounds__(kXBlock)
type_exchange_kernel(int64_t n, float *__restrict__ scales, float4 *__restrict__ rots,
                     uint8_t *__restrict__ types, float l2th, double theta,
                     uint32_t *__restrict__ counts) {
  int c2 = 0, c3 = 0;
  const int64_t groups = (n + 3) >> 2;
  for (int64_t g = (int64_t)blockIdx.x * kXBlock + threadIdx.x; g < groups;
       g += (int64_t)gridDim.x * kXBlock) {
    const int64_t i0 = g << 2;
    float sx[4], sy[4], sz[4];
    if (VEC && i0 + 4 <= n) {
      const float4 *s4 = reinterpret_cast<const float4 *>(scales + 3 * i0);
      const float4 u = s4[0], v = s4[1], w = s4[2];
      const uint32_t tw = *reinterpret_cast<const uint32_t *>(types + i0);
      sx[0] = u.x; sy[0] = u.y; sz[0] = u.z;
      sx[1] = u.w; sy[1] = v.x; sz[1] = v.y;
      sx[2] = v.z; sy[2] = v.w; sz[2] = w.x;
      sx[3] = w.y; sy[3] = w.z; sz[3] = w.w;
      unsigned moved;
      const uint32_t nw = exchange4(i0, 4, sx, sy, sz, tw, l2th, theta, rots, moved, c2, c3);
      if (moved) {  // the group's 48 bytes as three 16-byte stores
        float4 *o4 = reinterpret_cast<float4 *>(scales + 3 * i0);
        o4[0] = make_float4(sx[0], sy[0], sz[0], sx[1]);
        o4[1] = make_float4(sy[1], sz[1], sx[2], sy[2]);
        o4[2] = make_float4(sz[2], sx[3], sy[3], sz[3]);
      }
      if (nw != tw) *reinterpret_cast<uint32_t *>(types + i0) = nw;
    } else {
      const int k = (int)(n - i0 < 4 ? n - i0 : 4);
      uint32_t tw = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        sx[j] = sy[j] = sz[j] = 0.0f;
        if (j < k) {
          sx[j] = scales[3 * (i0 + j)];
          sy[j] = scales[3 * (i0 + j) + 1];
          sz[j] = scales[3 * (i0 + j) + 2];
          tw |= (uint32_t)types[i0 + j] << (8 * j);
        }
      }
      unsigned moved;
      const uint32_t nw = exchange4(i0, k, sx, sy, sz, tw, l2th, theta, rots, moved, c2, c3);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if ((moved >> j) & 1u) {
          scales[3 * (i0 + j)] = sx[j];
          scales[3 * (i0 + j) + 1] = sy[j];
          scales[3 * (i0 + j) + 2] = sz[j];
        }
        if (j < k && ((nw ^ tw) >> (8 * j)) & 0xffu) types[i0 + j] = (uint8_t)(nw >> (8 * j));
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
  const float l2th = theta > 0.0 ? (float)std::log2(theta) : -INFINITY;
  const int64_t groups = (n + 3) >> 2;
  int64_t grid = (groups + kXBlock - 1) / kXBlock;
  if (grid > n_cu) grid = n_cu;
  const bool vec = (reinterpret_cast<uintptr_t>(scales) & 15u) == 0 &&
                   (reinterpret_cast<uintptr_t>(types) & 3u) == 0;
  if (vec)
    hipLaunchKernelGGL(type_exchange_kernel<true>, dim3((unsigned)grid), dim3(kXBlock), 0, s, n,
                       scales, reinterpret_cast<float4 *>(rots), types, l2th, theta, counts);
  else
    hipLaunchKernelGGL(type_exchange_kernel<false>, dim3((unsigned)grid), dim3(kXBlock), 0, s, n,
                       scales, reinterpret_cast<float4 *>(rots), types, l2th, theta, counts);
}

}  // namespace hgs
