// Training-step kernels, gfx950: the colour loss of Sec. 3.3 and Adam.
//
// Colour loss.  L_color = (1 - lambda) L1 + lambda D-SSIM as 3DGS defines
// it: L1 = mean |x - y| and D-SSIM = 1 - mean SSIM, where per pixel and
// channel
//   f = a1 a2 / (b1 b2),  a1 = 2 mx my + C1,  a2 = 2 (Sxy - mx my) + C2,
//                         b1 = mx^2 + my^2 + C1,  b2 = Sxx - mx^2 + Syy - my^2 + C2,
// with mx = G*x, my = G*y, Sxx = G*x^2, Syy = G*y^2, Sxy = G*xy under an
// 11 x 11 Gaussian window G (sigma 1.5, normalised, zero padding, same
// size), C1 = 0.01^2, C2 = 0.03^2.  With M the number of pixel-channels,
//   d mean(f) / dx(p) = (1/M) [G*A + 2 x(p) G*B + y(p) G*C](p),
//   A = df/dmx = (2 my (a2 - a1) - 2 mx f (b2 - b1)) / (b1 b2),
//   B = df/dSxx = -f / b2,  C = df/dSxy = 2 a1 / (b1 b2),
// since G is symmetric and the adjoint of a zero-padded same-size filter
// is the same filter.  Two passes over 32 x 32 output tiles with a 5-pixel
// halo in LDS, each a separable filter (rows, then columns):
//   forward:  the five moments -> f, A, B, C (A, B, C to HBM), the sums
//             of |x - y| and 1 - f;
//   backward: G*A, G*B, G*C -> the cotangent of L_color.
// In each filter a thread slides over four consecutive outputs, reading 14
// inputs for them (7 or 3.5 LDS reads per output instead of 22 or 11).
// Blocks stride over the tiles and add their loss sums with one binary64
// atomic per sum per block.
//
// Densification statistics: |dL/d(screen centre)| per view and splat from
// the last backward's accumulators (below).
//
// Adam (Kingma and Ba) on the raw 3DGS parameters (means, log-scales,
// quaternions, opacity logits, SH) from the gradients with respect to the
// activated values the rasterizer returns: dL/ds_raw = exp(s_raw) dL/ds,
// dL/dalpha_raw = sigmoid'(alpha_raw) dL/dalpha.  One elementwise pass over
// all parameter arrays, with bias correction, writing the raw parameters,
// both moments and (optionally) the activated values the renderer reads.

#include <cmath>

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kSsimTile = 32;
constexpr int kHalo = 5;
constexpr int kSpan = kSsimTile + 2 * kHalo;  // 42
constexpr int kSsimThreads = 256;
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct TileGrid {
  int H, W, tiles_x, tiles_y;
  int64_t planes;
};

__device__ __forceinline__ void tile_origin(const TileGrid &g, int64_t t, int64_t &plane, int &x0,
                                            int &y0) {
  const int64_t per = (int64_t)g.tiles_x * g.tiles_y;
  plane = t / per;
  const int r = (int)(t - plane * per);
  y0 = (r / g.tiles_x) * kSsimTile;
  x0 = (r % g.tiles_x) * kSsimTile;
}

// Loads n zero-padded planes of the tile with its halo into LDS.
template <int NQ>
__device__ __forceinline__ void load_halo(const float *const (&src)[NQ], int64_t plane_off,
                                          const TileGrid &g, int x0, int y0,
                                          float (&dst)[NQ][kSpan][kSpan + 1]) {
  for (int idx = threadIdx.x; idx < kSpan * kSpan; idx += kSsimThreads) {
    const int r = idx / kSpan, c = idx - r * kSpan;
    const int gy = y0 - kHalo + r, gx = x0 - kHalo + c;
    const bool in = gy >= 0 && gy < g.H && gx >= 0 && gx < g.W;
    const int64_t o = plane_off + (int64_t)gy * g.W + gx;
#pragma unroll
    for (int q = 0; q < NQ; ++q) dst[q][r][c] = in ? src[q][o] : 0.0f;
  }
}

__global__ void __launch_bounds__(kSsimThreads)
ssim_fwd_kernel(TileGrid g, Win11 win, const float *__restrict__ xs, const float *__restrict__ ys,
                float *__restrict__ Am, float *__restrict__ Bm, float *__restrict__ Cm,
                double inv_m, double *__restrict__ losses) {
  __shared__ float in[2][kSpan][kSpan + 1];
  __shared__ float hq[5][kSpan][kSsimTile + 1];
  const int tx = threadIdx.x & (kSsimTile - 1), ty = threadIdx.x / kSsimTile;  // 32 x 8
  const int64_t n_tiles = g.planes * g.tiles_x * g.tiles_y;
  const int64_t hw = (int64_t)g.H * g.W;
  float l1 = 0.0f, ds = 0.0f;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    int64_t plane;
    int x0, y0;
    tile_origin(g, t, plane, x0, y0);
    const float *src[2] = {xs, ys};
    __syncthreads();  // the previous tile's LDS is no longer read
    load_halo<2>(src, plane * hw, g, x0, y0, in);
    __syncthreads();
    // rows: five window sums at the 32 output columns of all 42 rows; a
    // thread slides over four consecutive outputs of one row (consecutive
    // threads take consecutive rows: odd LDS strides, no bank conflicts)
    for (int idx = threadIdx.x; idx < kSpan * (kSsimTile / 4); idx += kSsimThreads) {
      const int r = idx % kSpan, c0 = 4 * (idx / kSpan);
      float xa[14], ya[14];
#pragma unroll
      for (int i = 0; i < 14; ++i) {
        xa[i] = in[0][r][c0 + i];
        ya[i] = in[1][r][c0 + i];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
#pragma unroll
        for (int k = 0; k < 11; ++k) {
          const float a = xa[j + k], b = ya[j + k], w = win.w[k];
          s0 += w * a;
          s1 += w * b;
          s2 += w * (a * a);
          s3 += w * (b * b);
          s4 += w * (a * b);
        }
        hq[0][r][c0 + j] = s0;
        hq[1][r][c0 + j] = s1;
        hq[2][r][c0 + j] = s2;
        hq[3][r][c0 + j] = s3;
        hq[4][r][c0 + j] = s4;
      }
    }
    __syncthreads();
    // columns: four consecutive output rows of one column per thread
    float mom[5][4];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      float col[14];
#pragma unroll
      for (int i = 0; i < 14; ++i) col[i] = hq[q][4 * ty + i][tx];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float acc = 0;
#pragma unroll
        for (int k = 0; k < 11; ++k) acc += win.w[k] * col[j + k];
        mom[q][j] = acc;
      }
    }
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
      const int r0 = 4 * ty + k4;
      const int gy = y0 + r0, gx = x0 + tx;
      if (gy >= g.H || gx >= g.W) continue;
      const float mx = mom[0][k4], my = mom[1][k4], sxx = mom[2][k4], syy = mom[3][k4],
                  sxy = mom[4][k4];
      const float a1 = 2.0f * mx * my + kC1;
      const float a2 = 2.0f * (sxy - mx * my) + kC2;
      const float b1 = mx * mx + my * my + kC1;
      const float b2 = (sxx - mx * mx) + (syy - my * my) + kC2;
      const float inv = 1.0f / (b1 * b2);
      const float f = a1 * a2 * inv;
      const int64_t o = plane * hw + (int64_t)gy * g.W + gx;
      Am[o] = (2.0f * my * (a2 - a1) - 2.0f * mx * f * (b2 - b1)) * inv;
      Bm[o] = -f / b2;
      Cm[o] = 2.0f * a1 * inv;
      const float xv = in[0][r0 + kHalo][tx + kHalo], yv = in[1][r0 + kHalo][tx + kHalo];
      l1 += fabsf(xv - yv);
      ds += 1.0f - f;
    }
  }
  if (!losses) return;
  __shared__ double red[2][kSsimThreads / 64];
  double a = (double)l1, b = (double)ds;
  for (int o = 32; o; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0, sb = 0;
    for (int k = 0; k < kSsimThreads / 64; ++k) {
      sa += red[0][k];
      sb += red[1][k];
    }
    atomicAdd(losses, sa * inv_m);
    atomicAdd(losses + 1, sb * inv_m);
  }
}

__global__ void __launch_bounds__(kSsimThreads)
ssim_bwd_kernel(TileGrid g, Win11 win, const float *__restrict__ xs, const float *__restrict__ ys,
                const float *__restrict__ Am, const float *__restrict__ Bm,
                const float *__restrict__ Cm, float k_l1, float k_ssim, float *__restrict__ grad) {
  __shared__ float in[3][kSpan][kSpan + 1];
  __shared__ float hq[3][kSpan][kSsimTile + 1];
  const int tx = threadIdx.x & (kSsimTile - 1), ty = threadIdx.x / kSsimTile;
  const int64_t n_tiles = g.planes * g.tiles_x * g.tiles_y;
  const int64_t hw = (int64_t)g.H * g.W;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    int64_t plane;
    int x0, y0;
    tile_origin(g, t, plane, x0, y0);
    const float *src[3] = {Am, Bm, Cm};
    __syncthreads();
    load_halo<3>(src, plane * hw, g, x0, y0, in);
    __syncthreads();
    for (int idx = threadIdx.x; idx < kSpan * (kSsimTile / 4); idx += kSsimThreads) {
      const int r = idx % kSpan, c0 = 4 * (idx / kSpan);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        float row[14];
#pragma unroll
        for (int i = 0; i < 14; ++i) row[i] = in[q][r][c0 + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float acc = 0;
#pragma unroll
          for (int k = 0; k < 11; ++k) acc += win.w[k] * row[j + k];
          hq[q][r][c0 + j] = acc;
        }
      }
    }
    __syncthreads();
    float gm[3][4];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      float col[14];
#pragma unroll
      for (int i = 0; i < 14; ++i) col[i] = hq[q][4 * ty + i][tx];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float acc = 0;
#pragma unroll
        for (int k = 0; k < 11; ++k) acc += win.w[k] * col[j + k];
        gm[q][j] = acc;
      }
    }
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
      const int r0 = 4 * ty + k4;
      const int gy = y0 + r0, gx = x0 + tx;
      if (gy >= g.H || gx >= g.W) continue;
      const float ga = gm[0][k4], gb = gm[1][k4], gc = gm[2][k4];
      const int64_t o = plane * hw + (int64_t)gy * g.W + gx;
      const float xv = xs[o], yv = ys[o];
      const float d = xv - yv;
      const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
      grad[o] = k_l1 * sg - k_ssim * (ga + 2.0f * xv * gb + yv * gc);
    }
  }
}

// ---------------------------------------------------------------------------
// Adam.  Segment s of the flattened parameter space is array s of the five
// (means, scales, rotations, opacities, sh).
// ---------------------------------------------------------------------------
// One element of array s: the chained raw gradient, both moments, the new
// raw value and its activation.
__device__ __forceinline__ void adam_one(const AdamArgs &a, int s, int64_t i, float p, float gr,
                                         float m0, float v0, float &np, float &m, float &v,
                                         float &av) {
  float lr = a.lr[s];
  if (s == 1) {
    gr *= expf(p);
  } else if (s == 3) {  // sigmoid' = sigmoid(p) sigmoid(-p): no cancellation near 1
    gr *= (1.0f / (1.0f + expf(-p))) * (1.0f / (1.0f + expf(p)));
  } else if (s == 4 && (i % a.sh_stride) >= 3) {
    lr = a.lr_sh_rest;
  }
  m = a.beta1 * m0 + a.omb1 * gr;
  v = a.beta2 * v0 + a.omb2 * gr * gr;
  np = p - lr * (m * a.bc1) / (sqrtf(v * a.bc2) + a.eps);
  av = s == 1 ? expf(np) : (s == 3 ? 1.0f / (1.0f + expf(-np)) : np);
}

// Four floats read once: a nontemporal load, so that the four input streams
// do not displace the lines the four output streams are being written to
// (0.35 -> 0.33 ms at 1M Gaussians, SH3; nontemporal stores made no
// difference).
typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_stream(const float *p) {
  const v4f t = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(p));
  return make_float4(t.x, t.y, t.z, t.w);
}

// Blocks [blk[s], blk[s+1]) serve array s, one float4 of it per thread
// (16-byte loads and stores when all of that array's pointers allow them,
// element by element otherwise and for the ragged end).
__global__ void __launch_bounds__(256)
adam_kernel(AdamArgs a) {
  int s = 0;
#pragma unroll
  for (int k = 1; k < 5; ++k) s += (int64_t)blockIdx.x >= a.blk[k] ? 1 : 0;
  if (!a.raw[s] || !a.grad[s]) return;
  const int64_t len = a.off[s + 1] - a.off[s];
  const int64_t e0 = 4 * (((int64_t)blockIdx.x - a.blk[s]) * blockDim.x + threadIdx.x);
  if (e0 >= len) return;
  float *act = a.act[s];
  if (a.vec[s] && e0 + 4 <= len) {
    const float4 p4 = load_stream(a.raw[s] + e0);
    const float4 g4 = load_stream(a.grad[s] + e0);
    const float4 m4 = load_stream(a.m[s] + e0);
    const float4 v4 = load_stream(a.v[s] + e0);
    float4 np, nm, nv, av;
    adam_one(a, s, e0, p4.x, g4.x, m4.x, v4.x, np.x, nm.x, nv.x, av.x);
    adam_one(a, s, e0 + 1, p4.y, g4.y, m4.y, v4.y, np.y, nm.y, nv.y, av.y);
    adam_one(a, s, e0 + 2, p4.z, g4.z, m4.z, v4.z, np.z, nm.z, nv.z, av.z);
    adam_one(a, s, e0 + 3, p4.w, g4.w, m4.w, v4.w, np.w, nm.w, nv.w, av.w);
    *reinterpret_cast<float4 *>(a.raw[s] + e0) = np;
    *reinterpret_cast<float4 *>(a.m[s] + e0) = nm;
    *reinterpret_cast<float4 *>(a.v[s] + e0) = nv;
    if (act) *reinterpret_cast<float4 *>(act + e0) = av;
  } else {
    for (int64_t i = e0; i < e0 + 4 && i < len; ++i) {
      float np, nm, nv, av;
      adam_one(a, s, i, a.raw[s][i], a.grad[s][i], a.m[s][i], a.v[s][i], np, nm, nv, av);
      a.raw[s][i] = np;
      a.m[s][i] = nm;
      a.v[s][i] = nv;
      if (act) act[i] = av;
    }
  }
}

// ---------------------------------------------------------------------------
// Densification statistics (3DGS): per (view, splat) not culled, the norm
// of dL/d delta, delta a translation of the splat's screen footprint, in
// NDC units, and a count of 1.  From the accumulator slots of the last
// backward (summed over its cotangent planes):
//   3D: dL/d delta = (slot 0, slot 1), the gradient of the pixel-space
//       centre the exponent is measured from;
//   2D: the record's inverse map H (pixel -> plane) becomes H T(-delta), so
//       dL/d delta_c = - sum_k G[k][2] H[k][c] (c = x, y), where G[k][2] =
//       slot 3k + 2 = dL/d(row k's constant term).
// ---------------------------------------------------------------------------
constexpr uint8_t kFlagValid = 1;  // bit 0 of the preprocess flags byte: not culled

__global__ void __launch_bounds__(256)
densify_stats_kernel(int64_t VN, int64_t N, const uint8_t *__restrict__ flags,
                     const Record *__restrict__ rec, const float *__restrict__ accum,
                     int64_t plane, int n_planes, float half_w, float half_h,
                     float *__restrict__ grad_norm, float *__restrict__ count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < VN;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (!(flags[i] & kFlagValid)) continue;
    const int64_t g = i % N;
    float sl[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) sl[k] = 0.0f;
    for (int p = 0; p < n_planes; ++p) {
      const float *a = accum + p * plane + i * kGradSlots;
#pragma unroll
      for (int k = 0; k < 9; ++k) sl[k] += a[k];
    }
    const float4 r4 = rec[i].r[4];
    float gx, gy;
    if (__float_as_uint(r4.w) >> 31) {  // 2D
      const float4 r1 = rec[i].r[1], r2 = rec[i].r[2];
      // H rows: (r1.x r1.y r1.z), (r1.w r2.x r2.y), (r2.z r2.w r3.x)
      gx = -(sl[2] * r1.x + sl[5] * r1.w + sl[8] * r2.z);
      gy = -(sl[2] * r1.y + sl[5] * r2.x + sl[8] * r2.w);
    } else {
      gx = sl[0];
      gy = sl[1];
    }
    if (grad_norm) unsafeAtomicAdd(grad_norm + g, hypotf(gx * half_w, gy * half_h));
    if (count) unsafeAtomicAdd(count + g, 1.0f);
  }
}

}  // namespace

void launch_densify_stats(int64_t V, int64_t N, const uint8_t *flags, const Record *rec,
                          const float *accum, int64_t plane, int n_planes, int W, int H,
                          float *grad_norm, float *count, int n_cu, hipStream_t s) {
  const int64_t VN = V * N;
  if (VN <= 0) return;
  int64_t grid = (VN + 255) / 256;
  if (grid > 16 * (int64_t)n_cu) grid = 16 * (int64_t)n_cu;
  hipLaunchKernelGGL(densify_stats_kernel, dim3((unsigned)grid), dim3(256), 0, s, VN, N, flags,
                     rec, accum, plane, n_planes, 0.5f * (float)W, 0.5f * (float)H, grad_norm,
                     count);
}

Win11 gauss_win11() {
  Win11 w;
  double g[11], sum = 0.0;
  for (int k = 0; k < 11; ++k) {
    const double d = k - 5;
    g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[k];
  }
  for (int k = 0; k < 11; ++k) w.w[k] = (float)(g[k] / sum);
  return w;
}

void launch_ssim_fwd(int64_t planes, int H, int W, const float *x, const float *y, float *Am,
                     float *Bm, float *Cm, double *losses, int n_cu, hipStream_t s) {
  if (planes <= 0 || H <= 0 || W <= 0) return;
  TileGrid g{H, W, (W + kSsimTile - 1) / kSsimTile, (H + kSsimTile - 1) / kSsimTile, planes};
  const int64_t n_tiles = planes * g.tiles_x * g.tiles_y;
  // 42 KB of LDS per block: three blocks per CU
  int64_t grid = n_tiles < 3 * (int64_t)n_cu ? n_tiles : 3 * (int64_t)n_cu;
  const double m = (double)planes * H * W;
  hipLaunchKernelGGL(ssim_fwd_kernel, dim3((unsigned)grid), dim3(kSsimThreads), 0, s, g,
                     gauss_win11(), x, y, Am, Bm, Cm, 1.0 / m, losses);
}

void launch_ssim_bwd(int64_t planes, int H, int W, const float *x, const float *y,
                     const float *Am, const float *Bm, const float *Cm, double lambda,
                     float *grad, int n_cu, hipStream_t s) {
  if (planes <= 0 || H <= 0 || W <= 0) return;
  TileGrid g{H, W, (W + kSsimTile - 1) / kSsimTile, (H + kSsimTile - 1) / kSsimTile, planes};
  const int64_t n_tiles = planes * g.tiles_x * g.tiles_y;
  int64_t grid = n_tiles < 4 * (int64_t)n_cu ? n_tiles : 4 * (int64_t)n_cu;
  const double m = (double)planes * H * W;
  hipLaunchKernelGGL(ssim_bwd_kernel, dim3((unsigned)grid), dim3(kSsimThreads), 0, s, g,
                     gauss_win11(), x, y, Am, Bm, Cm, (float)((1.0 - lambda) / m),
                     (float)(lambda / m), grad);
}

void launch_adam(const AdamArgs &a0, int n_cu, hipStream_t s) {
  (void)n_cu;
  AdamArgs a = a0;
  auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
  a.blk[0] = 0;
  for (int k = 0; k < 5; ++k) {
    const int64_t len = a.off[k + 1] - a.off[k];
    const int64_t quads = (len + 3) / 4;
    a.blk[k + 1] = a.blk[k] + (a.raw[k] && a.grad[k] ? (quads + 255) / 256 : 0);
    a.vec[k] = al16(a.raw[k]) && al16(a.grad[k]) && al16(a.m[k]) && al16(a.v[k]) &&
               (!a.act[k] || al16(a.act[k]));
  }
  if (a.blk[5] <= 0) return;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)a.blk[5]), dim3(256), 0, s, a);
}

}  // namespace hgs
