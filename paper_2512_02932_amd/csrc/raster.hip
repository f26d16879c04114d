// Per-tile compositing (forward) and its reverse pass (backward), gfx950.
//
// One 256-thread block per 16x16 tile.  The block's four wave64s each own an
// 8x8 quadrant.  The tile's depth-sorted splat list is staged through LDS in
// batches of 256 records, with coalesced loads.  Every lane of a wave
// evaluates the same splat at each step, so the 2D/3D branch is
// wave-uniform.
//
// Forward (Sec. 3.1, Eq. 1-2): d_i is the Mahalanobis distance under the
// projected covariance (3D) or u^2 + v^2 at the ray-splat intersection (2D).
// The contribution is alpha~ = min(0.99, alpha_eff e^{-d/2}).  A pair is
// skipped when alpha~ < 1/255 (false for NaN).  A pixel stops before the
// pair that would take its transmittance below 1e-4.  A block-wide vote ends
// a tile whose pixels are all done.
//
// Backward: each pixel walks its list in reverse from its last blended pair.
// It recovers T_i = T_{i+1} / (1 - alpha~_i) and carries the suffix
// S = alpha~ f + (1 - alpha~) S of the per-pair scalar
// f = <G_rgb, c> + G_depth depth + <G_n, n>.  dL/dalpha~ = T_i (f - S).  The
// 16 per-pair gradients are reduced across the wave and added with one
// vector atomic per wave into per-(view, splat) accumulators.

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr float kLn2 = 0.69314718055994531f;

// Exponent (in units of log2 e) of a pair, fixed operation order so the
// forward and backward kernels reach the same bits.
struct PairEval {
  float e;       // alpha~ = alpha_eff * 2^-e
  float depth;
  float xr, yr;  // pixel sample in the splat's local frame
  float a0, a1;  // 3D: dx, dy;  2D: U, V
  float rw;      // 2D: 1 / W
};

__device__ __forceinline__ PairEval eval_pair(bool is3d, float fxp, float fyp, const float4 &r0,
                                              const float4 &r1, const float4 &r2,
                                              const float4 &r3, const float4 &r4) {
#pragma clang fp contract(off)
  PairEval p;
  p.xr = fxp - r0.y;
  p.yr = fyp - r0.z;
  if (is3d) {
    const float dx = p.xr - r1.x, dy = p.yr - r1.y;
    const float t = __builtin_fmaf(r1.w, dy, r1.z * dx);  // A dx + B dy
    const float u = r2.x * dy;                             // C dy
    p.e = __builtin_fmaf(dx, t, u * dy);
    p.depth = r4.w;
    p.a0 = dx;
    p.a1 = dy;
    p.rw = 1.0f;
  } else {
    const float U = __builtin_fmaf(r1.x, p.xr, __builtin_fmaf(r1.y, p.yr, r1.z));
    const float V = __builtin_fmaf(r1.w, p.xr, __builtin_fmaf(r2.x, p.yr, r2.y));
    const float W = __builtin_fmaf(r2.z, p.xr, __builtin_fmaf(r2.w, p.yr, r3.x));
    const float rw = __builtin_amdgcn_rcpf(W);
    const float u = U * rw, v = V * rw;
    p.e = __builtin_fmaf(u, u, v * v);
    p.depth = rw;
    p.a0 = U;
    p.a1 = V;
    p.rw = rw;
  }
  return p;
}

__device__ __forceinline__ float exp2_neg(float e) { return __builtin_amdgcn_exp2f(-e); }

__global__ void __launch_bounds__(kBlock)
raster_fwd_kernel(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
                  const Record *__restrict__ rec, int W, int H, int tiles_x, int tiles_per_view,
                  DevOpts opt, RasterOut out) {
  __shared__ float4 srec[5][kBlock];
  const int tile = blockIdx.x;
  const int v = tile / tiles_per_view;
  const int t = tile - v * tiles_per_view;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int px = tx * kTile + (w & 1) * 8 + (lane & 7);
  const int py = ty * kTile + (w >> 1) * 8 + (lane >> 3);
  const bool inside = px < W && py < H;
  const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
  const uint2 rg = ranges[tile];

  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, dep = 0.0f, nx = 0.0f, ny = 0.0f, nz = 0.0f;
  uint32_t n = 0, last = 0, wc = 0;
  bool done = !inside;

  for (int64_t b = rg.x; b < (int64_t)rg.y; b += kBlock) {
    if (__syncthreads_and(done ? 1 : 0)) break;
    const int64_t idx = b + tid;
    if (idx < (int64_t)rg.y) {
      const Record *r = rec + vals[idx];
#pragma unroll
      for (int k = 0; k < 5; ++k) srec[k][tid] = r->r[k];
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)kBlock, (int64_t)rg.y - b);
    const uint32_t pos0 = (uint32_t)(b - rg.x);
    for (int j = 0; j < cnt; ++j) {
      if (__ballot(!done) == 0ull) break;
      const float4 r0 = srec[0][j], r1 = srec[1][j], r2 = srec[2][j], r3 = srec[3][j],
                   r4 = srec[4][j];
      const bool is3d = __builtin_amdgcn_readfirstlane(__float_as_int(r0.x)) != 0;
      const PairEval p = eval_pair(is3d, fxp, fyp, r0, r1, r2, r3, r4);
      const float raw = r0.w * exp2_neg(p.e);
      if (!done && raw >= kAlphaMin) {
        const float a = fminf(raw, kAlphaMax);
        const float Tn = T * (1.0f - a);
        if (Tn < kTMin) {
          done = true;
          wc |= 0x80000000u | (is3d ? 0u : 0x40000000u);
        } else {
          const float wg = a * T;
          cr = __builtin_fmaf(wg, r3.y, cr);
          cg = __builtin_fmaf(wg, r3.z, cg);
          cb = __builtin_fmaf(wg, r3.w, cb);
          dep = __builtin_fmaf(wg, p.depth, dep);
          nx = __builtin_fmaf(wg, r4.x, nx);
          ny = __builtin_fmaf(wg, r4.y, ny);
          nz = __builtin_fmaf(wg, r4.z, nz);
          T = Tn;
          ++n;
          wc += is3d ? 1u : (1u << 15);
          last = pos0 + (uint32_t)j + 1u;
        }
      }
    }
    __syncthreads();
  }
  if (!inside) return;
  const int64_t hw = (int64_t)H * W;
  const int64_t pix = (int64_t)py * W + px;
  const int64_t o1 = (int64_t)v * hw + pix;
  const int64_t o3 = (int64_t)v * 3 * hw + pix;
  if (out.rgb) {
    out.rgb[o3] = cr + T * opt.bg[0];
    out.rgb[o3 + hw] = cg + T * opt.bg[1];
    out.rgb[o3 + 2 * hw] = cb + T * opt.bg[2];
  }
  if (out.alpha) out.alpha[o1] = 1.0f - T;
  if (out.depth) out.depth[o1] = dep;
  if (out.normal) {
    out.normal[o3] = nx;
    out.normal[o3 + hw] = ny;
    out.normal[o3 + 2 * hw] = nz;
  }
  if (out.T_final) out.T_final[o1] = T;
  if (out.last) out.last[o1] = last;
  if (out.n_contrib) out.n_contrib[o1] = n;
  if (out.wcount) out.wcount[o1] = wc;
}

// Reduce 16 per-lane values over the wave so that lane L ends with the
// total of value ((L>>5)&1)*8 + ((L>>4)&1)*4 + ((L>>3)&1)*2 + ((L>>2)&1):
// a transposed reduce-scatter (halve the value set at each xor step).
__device__ __forceinline__ float wave_reduce_scatter16(float (&g)[16], int lane) {
  const bool b5 = lane & 32;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float send = b5 ? g[k] : g[k + 8];
    const float keep = b5 ? g[k + 8] : g[k];
    g[k] = keep + __shfl_xor(send, 32);
  }
  const bool b4 = lane & 16;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float send = b4 ? g[k] : g[k + 4];
    const float keep = b4 ? g[k + 4] : g[k];
    g[k] = keep + __shfl_xor(send, 16);
  }
  const bool b3 = lane & 8;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float send = b3 ? g[k] : g[k + 2];
    const float keep = b3 ? g[k + 2] : g[k];
    g[k] = keep + __shfl_xor(send, 8);
  }
  const bool b2 = lane & 4;
  float x = (b2 ? g[1] : g[0]) + __shfl_xor(b2 ? g[0] : g[1], 4);
  x += __shfl_xor(x, 2);
  x += __shfl_xor(x, 1);
  return x;
}

__global__ void __launch_bounds__(kBlock)
raster_bwd_kernel(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
                  const Record *__restrict__ rec, int W, int H, int tiles_x, int tiles_per_view,
                  DevOpts opt, const float *__restrict__ T_final,
                  const uint32_t *__restrict__ last_in, RasterGradIn gin,
                  float *__restrict__ accum) {
  __shared__ float4 srec[5][kBlock];
  __shared__ uint32_t sidx[kBlock];
  __shared__ uint32_t smax[4];
  const int tile = blockIdx.x;
  const int v = tile / tiles_per_view;
  const int t = tile - v * tiles_per_view;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int px = tx * kTile + (w & 1) * 8 + (lane & 7);
  const int py = ty * kTile + (w >> 1) * 8 + (lane >> 3);
  const bool inside = px < W && py < H;
  const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
  const uint2 rg = ranges[tile];

  float T = 1.0f;
  uint32_t L = 0;
  float Gr = 0, Gg = 0, Gb = 0, Ga = 0, Gd = 0, Gnx = 0, Gny = 0, Gnz = 0;
  if (inside) {
    const int64_t hw = (int64_t)H * W;
    const int64_t pix = (int64_t)py * W + px;
    const int64_t o1 = (int64_t)v * hw + pix;
    const int64_t o3 = (int64_t)v * 3 * hw + pix;
    T = T_final[o1];
    L = last_in[o1];
    if (gin.rgb) {
      Gr = gin.rgb[o3];
      Gg = gin.rgb[o3 + hw];
      Gb = gin.rgb[o3 + 2 * hw];
    }
    if (gin.alpha) Ga = gin.alpha[o1];
    if (gin.depth) Gd = gin.depth[o1];
    if (gin.normal) {
      Gnx = gin.normal[o3];
      Gny = gin.normal[o3 + hw];
      Gnz = gin.normal[o3 + 2 * hw];
    }
  }
  // suffix value beyond the last blended pair: background and alpha terms
  float S = Gr * opt.bg[0] + Gg * opt.bg[1] + Gb * opt.bg[2] - Ga;

  uint32_t wmax = L;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) wmax = max(wmax, (uint32_t)__shfl_xor((int)wmax, d));
  if (lane == 0) smax[w] = wmax;
  __syncthreads();
  const uint32_t bmax = max(max(smax[0], smax[1]), max(smax[2], smax[3]));
  const int qsel = lane >> 2;
  const int vidx = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
                   ((lane >> 2) & 1);

  for (int end = (int)bmax; end > 0; end -= kBlock) {
    const int start = end > kBlock ? end - kBlock : 0;
    __syncthreads();
    if (start + tid < end) {
      const uint32_t id = vals[rg.x + start + tid];
      sidx[tid] = id;
      const Record *r = rec + id;
#pragma unroll
      for (int k = 0; k < 5; ++k) srec[k][tid] = r->r[k];
    }
    __syncthreads();
    for (int j = end - 1; j >= start; --j) {
      if ((uint32_t)j >= wmax) continue;
      const int slot = j - start;
      const float4 r0 = srec[0][slot], r1 = srec[1][slot], r2 = srec[2][slot],
                   r3 = srec[3][slot], r4 = srec[4][slot];
      const bool is3d = __builtin_amdgcn_readfirstlane(__float_as_int(r0.x)) != 0;
      const PairEval p = eval_pair(is3d, fxp, fyp, r0, r1, r2, r3, r4);
      const float G = exp2_neg(p.e);
      const float raw = r0.w * G;
      const bool act = ((uint32_t)j < L) && (raw >= kAlphaMin);
      if (__ballot(act) == 0ull) continue;
      float g[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) g[k] = 0.0f;
      if (act) {
        const float a = fminf(raw, kAlphaMax);
        const bool clamped = raw > kAlphaMax;
        const float Ti = T * __builtin_amdgcn_rcpf(1.0f - a);
        const float f = Gr * r3.y + Gg * r3.z + Gb * r3.w + Gd * p.depth + Gnx * r4.x +
                        Gny * r4.y + Gnz * r4.z;
        const float dfa = f - S;
        const float ga = Ti * dfa;  // dL/d alpha~
        S = __builtin_fmaf(a, dfa, S);
        const float wg = a * Ti;
        T = Ti;
        g[10] = wg * Gr;
        g[11] = wg * Gg;
        g[12] = wg * Gb;
        g[13] = wg * Gnx;
        g[14] = wg * Gny;
        g[15] = wg * Gnz;
        const float ge = clamped ? 0.0f : -ga * a * kLn2;  // dL/de
        g[9] = clamped ? 0.0f : ga * G;                    // dL/d alpha_eff
        if (is3d) {
          const float dx = p.a0, dy = p.a1;
          g[0] = -ge * (2.0f * r1.z * dx + r1.w * dy);
          g[1] = -ge * (r1.w * dx + 2.0f * r2.x * dy);
          g[2] = ge * dx * dx;
          g[3] = ge * dx * dy;
          g[4] = ge * dy * dy;
          g[5] = wg * Gd;
        } else {
          const float rw = p.rw;
          const float rw2 = rw * rw;
          const float gU = ge * 2.0f * p.a0 * rw2;
          const float gV = ge * 2.0f * p.a1 * rw2;
          const float gW = -2.0f * ge * p.e * rw - wg * Gd * rw2;
          g[0] = gU * p.xr;
          g[1] = gU * p.yr;
          g[2] = gU;
          g[3] = gV * p.xr;
          g[4] = gV * p.yr;
          g[5] = gV;
          g[6] = gW * p.xr;
          g[7] = gW * p.yr;
          g[8] = gW;
        }
      }
      const float tot = wave_reduce_scatter16(g, lane);
      if ((lane & 3) == 0 && tot != 0.0f)
        unsafeAtomicAdd(accum + (size_t)sidx[slot] * kGradSlots + vidx, tot);
      (void)qsel;
    }
  }
}

}  // namespace

void launch_raster_fwd(const uint2 *ranges, const uint32_t *vals, const Record *rec,
                       const DevCam *cams, int V, int n_tiles_total, int W, int H, int tiles_x,
                       int tiles_per_view, DevOpts opt, RasterOut out, hipStream_t s) {
  (void)cams;
  (void)V;
  if (n_tiles_total == 0) return;
  hipLaunchKernelGGL(raster_fwd_kernel, dim3((unsigned)n_tiles_total), dim3(kBlock), 0, s, ranges,
                     vals, rec, W, H, tiles_x, tiles_per_view, opt, out);
}

void launch_raster_bwd(const uint2 *ranges, const uint32_t *vals, const Record *rec,
                       int n_tiles_total, int W, int H, int tiles_x, int tiles_per_view,
                       DevOpts opt, const float *T_final, const uint32_t *last, RasterGradIn g,
                       float *accum, hipStream_t s) {
  if (n_tiles_total == 0) return;
  hipLaunchKernelGGL(raster_bwd_kernel, dim3((unsigned)n_tiles_total), dim3(kBlock), 0, s, ranges,
                     vals, rec, W, H, tiles_x, tiles_per_view, opt, T_final, last, g, accum);
}

}  // namespace hgs
