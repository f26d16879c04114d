// Frequency-Decoupled Optimization (Sec. 3.3, Alg. 1; appendices on the
// DWT and on gradient conflicts), gfx950.
//
// Cotangents.  The level-1 Haar DWT acts on disjoint 2x2 blocks.  For a
// block [[a, b], [c, d]] of the residual r = I^ - I (rows y, y+1; columns
// x, x+1; zero outside the image, i.e. zero padding of an odd size):
//   LL = (a+b+c+d)/2, LH = (a+b-c-d)/2, HL = (a-b+c-d)/2, HH = (a-b-c+d)/2.
// Every band has n = V * 3 * ceil(H/2) * ceil(W/2) elements, and
//   L_low = sum LL^2 / n,  L_high = sum (LH^2 + HL^2 + HH^2) / n.
// The Haar block map is orthonormal, so its adjoint is its inverse and the
// weighted cotangents on the block's four pixels are
//   grad_low  = lambda_low * LL / n            (the same on all four),
//   grad_high = lambda_high / n * (LH s1 + HL s2 + HH s1 s2)
// with s1 = +1 on row y, -1 on row y+1 and s2 = +1 on column x, -1 on x+1.
// Threads stride over the (view, channel, block) triples, two per
// iteration: 8 bytes read and 8 written per pixel and image, the bytes of a
// copy.
//
// Projection (Alg. 1).  Per primitive i with parameter gradients g_color,
// g_low, g_high (each the concatenation means 3, scales 3, rotations 4,
// opacity 1, SH 3K): d = g_low . g_high in binary64 (products of binary32
// values are exact there, so the sign -- the conflict decision -- is that
// of the exact dot product up to the rounding of a 59-term sum).  If d < 0
// the 2D primitive (type 0) removes from g_high its component along g_low
// (Eq. 9), a 3D one removes from g_low its component along g_high (Eq. 10).
// The update g_color + g_low + g_high is then
//   g_color + (1 - c) g_low + g_high   (2D, c = d / |g_low|^2) or
//   g_color + g_low + (1 - c) g_high   (3D, c = d / |g_high|^2),
// formed in binary64 and rounded once.  Sixteen lanes share a primitive so
// that its gradients are read as contiguous runs (one lane per SH element)
// rather than one 192-byte run per lane.

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kFdoBlock = 1024;

__device__ __forceinline__ void block_add2(double a, double b, double *out) {
  __shared__ double red[2][kFdoBlock / 64];
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
    double x = 0.0, y = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      x += red[0][k];
      y += red[1][k];
    }
    atomicAdd(out, x);
    atomicAdd(out + 1, y);
  }
}

// The residual of one 2x2 block (zero outside the image) and its offset.
struct Block4 {
  float a, b, c, d;
  int64_t o;
  bool x1, y1;
};

__device__ __forceinline__ Block4 load_block(int64_t t, int64_t per, int mw, int H, int W,
                                             int64_t hw, const float *__restrict__ ren,
                                             const float *__restrict__ tgt) {
  Block4 k;
  const int64_t pl = t / per;
  const int rem = (int)(t - pl * per);
  const int bi = rem / mw, bj = rem - bi * mw;
  const int y = 2 * bi, x = 2 * bj;
  k.y1 = y + 1 < H;
  k.x1 = x + 1 < W;
  k.o = pl * hw + (int64_t)y * W + x;
  const int64_t o = k.o;
  k.a = ren[o] - tgt[o];
  k.b = k.x1 ? ren[o + 1] - tgt[o + 1] : 0.0f;
  k.c = k.y1 ? ren[o + W] - tgt[o + W] : 0.0f;
  k.d = (k.x1 && k.y1) ? ren[o + W + 1] - tgt[o + W + 1] : 0.0f;
  return k;
}

__device__ __forceinline__ void store_block(const Block4 &k, int W, float kl, float kh,
                                            float *__restrict__ g_low, float *__restrict__ g_high,
                                            float &sl, float &sh) {
  const float ll = 0.5f * ((k.a + k.b) + (k.c + k.d));
  const float lh = 0.5f * ((k.a + k.b) - (k.c + k.d));
  const float hl = 0.5f * ((k.a - k.b) + (k.c - k.d));
  const float hh = 0.5f * ((k.a - k.b) - (k.c - k.d));
  sl += ll * ll;
  sh += lh * lh + hl * hl + hh * hh;
  const int64_t o = k.o;
  if (g_low) {
    const float v = kl * ll;
    g_low[o] = v;
    if (k.x1) g_low[o + 1] = v;
    if (k.y1) g_low[o + W] = v;
    if (k.x1 && k.y1) g_low[o + W + 1] = v;
  }
  if (g_high) {
    g_high[o] = kh * ((lh + hl) + hh);
    if (k.x1) g_high[o + 1] = kh * ((lh - hl) - hh);
    if (k.y1) g_high[o + W] = kh * ((hl - lh) - hh);
    if (k.x1 && k.y1) g_high[o + W + 1] = kh * (hh - (lh + hl));
  }
}

// Each thread takes two blocks per iteration (loads of both first).
__global__ void __launch_bounds__(kFdoBlock)
fdo_cotangents_kernel(int64_t planes, int H, int W, const float *__restrict__ ren,
                      const float *__restrict__ tgt, float kl, float kh, double inv_n,
                      float *__restrict__ g_low, float *__restrict__ g_high,
                      double *__restrict__ losses) {
  const int mh = (H + 1) >> 1, mw = (W + 1) >> 1;
  const int64_t per = (int64_t)mh * mw;
  const int64_t total = planes * per;
  const int64_t hw = (int64_t)H * W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  float sl = 0.0f, sh = 0.0f;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += 2 * stride) {
    const int64_t t2 = t + stride;
    const Block4 p = load_block(t, per, mw, H, W, hw, ren, tgt);
    Block4 q;
    if (t2 < total) q = load_block(t2, per, mw, H, W, hw, ren, tgt);
    store_block(p, W, kl, kh, g_low, g_high, sl, sh);
    if (t2 < total) store_block(q, W, kl, kh, g_low, g_high, sl, sh);
  }
  if (losses) block_add2((double)sl * inv_n, (double)sh * inv_n, losses);
}

// Parameter-gradient arrays of one set, structure of arrays.
struct GradSet {
  const float *m, *s, *r, *o, *sh;
};

// 16 lanes per primitive: lane j < 11 holds parameter j of (means, scales,
// rotations, opacity) and every lane holds SH elements j, j + 16, j + 32.
// A wave reads four primitives' gradients as contiguous runs, each value
// once, and keeps them in registers for the update.
constexpr int kLanesPerPrim = 16;

__device__ __forceinline__ const float *param_ptr(const GradSet &g, int j, int64_t i) {
  if (j < 3) return g.m ? g.m + 3 * i + j : nullptr;
  if (j < 6) return g.s ? g.s + 3 * i + (j - 3) : nullptr;
  if (j < 10) return g.r ? g.r + 4 * i + (j - 6) : nullptr;
  if (j == 10) return g.o ? g.o + i : nullptr;
  return nullptr;
}

__device__ __forceinline__ float *out_ptr(float *om, float *os, float *orot, float *oo, int j,
                                          int64_t i) {
  if (j < 3) return om ? om + 3 * i + j : nullptr;
  if (j < 6) return os ? os + 3 * i + (j - 3) : nullptr;
  if (j < 10) return orot ? orot + 4 * i + (j - 6) : nullptr;
  if (j == 10) return oo ? oo + i : nullptr;
  return nullptr;
}

__device__ __forceinline__ float ldp(const float *p) { return p ? *p : 0.0f; }

// One primitive's values held by a lane: its parameter slot j (< 11) and
// SH elements j, j + 16, j + 32 of the three sets, and the type.
template <int K>
struct PrimLane {
  static constexpr int kSH = 3 * K;
  static constexpr int kR = (kSH + kLanesPerPrim - 1) / kLanesPerPrim;
  float c0, l0, h0, cs[kR], ls[kR], hs[kR];
  uint8_t t;
  __device__ __forceinline__ void load(const GradSet &gc, const GradSet &gl, const GradSet &gh,
                                       const uint8_t *types, int j, int64_t i) {
    c0 = ldp(param_ptr(gc, j, i));
    l0 = ldp(param_ptr(gl, j, i));
    h0 = ldp(param_ptr(gh, j, i));
    const int64_t base = (int64_t)kSH * i;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int e = j + kLanesPerPrim * r;
      const bool in = e < kSH;
      cs[r] = (in && gc.sh) ? gc.sh[base + e] : 0.0f;
      ls[r] = (in && gl.sh) ? gl.sh[base + e] : 0.0f;
      hs[r] = (in && gh.sh) ? gh.sh[base + e] : 0.0f;
    }
    t = types[i];
  }
  // Alg. 1 for this primitive; returns 1 on the group's first lane if it
  // conflicts.
  __device__ __forceinline__ uint32_t project(int j, int64_t i, float *om, float *os, float *orot,
                                              float *oo, float *osh, int accumulate) const {
    // d = g_low . g_high, |g_low|^2, |g_high|^2 in binary64 over the 16 lanes
    double d = (double)l0 * h0, nl = (double)l0 * l0, nh = (double)h0 * h0;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      d = fma((double)ls[r], (double)hs[r], d);
      nl = fma((double)ls[r], (double)ls[r], nl);
      nh = fma((double)hs[r], (double)hs[r], nh);
    }
#pragma unroll
    for (int o = kLanesPerPrim / 2; o; o >>= 1) {
      d += __shfl_xor(d, o);
      nl += __shfl_xor(nl, o);
      nh += __shfl_xor(nh, o);
    }
    double wl = 1.0, wh = 1.0;
    if (d < 0.0) {
      if (t == 0)
        wl = 1.0 - d / nl;  // Eq. 9: g_high loses its component along g_low
      else
        wh = 1.0 - d / nh;  // Eq. 10: g_low loses its component along g_high
    }
    float *dst = out_ptr(om, os, orot, oo, j, i);
    if (dst) {
      const float v = (float)((double)c0 + wl * (double)l0 + wh * (double)h0);
      *dst = accumulate ? *dst + v : v;
    }
    if (osh) {
      const int64_t base = (int64_t)kSH * i;
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const int e = j + kLanesPerPrim * r;
        if (e < kSH) {
          const float v = (float)((double)cs[r] + wl * (double)ls[r] + wh * (double)hs[r]);
          osh[base + e] = accumulate ? osh[base + e] + v : v;
        }
      }
    }
    return (d < 0.0 && j == 0) ? 1u : 0u;
  }
};

// Each 16-lane group takes two primitives per iteration and issues all
// their loads before either reduction.
template <int K>
__global__ void __launch_bounds__(kFdoBlock)
fdo_project_kernel(int64_t n, const uint8_t *__restrict__ types, GradSet gc, GradSet gl,
                   GradSet gh, float *om, float *os, float *orot, float *oo, float *osh,
                   int accumulate, uint32_t *__restrict__ n_conflict) {
  const int j = threadIdx.x & (kLanesPerPrim - 1);
  const int64_t step = (int64_t)gridDim.x * (blockDim.x / kLanesPerPrim);
  uint32_t conflicts = 0;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanesPerPrim; i < n;
       i += 2 * step) {
    const int64_t i2 = i + step;
    PrimLane<K> a, b;
    a.load(gc, gl, gh, types, j, i);
    if (i2 < n) b.load(gc, gl, gh, types, j, i2);
    conflicts += a.project(j, i, om, os, orot, oo, osh, accumulate);
    if (i2 < n) conflicts += b.project(j, i2, om, os, orot, oo, osh, accumulate);
  }
  if (!n_conflict) return;
  __shared__ uint32_t red[kFdoBlock / 64];
  for (int o = 32; o; o >>= 1) conflicts += __shfl_xor(conflicts, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = conflicts;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    if (t) atomicAdd(n_conflict, t);
  }
}

}  // namespace

void launch_fdo_cotangents(int64_t planes, int H, int W, const float *ren, const float *tgt,
                           double lambda_low, double lambda_high, float *g_low, float *g_high,
                           double *losses, int n_cu, hipStream_t s) {
  const int64_t per = (int64_t)((H + 1) / 2) * ((W + 1) / 2);
  const int64_t total = planes * per;
  if (total <= 0) return;
  const double n = (double)total;
  // one block per CU at most: each block ends with two same-address
  // binary64 atomics for the losses, and those serialise
  int64_t grid = (total + 2 * kFdoBlock - 1) / (2 * kFdoBlock);
  if (grid > n_cu) grid = n_cu;
  hipLaunchKernelGGL(fdo_cotangents_kernel, dim3((unsigned)grid), dim3(kFdoBlock), 0, s, planes,
                     H, W, ren, tgt, (float)(lambda_low / n), (float)(lambda_high / n), 1.0 / n,
                     g_low, g_high, losses);
}

void launch_fdo_project(int64_t n, int sh_coeffs, const uint8_t *types, const float *const *gc,
                        const float *const *gl, const float *const *gh, float *const *out,
                        int accumulate, uint32_t *n_conflict, int n_cu, hipStream_t s) {
  if (n <= 0) return;
  const GradSet c{gc[0], gc[1], gc[2], gc[3], gc[4]};
  const GradSet l{gl[0], gl[1], gl[2], gl[3], gl[4]};
  const GradSet h{gh[0], gh[1], gh[2], gh[3], gh[4]};
  const int64_t per_block = 2 * (kFdoBlock / kLanesPerPrim);
  int64_t blocks = (n + per_block - 1) / per_block;
  if (blocks > 2 * (int64_t)n_cu) blocks = 2 * (int64_t)n_cu;
  const dim3 grid((unsigned)blocks);
#define HGS_FDO_PROJ(KK)                                                                  \
  hipLaunchKernelGGL(fdo_project_kernel<KK>, grid, dim3(kFdoBlock), 0, s, n, types, c, l, h, \
                     out[0], out[1], out[2], out[3], out[4], accumulate, n_conflict)
  switch (sh_coeffs) {
    case 1: HGS_FDO_PROJ(1); break;
    case 4: HGS_FDO_PROJ(4); break;
    case 9: HGS_FDO_PROJ(9); break;
    default: HGS_FDO_PROJ(16); break;
  }
#undef HGS_FDO_PROJ
}

}  // namespace hgs
