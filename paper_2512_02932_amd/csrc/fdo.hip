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
// One thread per (view, channel, block): 8 bytes read and 8 written per
// pixel and image, the bytes of a copy.
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
// formed in binary64 and rounded once.

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

__global__ void __launch_bounds__(kFdoBlock)
fdo_cotangents_kernel(int64_t planes, int H, int W, const float *__restrict__ ren,
                      const float *__restrict__ tgt, float kl, float kh, double inv_n,
                      float *__restrict__ g_low, float *__restrict__ g_high,
                      double *__restrict__ losses) {
  const int mh = (H + 1) >> 1, mw = (W + 1) >> 1;
  const int64_t per = (int64_t)mh * mw;
  const int64_t total = planes * per;
  const int64_t hw = (int64_t)H * W;
  float sl = 0.0f, sh = 0.0f;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pl = t / per;
    const int rem = (int)(t - pl * per);
    const int bi = rem / mw, bj = rem - bi * mw;
    const int y = 2 * bi, x = 2 * bj;
    const bool y1 = y + 1 < H, x1 = x + 1 < W;
    const int64_t o = pl * hw + (int64_t)y * W + x;
    const float a = ren[o] - tgt[o];
    const float b = x1 ? ren[o + 1] - tgt[o + 1] : 0.0f;
    const float c = y1 ? ren[o + W] - tgt[o + W] : 0.0f;
    const float d = (x1 && y1) ? ren[o + W + 1] - tgt[o + W + 1] : 0.0f;
    const float ll = 0.5f * ((a + b) + (c + d));
    const float lh = 0.5f * ((a + b) - (c + d));
    const float hl = 0.5f * ((a - b) + (c - d));
    const float hh = 0.5f * ((a - b) - (c - d));
    sl += ll * ll;
    sh += lh * lh + hl * hl + hh * hh;
    if (g_low) {
      const float v = kl * ll;
      g_low[o] = v;
      if (x1) g_low[o + 1] = v;
      if (y1) g_low[o + W] = v;
      if (x1 && y1) g_low[o + W + 1] = v;
    }
    if (g_high) {
      g_high[o] = kh * ((lh + hl) + hh);
      if (x1) g_high[o + 1] = kh * ((lh - hl) - hh);
      if (y1) g_high[o + W] = kh * ((hl - lh) - hh);
      if (x1 && y1) g_high[o + W + 1] = kh * (hh - (lh + hl));
    }
  }
  if (losses) block_add2((double)sl * inv_n, (double)sh * inv_n, losses);
}

// Parameter-gradient arrays of one set, structure of arrays.
struct GradSet {
  const float *m, *s, *r, *o, *sh;
};

__device__ __forceinline__ float ld(const float *p, int64_t i) { return p ? p[i] : 0.0f; }

template <int K>
__global__ void __launch_bounds__(kFdoBlock)
fdo_project_kernel(int64_t n, const uint8_t *__restrict__ types, GradSet gc, GradSet gl,
                   GradSet gh, float *om, float *os, float *orot, float *oo, float *osh,
                   int accumulate, uint32_t *__restrict__ n_conflict) {
  uint32_t conflicts = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    // pass 1: d, |g_low|^2, |g_high|^2
    double d = 0.0, nl = 0.0, nh = 0.0;
    auto acc = [&](const float *pl, const float *ph, int64_t j) {
      const double a = ld(pl, j), b = ld(ph, j);
      d = fma(a, b, d);
      nl = fma(a, a, nl);
      nh = fma(b, b, nh);
    };
#pragma unroll
    for (int k = 0; k < 3; ++k) acc(gl.m, gh.m, 3 * i + k);
#pragma unroll
    for (int k = 0; k < 3; ++k) acc(gl.s, gh.s, 3 * i + k);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc(gl.r, gh.r, 4 * i + k);
    acc(gl.o, gh.o, i);
#pragma unroll 8
    for (int k = 0; k < 3 * K; ++k) acc(gl.sh, gh.sh, (int64_t)3 * K * i + k);
    double wl = 1.0, wh = 1.0;
    if (d < 0.0) {
      ++conflicts;
      if (types[i] == 0)
        wl = 1.0 - d / nl;  // Eq. 9: g_high loses its component along g_low
      else
        wh = 1.0 - d / nh;  // Eq. 10: g_low loses its component along g_high
    }
    // pass 2: the update
    auto put = [&](float *dst, const float *pc, const float *pl, const float *ph, int64_t j) {
      if (!dst) return;
      const double v = (double)ld(pc, j) + wl * (double)ld(pl, j) + wh * (double)ld(ph, j);
      dst[j] = accumulate ? dst[j] + (float)v : (float)v;
    };
#pragma unroll
    for (int k = 0; k < 3; ++k) put(om, gc.m, gl.m, gh.m, 3 * i + k);
#pragma unroll
    for (int k = 0; k < 3; ++k) put(os, gc.s, gl.s, gh.s, 3 * i + k);
#pragma unroll
    for (int k = 0; k < 4; ++k) put(orot, gc.r, gl.r, gh.r, 4 * i + k);
    put(oo, gc.o, gl.o, gh.o, i);
#pragma unroll 8
    for (int k = 0; k < 3 * K; ++k) put(osh, gc.sh, gl.sh, gh.sh, (int64_t)3 * K * i + k);
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
  int64_t grid = (total + kFdoBlock - 1) / kFdoBlock;
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
  int64_t blocks = (n + kFdoBlock - 1) / kFdoBlock;
  if (blocks > n_cu) blocks = n_cu;
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
