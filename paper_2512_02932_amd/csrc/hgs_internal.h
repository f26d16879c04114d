// Internal declarations of the gfx950 hybrid rasterizer (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hgs {

constexpr int kTile = 16;            // 16x16 pixel tiles
constexpr int kBlock = 256;          // one thread per pixel of a tile
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr int kGradSlots = 16;       // per-(view, splat) gradient accumulator

// One view, as the kernels see it.  The float fields are the caller's
// values unchanged: the structural decisions use them bit for bit.
struct DevCam {
  float V[12];          // rows of the 3x4 world->camera matrix
  float fx, fy, cx, cy;
  float znear;
  int32_t W, H;
  int32_t tiles_x, tiles_y;
  int32_t tile_base;    // first global tile id of this view
  int32_t pad[2];
  double Vd[12];        // same matrix in binary64
  double Vinv[9];       // inverse of the 3x3 rotation part
  double o[3];          // camera centre, -R^{-1} t
};

struct DevOpts {
  float bg[3];
  float dilation;
  float lambda_z, theta_z, temp_z;
  float pad;
};

// Per-(view, splat) record read by the raster kernels: five float4, the
// same size for both types so a batch loads uniformly.
//   r0 = (x0, y0, x1, y1)  the splat's inclusive pixel rectangle; (x0, y0) is
//                          also the origin of the splat's local pixel frame
//   r4 = (nx, ny, nz, a)   camera-space normal; |a| = alpha_eff, and the sign
//                          bit of a marks a 2D surfel
//   3D: r1 = (mx, my, A, B), r2 = (C, z, 0, 0), r3 = (0, r, g, b)
//       exponent = A dx^2 + B dx dy + C dy^2, dx = x+1/2-x0-mx,
//       alpha~ = alpha_eff 2^-exponent  (A, B, C = log2(e)/2 * conic, B x2)
//   2D: r1 = (H00, H01, H02, H10), r2 = (H11, H12, H20, H21),
//       r3 = (H22, r, g, b)
//       (U, V, W) = H (x', y', 1), x' = x+1/2-x0; exponent = (U^2+V^2)/W^2,
//       depth = 1/W.  H is the inverse of the surfel's plane-to-pixel map,
//       rows 0 and 1 scaled by sqrt(log2(e)/2).
struct Record {
  float4 r[5];
};

struct SceneDev {
  int64_t n;
  int32_t sh_degree;
  const float *means, *scales, *rots, *opac, *sh;
  const uint8_t *types;
};

// ----- launchers (all enqueue on `s`) -----
// flags per (view, splat): bit 0 valid, bit 1 normal negated, bits 2-3 normal axis
void launch_preprocess(const SceneDev &sc, const DevCam *cams, int V, DevOpts opt,
                       Record *rec, uint32_t *tiles, uint32_t *zbits, int4 *rect,
                       uint8_t *flags, hipStream_t s);
void launch_preprocess_bwd(const SceneDev &sc, const DevCam *cams, int V, DevOpts opt,
                           const uint8_t *flags, const int4 *rect, const float *accum,
                           float *g_means, float *g_scales, float *g_rots, float *g_opac,
                           float *g_sh, int accumulate, hipStream_t s);

// Exclusive scan of n uint32 values; writes the 64-bit total to *total
// (device).  `tmp` must hold scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
void launch_scan(const uint32_t *in, uint32_t *out, int64_t n, uint64_t *total, void *tmp,
                 hipStream_t s);

void launch_duplicate(const uint32_t *offsets, const uint32_t *tiles, const int4 *rect,
                      const uint32_t *zbits, const DevCam *cams, int V, int64_t N,
                      uint64_t *keys, uint32_t *vals, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits.
// Buffers a/b ping-pong; returns 0 if the result is in (ka, va), 1 if in (kb, vb).
size_t sort_tmp_bytes(int64_t n);
int launch_radix_sort(uint64_t *ka, uint32_t *va, uint64_t *kb, uint32_t *vb, int64_t n,
                      int bits, void *tmp, hipStream_t s);

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
void launch_ranges(const uint64_t *keys, int64_t D, uint2 *ranges, hipStream_t s);

struct RasterOut {
  float *rgb, *alpha, *depth, *normal;
  float *T_final;
  uint32_t *last, *n_contrib;
  // per pixel: bits 0-14 blended 3D pairs, 15-29 blended 2D pairs, bit 30 the
  // stopping pair was 2D, bit 31 the pixel stopped (work accounting)
  uint32_t *wcount;
};
void launch_raster_fwd(const uint2 *ranges, const uint32_t *vals, const Record *rec,
                       const DevCam *cams, int V, int n_tiles_total, int W, int H,
                       int tiles_x, int tiles_per_view, DevOpts opt, RasterOut out,
                       hipStream_t s);

struct RasterGradIn {
  const float *rgb, *alpha, *depth, *normal;
};
void launch_raster_bwd(const uint2 *ranges, const uint32_t *vals, const Record *rec,
                       int n_tiles_total, int W, int H, int tiles_x, int tiles_per_view,
                       DevOpts opt, const float *T_final, const uint32_t *last,
                       RasterGradIn g, float *accum, hipStream_t s);

}  // namespace hgs
