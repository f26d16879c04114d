// Internal declarations of the gfx950 hybrid rasterizer (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hgs {

constexpr int kTile = 16;            // 16x16 pixel tiles
constexpr int kBlock = 256;          // one thread per pixel of a tile
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

// Render options as the kernels take them.  rr0 is the smallest binary32
// >= 2 ln(1 / alpha_min) (the radius^2 of the support of an opaque splat),
// inv_amin = 1 / alpha_min rounded to binary32 (culling bounds only).
struct DevOpts {
  float bg[3];
  float dilation;
  float lambda_z, theta_z, temp_z;
  float alpha_min, alpha_max, t_min;
  float rr0, inv_amin;
  uint32_t out_mask;
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

// One request of a batched launch: a scene seen by one camera.  Its
// instances are [inst_base, inst_base + scene.n) and its tiles start at
// cam.tile_base.  Output images are [C, H, W] per request (NULL: not
// written).  Slots are ordered by inst_base and by tile_base.
struct Slot {
  SceneDev scene;
  DevCam cam;
  int64_t inst_base;
  float *rgb, *alpha, *depth, *normal;
};

// Last slot r < ns with slots[r].inst_base <= i (binary search).
__device__ inline int slot_of_instance(const Slot *slots, int ns, int64_t i) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (slots[mid].inst_base <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Last slot r < ns with slots[r].cam.tile_base <= t (binary search).
__device__ inline int slot_of_tile(const Slot *slots, int ns, int t) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (slots[mid].cam.tile_base <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ----- launchers (all enqueue on `s`) -----
// flags per (view, splat): bit 0 valid, bit 1 normal negated, bits 2-3 normal axis
// prect (may be NULL): each instance's tile rectangle packed in 32 bits,
// see pack_tile_rect.
void launch_preprocess(const SceneDev &sc, const DevCam *cams, int V, DevOpts opt,
                       Record *rec, uint32_t *tiles, uint32_t *zbits, int4 *rect,
                       uint8_t *flags, uint32_t *prect, hipStream_t s);

// Tile rectangle of an instance in one word: first tile column and row
// (bits 0-7, 8-15), width and height in tiles minus one (16-23, 24-31);
// kNoTiles for an instance that covers no tile, kWideRect for one whose
// rectangle reaches past tile column or row 255 (its count and rectangle
// are then read from the tiles and rect arrays).
constexpr uint32_t kNoTiles = 0xffffffffu, kWideRect = 0xfffffffeu;
__host__ __device__ inline bool tile_rect_packs(int4 r) {
  return (r.z >> 4) <= 255 && (r.w >> 4) <= 255;
}
__host__ __device__ inline uint32_t pack_tile_rect(int4 r) {
  const uint32_t tx0 = (uint32_t)r.x >> 4, ty0 = (uint32_t)r.y >> 4;
  return tx0 | (ty0 << 8) | ((((uint32_t)r.z >> 4) - tx0) << 16) |
         ((((uint32_t)r.w >> 4) - ty0) << 24);
}
__host__ __device__ inline uint32_t packed_tile_count(uint32_t p) {
  return p == kNoTiles ? 0u : (((p >> 16) & 255u) + 1u) * ((p >> 24) + 1u);
}
// The same for a batch of requests: instances [0, *n_inst) of the slot
// table (grid sized by the capacity inst_cap).
void launch_preprocess_slots(const Slot *slots, const int *n_slots, const uint64_t *n_inst,
                             DevOpts opt, int64_t inst_cap, Record *rec, uint32_t *tiles,
                             uint32_t *zbits, int4 *rect, uint8_t *flags, uint32_t *prect,
                             hipStream_t s);
void launch_preprocess_bwd(const SceneDev &sc, const DevCam *cams, int V, DevOpts opt,
                           const uint8_t *flags, const int4 *rect, const float *accum,
                           float *g_means, float *g_scales, float *g_rots, float *g_opac,
                           float *g_sh, int accumulate, hipStream_t s);
// FDO with one view.  Planes at accum, accum + plane, accum + 2 plane hold
// the colour, low and high slots.  One thread per primitive forms its
// Alg. 1 weights (w_low, w_high) from g_low and g_high, adds the number of
// conflicting primitives to *n_conflict (may be NULL), and writes (or adds,
// if accumulate) the update g_color + w_low g_low + w_high g_high as the
// chain of the slots c + w_low l + w_high h (the chain is linear in them).
void launch_fdo_fused_bwd(const SceneDev &sc, const DevCam *cams, DevOpts opt,
                          const uint8_t *flags, const int4 *rect, const float *accum,
                          int64_t plane, uint32_t *n_conflict, float *g_means, float *g_scales,
                          float *g_rots, float *g_opac, float *g_sh, int accumulate,
                          hipStream_t s);

// Counts.  Every launcher below takes a host count n that sizes the grid.
// Where it also takes n_dev (may be NULL), the kernels use min(n, *n_dev):
// the count then lives on the device and a captured launch stays valid for
// any count up to the capacity n.

// Exclusive scan of n uint32 values; writes the 64-bit total to *total
// (device).  `tmp` must hold scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
void launch_scan(const uint32_t *in, uint32_t *out, int64_t n, uint64_t *total, void *tmp,
                 hipStream_t s, const uint64_t *n_dev = nullptr);

// out[j] = in[idx[j]] for j < n.
void launch_gather(const uint32_t *in, const uint32_t *idx, int64_t n, uint32_t *out,
                   hipStream_t s, const uint64_t *n_dev = nullptr);

// Pairs of the V*N instances taken in the order `order` (a permutation):
// instance order[j] writes its (global tile id, instance id) pairs at
// offsets[j], the exclusive scan of tiles[order[.]].
// Pairs at or past pair_cap are dropped and set *overflow = 1 (overflow may
// be NULL only if the caller knows the pairs fit).
// prect_sorted: the packed tile rectangles in the order `order` (from the
// depth sort's gather); tiles and rect are read only for kWideRect entries.
// zero[0, zero_n) (may be empty) is cleared by the same launch.
void launch_duplicate(const uint32_t *order, const uint32_t *offsets, const uint32_t *tiles,
                      const int4 *rect, const uint32_t *prect_sorted, const DevCam *cams, int V,
                      int64_t N, uint64_t pair_cap, uint32_t *keys, uint32_t *vals,
                      uint32_t *overflow, uint32_t *zero, int64_t zero_n, hipStream_t s);

// Copies n host cameras to dst through kernel arguments (up to
// kCamsPerUpload per launch), so that a captured graph carries the camera
// values themselves rather than a host address.
constexpr int kCamsPerUpload = 8;
// Up to kMax small uint32 arrays cleared by the same launch.
struct ZeroList {
  static constexpr int kMax = 3;
  uint32_t *p[kMax] = {nullptr, nullptr, nullptr};
  int n[kMax] = {0, 0, 0};
};
void launch_upload_cams(const DevCam *host, int n, DevCam *dst, hipStream_t s,
                        ZeroList z = ZeroList{});
// The same for a batch of slots, with the instance count on the device.
// Pairs at or past pair_cap are dropped and set *overflow = 1.
void launch_duplicate_slots(const uint32_t *order, const uint32_t *offsets,
                            const uint32_t *tiles, const int4 *rect, const uint32_t *prect_sorted,
                            const Slot *slots, const int *n_slots, int64_t inst_cap,
                            const uint64_t *n_inst, uint64_t pair_cap, uint32_t *keys,
                            uint32_t *vals, uint32_t *overflow, hipStream_t s);

// Stable LSD radix sort of n (u32 key, u32 value) pairs on the low `bits`
// bits (at most 32), 8 bits per pass.  The passes read (k0, v0) (v0 NULL:
// value = index) and ping-pong between (ka, va) and (kb, vb).  k0/v0 may
// alias kb/vb but not ka/va; when they alias neither, a pass whose digit is
// the same for every key is skipped on the device.  Returns 0 if the result
// is in (ka, va), 1 if in (kb, vb) (fixed by the number of passes).
// zero_free: keys equal to 0 are don't-care (their place among the other
// keys may be anything), so a pass whose digit is the same for every other
// key is skipped as well; the other keys' order is exact.  `tmp` holds
// sort_tmp_bytes(n) bytes.  If gather_dst is given, the last pass also
// writes gather_dst[j] = gather_src[value j] of the sorted order; with
// gather_dst2 as well, gather_src holds packed tile rectangles and the pass
// writes gather_dst[j] = their tile counts (from gather_tiles for kWideRect
// words), gather_dst2[j] = the words.  err (may
// be NULL): bit 1 is set if a pass's look-back gave up (never expected).
// zeroed_words (may be NULL): kSortWords uint32 the caller has cleared on
// the stream, used for the sort's digit counts and tickets instead of the
// head of tmp (which is then not cleared by a launch of its own).
constexpr int kSortWords = 4 * 256 + 4 + 1;
size_t sort_tmp_bytes(int64_t n);
int launch_radix_sort(const uint32_t *k0, const uint32_t *v0, uint32_t *ka, uint32_t *va,
                      uint32_t *kb, uint32_t *vb, int64_t n, int bits, void *tmp, hipStream_t s,
                      const uint64_t *n_dev = nullptr, const uint32_t *gather_src = nullptr,
                      uint32_t *gather_dst = nullptr, uint32_t *err = nullptr,
                      uint32_t *zeroed_words = nullptr, uint32_t *gather_dst2 = nullptr,
                      const uint32_t *gather_tiles = nullptr, bool zero_free = false);

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// Up to kMax uint32 arrays set to zero in one launch (p[a] may be NULL when
// n[a] is 0).
struct FillList {
  static constexpr int kMax = 6;
  uint32_t *p[kMax] = {};
  int64_t n[kMax] = {};
};
void launch_zero_list(const FillList &f, hipStream_t s);
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
// ranges[t] = [first, last + 1) of tile t in the tile-sorted keys (ranges
// must be zeroed first).
void launch_ranges(const uint32_t *keys, int64_t D, uint2 *ranges, hipStream_t s,
                   const uint64_t *D_dev = nullptr);

struct RasterOut {
  float *rgb, *alpha, *depth, *normal;
  float *T_final;
  uint32_t *last, *n_contrib;
  // per pixel: bits 0-14 blended 3D pairs, 15-29 blended 2D pairs, bit 30 the
  // stopping pair was 2D, bit 31 the pixel stopped (work accounting)
  uint32_t *wcount;
  // per tile (may be NULL; zero at launch): .y receives 8 times the largest
  // number of list positions one of the tile's forward waves blended, the
  // backward's work per wave, laid out as ranges so that launch_tile_order
  // can order the backward's tiles by it
  uint2 *vis;
};
// bmask (may be NULL): receives the blend masks the backward walks,
// raster_mask_words(D capacity, tiles) 64-bit words.
inline int64_t raster_mask_words(int64_t pairs, int64_t tiles) {
  return 8 * ((pairs >> 6) + tiles + 1);
}
// order[n_tiles_total]: the tiles by pair-list length, longest first (from
// ranges), the order in which the raster launches below start their tiles.
// n_tiles_dev (may be NULL): the tile count on the device (at most
// n_tiles_total).  n_split (may be NULL): receives how many tiles, at the
// front of the order, have a non-empty pair list (the batch forward walks
// those with half-quadrant waves).
// total_out (may be NULL; mapped pinned host memory): receives *total, the
// render's pair count, without a copy command of its own.  clear (may be
// NULL): n_tiles entries set to zero (a RasterOut::vis for the forward).
void launch_tile_order(const uint2 *ranges, int n_tiles_total, uint32_t *order, hipStream_t s,
                       const int *n_tiles_dev = nullptr, uint32_t *n_split = nullptr,
                       const uint64_t *total = nullptr, uint64_t *total_out = nullptr,
                       uint2 *clear = nullptr);
// The backward's set-up in one launch: order[n_tiles_total] receives the
// tiles by vis (a RasterOut::vis of the forward, as launch_tile_order orders
// by ranges) while the other workgroups set acc[0..n) to zero (acc 16-byte
// aligned, n a multiple of 4).
void launch_order_and_clear(const uint2 *vis, int n_tiles_total, uint32_t *order, float *acc,
                            int64_t n, hipStream_t s);
// order (may be NULL: tile index order): from launch_tile_order.
void launch_raster_fwd(const uint2 *ranges, const uint32_t *order, const uint32_t *vals,
                       const Record *rec, int n_tiles_total, int W, int H, int tiles_x,
                       int tiles_per_view, DevOpts opt, RasterOut out, uint64_t *bmask,
                       hipStream_t s);

// Forward of a batch of slots on a persistent grid of n_blocks wave64s (a
// multiple of 8) that pull work units from the counters queue[kQueueStride x],
// x = 0..7 (zero at launch; one per XCD, each on a 256-byte line of its
// own) over the device tile count *n_tiles: with order and n_split (from
// launch_tile_order), the per-view forward's waves in that order, else
// (tile, quadrant).  Writes each slot's images.
constexpr int kQueueStride = 64;
constexpr int kQueueWords = 8 * kQueueStride;
void launch_raster_fwd_queue(const uint2 *ranges, const uint32_t *vals, const Record *rec,
                             const Slot *slots, const int *n_slots, const int *n_tiles,
                             int n_blocks, DevOpts opt, uint32_t *queue, hipStream_t s,
                             const uint32_t *order = nullptr, const uint32_t *n_split = nullptr);

struct RasterGradIn {
  const float *rgb, *alpha, *depth, *normal;
};
void launch_raster_bwd(const uint2 *ranges, const uint32_t *order, const uint32_t *vals,
                       const Record *rec, int n_tiles_total, int W, int H, int tiles_x,
                       int tiles_per_view, DevOpts opt, const float *T_final,
                       const uint32_t *last, const uint64_t *bmask, RasterGradIn g,
                       float *accum, hipStream_t s);
// Two RGB-only cotangent images [V,3,H,W] (NULL = zero).
struct RgbSets {
  const float *rgb[2];
};
// The backward with three cotangent sets in one traversal: g (all channels)
// into accum, rgb2.rgb[k] into accum + (k + 1) * plane (floats).
void launch_raster_bwd_sets(const uint2 *ranges, const uint32_t *order, const uint32_t *vals,
                            const Record *rec, int n_tiles_total, int W, int H, int tiles_x,
                            int tiles_per_view, DevOpts opt, const float *T_final,
                            const uint32_t *last, const uint64_t *bmask, RasterGradIn g,
                            RgbSets rgb2, float *accum, int64_t plane, hipStream_t s);

// Adaptive Type Exchange in place on n primitives (rotations: float4 per
// primitive, 16-byte aligned).  counts (may be NULL): [0] += switched 3D->2D,
// [1] += 2D->3D.  At most n_cu blocks.
void launch_type_exchange(int64_t n, float *scales, float *rots, uint8_t *types, double theta,
                          uint32_t *counts, int n_cu, hipStream_t s);

// Frequency losses of ren against tgt ([planes, H, W], planes = V * 3):
// weighted cotangents into g_low / g_high (either may be NULL) and, if
// losses != NULL, losses[0] += L_low, losses[1] += L_high (double, device).
// At most n_cu blocks.
void launch_fdo_cotangents(int64_t planes, int H, int W, const float *ren, const float *tgt,
                           double lambda_low, double lambda_high, float *g_low, float *g_high,
                           double *losses, int n_cu, hipStream_t s);
// Alg. 1 per primitive.  gc, gl, gh, out: 5 pointers each (means, scales,
// rotations, opacities, SH with sh_coeffs coefficients; NULL = zero / not
// written).  n_conflict (may be NULL) += number of conflicting primitives.
void launch_fdo_project(int64_t n, int sh_coeffs, const uint8_t *types, const float *const *gc,
                        const float *const *gl, const float *const *gh, float *const *out,
                        int accumulate, uint32_t *n_conflict, int n_cu, hipStream_t s);

// Colour loss (L1 + D-SSIM).  Win11: the normalised 11-tap Gaussian
// (sigma 1.5) of the SSIM window.  launch_ssim_fwd writes the derivative
// maps A, B, C ([planes, H, W]) and adds mean |x - y| and 1 - mean SSIM
// into losses[0], losses[1] (may be NULL); launch_ssim_bwd writes the
// cotangent of (1 - lambda) L1 + lambda D-SSIM.
struct Win11 {
  float w[11];
};
Win11 gauss_win11();
void launch_ssim_fwd(int64_t planes, int H, int W, const float *x, const float *y, float *Am,
                     float *Bm, float *Cm, double *losses, int n_cu, hipStream_t s);
void launch_ssim_bwd(int64_t planes, int H, int W, const float *x, const float *y,
                     const float *Am, const float *Bm, const float *Cm, double lambda,
                     float *grad, int n_cu, hipStream_t s);

// Adam over the five parameter arrays (means, scales, rotations,
// opacities, sh) flattened: array s holds elements [off[s], off[s+1]).
// NULL raw or grad skips an array; NULL act does not write activated values.
struct AdamArgs {
  float *raw[5], *m[5], *v[5], *act[5];
  const float *grad[5];
  int64_t off[6];
  float lr[5], lr_sh_rest, beta1, beta2, omb1, omb2, eps, bc1, bc2;  // omb = 1 - beta
  int64_t sh_stride;  // 3 K: SH elements of one primitive (the first 3 are DC)
  int64_t blk[6];     // set by launch_adam: blocks [blk[s], blk[s+1]) serve array s
  int vec[5];         // set by launch_adam: array s is 16-byte aligned throughout
};
void launch_adam(const AdamArgs &a, int n_cu, hipStream_t s);

// Densification statistics from n_planes accumulator planes ([V*N, 16]
// each, `plane` floats apart): grad_norm[g] += |dL/d screen centre| in NDC
// units and count[g] += 1 per view in which splat g is not culled.
void launch_densify_stats(int64_t V, int64_t N, const uint8_t *flags, const Record *rec,
                          const float *accum, int64_t plane, int n_planes, int W, int H,
                          float *grad_norm, float *count, int n_cu, hipStream_t s);

}  // namespace hgs
