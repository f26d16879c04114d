// Per-tile compositing (forward) and its reverse pass (backward), gfx950.
//
// Work unit: one wave64 per half quadrant (8x4 pixels) of a 16x16 tile,
// launched as its own workgroup so that waves never wait for each other.
// Every pixel is held by two lanes, l and l + 32, which take consecutive
// records of the list: each step evaluates two records, one per 32-lane
// half, and both halves run the pixel's compositing chain over the two in
// list order.  (A whole-quadrant forward wave, one pixel per lane, remains
// for tiles below the split threshold, which is zero.)  The eight waves of
// a tile are given block ids that the dispatcher sends to the same XCD, so
// the tile's pair list and records are fetched into one L2.  A wave walks
// its tile's depth-sorted pair list in chunks of 64: each lane loads one
// pair's 80-byte record (the next chunk is prefetched into registers while
// the current one is composited), tests the record's pixel rectangle
// against the wave's box, and the hits are compacted in list order into
// the wave's LDS slots (ballot + mbcnt).  The serial loop then visits only
// those records, read from LDS; the 2D/3D branch is per 32-lane half.
// Skipping a record whose rectangle misses the box changes nothing: the
// rectangle bounds the support where alpha~ >= alpha_min.
//
// Forward (Sec. 3.1, Eq. 1-2): d_i is the Mahalanobis distance under the
// projected covariance (3D) or u^2 + v^2 at the ray-splat intersection (2D).
// The contribution is alpha~ = min(alpha_max, alpha_eff e^{-d/2}).  A pair
// is skipped when alpha~ < alpha_min (false for NaN).  A pixel stops before
// the pair that would take its transmittance below t_min (defaults 0.99,
// 1/255 and 1e-4, the thresholds of the rasterizer the paper builds on).
// A wave stops when its pixels are done.
//
// Backward: each pixel walks its list in reverse from its last blended pair.
// It recovers T_i = T_{i+1} / (1 - alpha~_i) and carries the suffix
// S = alpha~ f + (1 - alpha~) S of the per-pair scalar
// f = <G_rgb, c> + G_depth depth + <G_n, n>.  dL/dalpha~ = T_i (f - S).  The
// 16 per-pair gradient terms are reduced over each 32-lane half in
// registers (a transposed reduce-scatter on the cross-lane swap and DPP
// paths, no LDS) and added with one atomic instruction per step (16 lanes
// per half) into the per-(view, splat) accumulators.

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr float kLn2 = 0.69314718055994531f;
constexpr int kWave = 64;  // one wave64 per 8x8 quadrant of a tile; also the chunk length

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
                                              const float4 &r3) {
#pragma clang fp contract(off)
  PairEval p;
  p.xr = fxp - r0.x;
  p.yr = fyp - r0.y;
  if (is3d) {
    const float dx = p.xr - r1.x, dy = p.yr - r1.y;
    const float t = __builtin_fmaf(r1.w, dy, r1.z * dx);  // A dx + B dy
    const float u = r2.x * dy;                             // C dy
    p.e = __builtin_fmaf(dx, t, u * dy);
    p.depth = r2.y;
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

// The next batch's record of this lane, held in five registers while the
// current batch is composited.
#define HGS_FETCH(rec, id, q0, q1, q2, q3, q4) \
  do {                                        \
    const float4 *p_ = (rec)[id].r;           \
    q0 = p_[0];                               \
    q1 = p_[1];                               \
    q2 = p_[2];                               \
    q3 = p_[3];                               \
    q4 = p_[4];                               \
  } while (0)

struct Quad {
  int tile;
  int v;           // view
  int sub;         // 0..7: quadrant * 2 + half, the wave's blend-mask region
  int qx, qy;      // top-left pixel of the wave's box
  int rows;        // 8 (a quadrant) or 4 (half a quadrant of a long-list tile)
  int px, py;      // this lane's pixel
  float fx, fy;    // pixel sample (x + 1/2, y + 1/2)
  bool inside;
};

// Tiles whose pair list is at least this long (every tile: the threshold is
// zero) are walked by two waves per quadrant, each on 8 x 4 pixels and
// culling against its own half.  Each pixel is held by two lanes (l and
// l + 32), which evaluate two consecutive records at once: a step reads two
// records from LDS and composites both, where a whole-quadrant wave reads
// one, and a half meets fewer splats than the whole quadrant.  The
// whole-quadrant walk remains for the batch forward's empty tiles.
constexpr uint32_t kSplitLen = 0;

// Quadrant `quad` of the view-local tile r (row-major over tiles_x columns);
// with split, its half `half` (rows 4 half .. 4 half + 3).
__device__ __forceinline__ Quad make_quad(int tile, int v, int r, int quad, int W, int H,
                                          int tiles_x, bool split = false, int half = 0) {
  Quad q;
  q.tile = tile;
  q.v = v;
  q.sub = quad * 2 + (split ? half : 0);
  const int ty = r / tiles_x;
  const int tx = r - ty * tiles_x;
  q.rows = split ? 4 : 8;
  q.qx = tx * kTile + (quad & 1) * 8;
  q.qy = ty * kTile + (quad >> 1) * 8 + (split ? 4 * half : 0);
  const int lane = threadIdx.x;
  // a half quadrant's 32 pixels are held twice: by lane l and lane l + 32
  q.px = q.qx + (lane & 7);
  q.py = q.qy + ((lane >> 3) & (q.rows - 1));
  q.fx = (float)q.px + 0.5f;
  q.fy = (float)q.py + 0.5f;
  q.inside = q.px < W && q.py < H;
  return q;
}

// Forward: blocks 64g + 8j + x hold tile slot 8g + x, quadrant j / 2, half
// j % 2, so the eight waves of a tile share x = block id mod 8, the XCD the
// dispatcher assigns them to.  Slot s is tile order[s] (longest pair lists
// first, see tile_order_kernel), or tile s without an order.  Returns false for the second-half wave of a
// tile that is not split (that wave has nothing to do).
__device__ __forceinline__ bool quad_of(const uint2 *ranges, const uint32_t *order, int n_tiles,
                                        int W, int H, int tiles_x, int tiles_per_view, Quad &q,
                                        uint2 &rg) {
  const int b = blockIdx.x;
  const int slot = (b >> 6) * 8 + (b & 7);
  if (slot >= n_tiles) return false;
  const int tile = order ? (int)order[slot] : slot;
  const int j = (b >> 3) & 7;
  rg = ranges[tile];
  const bool split = rg.y - rg.x >= kSplitLen;
  if (!split && (j & 1)) return false;
  const int v = tile / tiles_per_view;
  q = make_quad(tile, v, tile - v * tiles_per_view, j >> 1, W, H, tiles_x, split, j & 1);
  return true;
}

// Blend masks: for each wave (quadrant, or half quadrant of a split tile),
// one 64-bit word per chunk of 64 positions of its tile's pair list, bit j
// set if the pair at position 64 c + j was blended at one or more of the
// wave's pixels.  The forward writes them and the backward walks only those
// pairs (a pair blended at no pixel of the wave contributes nothing to its
// gradients).  Tile t with pair range [a, a + n) owns the words
// [8 (a / 64 + t), 8 (a / 64 + t) + 8 ceil(n / 64)), wave region s = 2
// quadrant + half the s-th run of ceil(n / 64): since floor(a / 64) +
// floor(n / 64) <= floor((a + n) / 64), the regions of consecutive tiles
// never overlap, and all fit in 8 (D / 64 + T + 1) words.
__device__ __forceinline__ uint64_t *quad_mask_words(uint64_t *bmask, uint2 rg, int tile,
                                                     int sub) {
  const uint32_t n = rg.y - rg.x;
  const uint64_t base = 8ull * ((uint64_t)(rg.x >> 6) + (uint64_t)tile);
  return bmask + base + (uint64_t)sub * ((n + 63u) >> 6);
}

// Output images of one view: channel planes of H*W pixels (NULL: skip).
struct ViewOut {
  float *rgb, *alpha, *depth, *normal, *T_final;
  uint32_t *last, *n_contrib, *wcount;
  uint2 *vis;  // per tile, not per view (see RasterOut)
};

// 2D record: U, V, W (rows of the inverse map, affine in the local pixel
// frame) span intervals over the box of the quadrant's pixel samples, with
// their extremes at the corners; each interval is widened by the rounding
// of a binary32 evaluation.  If W's interval excludes 0, the exponent
// e = (U^2 + V^2) / W^2 is at least (min U^2 + min V^2) / max W^2 at every
// sample, and the record is dropped if that bound exceeds
// log2(alpha_eff / alpha_min) by a margin.
__device__ __forceinline__ bool meets_2d(const float4 &r0, const float4 &r1, const float4 &r2,
                                         const float4 &r3, const float4 &r4, float qx, float qy,
                                         float ylast, float inv_amin) {
  const float xa = (qx + 0.5f) - r0.x, xb = (qx + 7.5f) - r0.x;
  const float ya = (qy + 0.5f) - r0.y, yb = (ylast + 0.5f) - r0.y;
  const float mx = fmaxf(fabsf(xa), fabsf(xb)), my = fmaxf(fabsf(ya), fabsf(yb));
  auto span = [&](float a, float b, float c, float &lo, float &hi) {
    const float t0 = __builtin_fmaf(a, xa, __builtin_fmaf(b, ya, c));
    const float t1 = __builtin_fmaf(a, xb, __builtin_fmaf(b, ya, c));
    const float t2 = __builtin_fmaf(a, xa, __builtin_fmaf(b, yb, c));
    const float t3 = __builtin_fmaf(a, xb, __builtin_fmaf(b, yb, c));
    const float pad = 1e-6f * (fabsf(a) * mx + fabsf(b) * my + fabsf(c));
    lo = fminf(fminf(t0, t1), fminf(t2, t3)) - pad;
    hi = fmaxf(fmaxf(t0, t1), fmaxf(t2, t3)) + pad;
  };
  auto sqmin = [](float lo, float hi) {
    return (lo <= 0.0f && hi >= 0.0f) ? 0.0f : fminf(lo * lo, hi * hi);
  };
  float ul, uh, vl, vh, wl, wh;
  span(r1.x, r1.y, r1.z, ul, uh);
  span(r1.w, r2.x, r2.y, vl, vh);
  span(r2.z, r2.w, r3.x, wl, wh);
  if (!(wl > 0.0f || wh < 0.0f)) return true;  // W may vanish (or NaN): keep
  const float w2 = fmaxf(wl * wl, wh * wh);
  const float elb = (sqmin(ul, uh) + sqmin(vl, vh)) / w2;
  const float lim = __builtin_amdgcn_logf(fabsf(r4.w) * inv_amin);
  return !(elb > lim + 1e-3f + 1e-3f * fabsf(lim));
}

// Can the record reach alpha~ >= alpha_min at a pixel of the quadrant?  Its
// inclusive pixel rectangle (r0) must meet the quadrant.  For a 3D record
// the exponent e = A dx^2 + B dx dy + C dy^2 (positive definite) is also
// minimised over the box spanned by the quadrant's pixel samples (the
// minimum of a convex quadratic over a box: 0 if the centre is inside, else
// the least of the four edge minima, each at its clamped stationary point);
// the record is dropped only if that lower bound of e at every sample
// exceeds log2(alpha_eff / alpha_min) by more than a margin that covers the
// rounding of the binary32 evaluation in eval_pair.  Dropping a record that
// contributes to no pixel of the quadrant changes nothing.
__device__ __forceinline__ bool meets(const float4 &r0, const float4 &r1, const float4 &r2,
                                      const float4 &r3, const float4 &r4, const Quad &q,
                                      float inv_amin) {
  const float qx = (float)q.qx, qy = (float)q.qy, ylast = (float)(q.qy + q.rows - 1);
  if (!(r0.x <= qx + 7.0f && r0.z >= qx && r0.y <= ylast && r0.w >= qy)) return false;
  if (__float_as_uint(r4.w) >> 31) return meets_2d(r0, r1, r2, r3, r4, qx, qy, ylast, inv_amin);
  const float A = r1.z, B = r1.w, C = r2.x;
  if (!(A > 0.0f && C > 0.0f)) return true;
  // sample box in the record's frame, as eval_pair forms dx, dy
  const float x0 = ((qx + 0.5f) - r0.x) - r1.x, x1 = ((qx + 7.5f) - r0.x) - r1.x;
  const float y0 = ((qy + 0.5f) - r0.y) - r1.y, y1 = ((ylast + 0.5f) - r0.y) - r1.y;
  if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return true;
  const float hA = -0.5f * B * __builtin_amdgcn_rcpf(A), hC = -0.5f * B * __builtin_amdgcn_rcpf(C);
  auto at = [&](float x, float y) { return x * (A * x + B * y) + C * y * y; };
  const float ya = fminf(fmaxf(hC * x0, y0), y1), yb = fminf(fmaxf(hC * x1, y0), y1);
  const float xa = fminf(fmaxf(hA * y0, x0), x1), xb = fminf(fmaxf(hA * y1, x0), x1);
  const float emin = fminf(fminf(at(x0, ya), at(x1, yb)), fminf(at(xa, y0), at(xb, y1)));
  const float lim = __builtin_amdgcn_logf(fabsf(r4.w) * inv_amin);
  return !(emin > lim + 1e-3f + 1e-4f * fabsf(lim));
}

// Issue priority of a wave by the length of the list it walks: the long
// lists of the few dense tiles set the kernel's critical path, so their
// waves win issue slots over the short ones sharing their SIMD.
__device__ __forceinline__ void prio_for_list(int n) {
  if (n > 2048) __builtin_amdgcn_s_setprio(3);
  else if (n > 768) __builtin_amdgcn_s_setprio(2);
  else if (n > 256) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

__device__ __forceinline__ int lane_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ bool is3d_of(const float4 &r4) {
  return (__builtin_amdgcn_readfirstlane(__float_as_int(r4.w)) >> 31) == 0;
}

// Exponent e (alpha~ = alpha_eff 2^-e) and depth value d of a record at this
// lane's pixel, in the operation order of eval_pair.
__device__ __forceinline__ void fwd_exponent(bool two, const Quad &q, const float4 &r0,
                                             const float4 &r1, const float4 &r2,
                                             const float4 &r3, float &e, float &d) {
#pragma clang fp contract(off)
  const float xr = q.fx - r0.x, yr = q.fy - r0.y;
  if (two) {
    const float U = __builtin_fmaf(r1.x, xr, __builtin_fmaf(r1.y, yr, r1.z));
    const float V = __builtin_fmaf(r1.w, xr, __builtin_fmaf(r2.x, yr, r2.y));
    const float Wh = __builtin_fmaf(r2.z, xr, __builtin_fmaf(r2.w, yr, r3.x));
    const float rw = __builtin_amdgcn_rcpf(Wh);
    const float uu = U * rw, vv = V * rw;
    e = __builtin_fmaf(uu, uu, vv * vv);
    d = rw;
  } else {
    const float dx = xr - r1.x, dy = yr - r1.y;
    const float t = __builtin_fmaf(r1.w, dy, r1.z * dx);
    const float u3 = r2.x * dy;
    e = __builtin_fmaf(dx, t, u3 * dy);
    d = r2.y;
  }
}

// One pair of the compositing chain at a pixel: its contribution a (0 unless
// raw >= thr, clamped at alpha_max), the stop before a pair that would take
// T below t_min, and the pair's weight a T (0 at the stop).  thr is the
// activity threshold: alpha_min while the pixel composites, +inf once it has
// stopped, so one compare serves both.  raw >= thr is false for NaN, so the
// integer min of the bit patterns (the float min for numbers >= +0) only
// sees numbers >= +0.
__device__ __forceinline__ void fwd_step(float raw, int amax_bits, float tmin, float &T,
                                         float &thr, float &wg) {
  const float a = raw >= thr ? __int_as_float(min(__float_as_int(raw), amax_bits)) : 0.0f;
  const float Tn = T * (1.0f - a);
  const bool stop = Tn < tmin;
  wg = stop ? 0.0f : a * T;
  thr = stop ? __builtin_inff() : thr;
  T = stop ? T : Tn;
}

// Composites one quadrant: the wave's 64 pixels over the tile's pair range.
// kAcct: also count blended pairs by type for the work accounting (wcount).
template <bool kAcct>
__device__ __forceinline__ void raster_fwd_quad(const Quad &q, uint2 rg, const uint32_t *vals,
                                                const Record *rec, int W, int H,
                                                const DevOpts &opt, const ViewOut &out,
                                                uint64_t *wm, float4 (*srec)[kWave],
                                                uint32_t *spos) {
  const int lane = threadIdx.x;
  const int n = (int)(rg.y - rg.x);
  prio_for_list(n);

  // thr is the activity threshold: alpha_min while the pixel composites, +inf
  // once it has stopped, so one compare gives both tests.
  float T = 1.0f;
  float thr = q.inside ? opt.alpha_min : __builtin_inff();
  // alpha_max as bits: for numbers >= +0 (raw always is, where it counts)
  // the integer min of the bit patterns is the float min, in one op
  const int amax_bits = __float_as_int(opt.alpha_max);
  const float tmin = opt.t_min, inv_amin = opt.inv_amin;
  int lastk = -1;  // compacted slot of this lane's last blended pair in the chunk
  uint32_t nvis = 0;  // positions blended at one or more of the wave's pixels
  float cr = 0.0f, cg = 0.0f, cb = 0.0f, dep = 0.0f, nx = 0.0f, ny = 0.0f, nz = 0.0f;
  uint32_t cnt = 0, last = 0, wc = 0;

  // pipeline: records of chunk c in q0..q4, list entry of chunk c + 64 in nid
  float4 q0 = make_float4(0, 0, 0, 0), q1 = q0, q2 = q0, q3 = q0, q4 = q0;
  uint32_t nid = 0;
  if (lane < n) HGS_FETCH(rec, vals[rg.x + lane], q0, q1, q2, q3, q4);
  if (kWave + lane < n) nid = vals[rg.x + kWave + lane];
  for (int c = 0; c < n; c += kWave) {
    if (__ballot(thr < 1.0f) == 0ull) break;
    const bool hit = (c + lane < n) && meets(q0, q1, q2, q3, q4, q, inv_amin);
    const uint64_t m = __ballot(hit);
    __syncthreads();  // the previous chunk's slots have been read
    if (hit) {
      const int slot = lane_rank(m);
      srec[0][slot] = q0;
      srec[1][slot] = q1;
      srec[2][slot] = q2;
      srec[3][slot] = q3;
      srec[4][slot] = q4;
      spos[slot] = (uint32_t)(c + lane);
    }
    const int k_end = __popcll(m);
    // a half-quadrant wave takes records in pairs: an odd count gets a zero
    // record (raw 0, never active) in the free slot after the last
    if (q.rows != 8 && (k_end & 1) && lane < 5) srec[lane][k_end] = make_float4(0, 0, 0, 0);
    __syncthreads();
    if (c + kWave + lane < n) HGS_FETCH(rec, nid, q0, q1, q2, q3, q4);
    if (c + 2 * kWave + lane < n) nid = vals[rg.x + c + 2 * kWave + lane];
    uint64_t used = 0;  // compacted slots blended at one or more lanes
    if (q.rows == 8) {
      for (int k0 = 0; k0 < k_end; k0 += 2) {
        if (__ballot(thr < 1.0f) == 0ull) break;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int k = k0 + j;
          if (k >= k_end) break;
          const float4 r0 = srec[0][k], r1 = srec[1][k], r2 = srec[2][k], r3 = srec[3][k],
                       r4 = srec[4][k];
          // r3.x is used by the 2D branch only; naming it here keeps r3 one
          // 16-byte LDS read instead of pieces with an address of their own
          asm volatile("" ::"v"(r3.x));
          // the type is the same at every lane (one record): a scalar branch,
          // so a 3D pair does not pay for the 2D form's reciprocal
          const bool two = !is3d_of(r4);
          float e, d;
          fwd_exponent(two, q, r0, r1, r2, r3, e, d);
          const float raw = fabsf(r4.w) * exp2_neg(e);
          // active: raw >= thr (false for NaN).  An inactive pair has a = 0,
          // so only an active pair can take T below t_min (the stop); the
          // weight is 0 unless the pair is blended, and the accumulations run
          // unconditionally (record values are finite, see preprocess).
          const float thr0 = thr;
          float wg;
          fwd_step(raw, amax_bits, tmin, T, thr, wg);
          cr = __builtin_fmaf(wg, r3.y, cr);
          cg = __builtin_fmaf(wg, r3.z, cg);
          cb = __builtin_fmaf(wg, r3.w, cb);
          dep = __builtin_fmaf(wg, raw >= thr0 ? d : 0.0f, dep);  // 1/W is inf where W = 0
          nx = __builtin_fmaf(wg, r4.x, nx);
          ny = __builtin_fmaf(wg, r4.y, ny);
          nz = __builtin_fmaf(wg, r4.z, nz);
          const bool bl = wg > 0.0f;
          used |= (__ballot(bl) != 0ull) ? (1ull << k) : 0ull;
          cnt += bl ? 1u : 0u;
          lastk = bl ? k : lastk;
          if constexpr (kAcct) {
            wc += bl ? (two ? (1u << 15) : 1u) : 0u;
            wc |= thr0 < 1.0f && !(thr < 1.0f) ? (0x80000000u | (two ? 0x40000000u : 0u)) : 0u;
          }
        }
      }
    } else {
      // Half quadrant: lane l and lane l + 32 hold the same pixel.  Each step
      // the lower half evaluates record k0 and the upper half record k0 + 1
      // (the two exponents in parallel); both halves then run the same
      // transmittance chain over the two records in list order, so T, the
      // activity and stop decisions are those of the one-record walk, and
      // each half accumulates its own record's weighted values.  The halves'
      // sums are added at the end.
      // Each half also keeps its own count of blended records and its own
      // last blended slot; the two are combined at the chunk's end (last)
      // and at the end (count).
      const int hi = lane >> 5;
      const bool upper = lane >= 32;
      for (int k0 = 0; k0 < k_end; k0 += 2) {
        if (__ballot(thr < 1.0f) == 0ull) break;
        const int k = k0 + hi;
        const float4 r0 = srec[0][k], r1 = srec[1][k], r2 = srec[2][k], r3 = srec[3][k],
                     r4 = srec[4][k];
        asm volatile("" ::"v"(r3.x));
        // the halves' records may differ in type: a per-lane branch
        const bool two = (__float_as_uint(r4.w) >> 31) != 0u;
        float e, d;
        fwd_exponent(two, q, r0, r1, r2, r3, e, d);
        const float raw = fabsf(r4.w) * exp2_neg(e);
        const auto rr = __builtin_amdgcn_permlane32_swap(__float_as_uint(raw),
                                                         __float_as_uint(raw), false, false);
        const float raw0 = __uint_as_float(rr[0]), raw1 = __uint_as_float(rr[1]);
        const float thr0 = thr;
        float wg0, wg1;
        fwd_step(raw0, amax_bits, tmin, T, thr, wg0);
        const float thr1 = thr;
        fwd_step(raw1, amax_bits, tmin, T, thr, wg1);
        // this half's record; a blended record (weight > 0) is active, so
        // its d is finite (1/W is inf where W = 0), and a record that is not
        // blended adds 0 whichever d it gets
        const float wg = upper ? wg1 : wg0;
        const bool bl = wg > 0.0f;
        cr = __builtin_fmaf(wg, r3.y, cr);
        cg = __builtin_fmaf(wg, r3.z, cg);
        cb = __builtin_fmaf(wg, r3.w, cb);
        dep = __builtin_fmaf(wg, bl ? d : 0.0f, dep);
        nx = __builtin_fmaf(wg, r4.x, nx);
        ny = __builtin_fmaf(wg, r4.y, ny);
        nz = __builtin_fmaf(wg, r4.z, nz);
        const uint64_t bm = __ballot(bl);  // bits 0-31: record k0, 32-63: k0 + 1
        uint32_t bm_hi = (uint32_t)(bm >> 32);
        asm("" : "+s"(bm_hi));  // a 32-bit scalar compare, not a 64-bit vector one
        used |= ((uint32_t)bm != 0u ? (1ull << k0) : 0ull) | (bm_hi != 0u ? (2ull << k0) : 0ull);
        cnt += bl ? 1u : 0u;
        lastk = bl ? k : lastk;
        if constexpr (kAcct) {
          const bool bl0 = wg0 > 0.0f, bl1 = wg1 > 0.0f;
          const uint64_t tb = __ballot(two);
          const bool two0 = tb & 1ull, two1 = (tb >> 32) & 1ull;
          wc += bl0 ? (two0 ? (1u << 15) : 1u) : 0u;
          wc |= thr0 < 1.0f && !(thr1 < 1.0f) ? (0x80000000u | (two0 ? 0x40000000u : 0u)) : 0u;
          wc += bl1 ? (two1 ? (1u << 15) : 1u) : 0u;
          wc |= thr1 < 1.0f && !(thr < 1.0f) ? (0x80000000u | (two1 ? 0x40000000u : 0u)) : 0u;
        }
      }
      // the later of the two halves' last blended slots
      lastk = max(lastk, (int)__builtin_amdgcn_permlane32_swap(lastk, lastk, false, false)[upper ? 0 : 1]);
    }
    if (lastk >= 0) last = spos[lastk] + 1u;
    lastk = -1;
    if (wm || out.vis) {  // the chunk's positions blended in this quadrant
      const uint64_t pm = __ballot(hit && ((used >> lane_rank(m)) & 1ull));
      if (wm && lane == 0) wm[c >> 6] = pm;
      nvis += (uint32_t)__popcll(pm);
    }
  }
  if (out.vis && lane == 0) atomicMax(&out.vis[q.tile].y, 8u * nvis);
  if (q.rows != 8) {  // half quadrant: add the upper half's sums to the lower's
    auto fold = [](float &x) {
      const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x),
                                                      false, false);
      x = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    };
    fold(cr);
    fold(cg);
    fold(cb);
    fold(dep);
    fold(nx);
    fold(ny);
    fold(nz);
    cnt += __builtin_amdgcn_permlane32_swap(cnt, cnt, false, false)[1];
    if (lane >= 32) return;
  }
  if (!q.inside) return;
  const int64_t hw = (int64_t)H * W;
  const int64_t o1 = (int64_t)q.py * W + q.px;
  const int64_t o3 = o1;
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
  if (out.n_contrib) out.n_contrib[o1] = cnt;
  if (kAcct && out.wcount) out.wcount[o1] = wc;
}

// Views of one size: the block id picks the tile and quadrant (quad_of).  At
// most 80 VGPRs: six waves per SIMD (the half-quadrant walk takes 88 when
// left alone, which allows five).
template <bool kAcct>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(6)))
raster_fwd_kernel(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ order,
                  const uint32_t *__restrict__ vals, const Record *__restrict__ rec, int n_tiles,
                  int W, int H, int tiles_x, int tiles_per_view, DevOpts opt, RasterOut out,
                  uint64_t *__restrict__ bmask) {
  __shared__ float4 srec[5][kWave];
  __shared__ uint32_t spos[kWave];
  Quad q;
  uint2 rg;
  if (!quad_of(ranges, order, n_tiles, W, H, tiles_x, tiles_per_view, q, rg)) return;
  const int64_t hw = (int64_t)H * W, v = q.v;
  ViewOut vo;
  vo.rgb = out.rgb ? out.rgb + v * 3 * hw : nullptr;
  vo.alpha = out.alpha ? out.alpha + v * hw : nullptr;
  vo.depth = out.depth ? out.depth + v * hw : nullptr;
  vo.normal = out.normal ? out.normal + v * 3 * hw : nullptr;
  vo.T_final = out.T_final ? out.T_final + v * hw : nullptr;
  vo.last = out.last ? out.last + v * hw : nullptr;
  vo.n_contrib = out.n_contrib ? out.n_contrib + v * hw : nullptr;
  vo.wcount = out.wcount ? out.wcount + v * hw : nullptr;
  vo.vis = out.vis;
  raster_fwd_quad<kAcct>(q, rg, vals, rec, W, H, opt, vo,
                         bmask ? quad_mask_words(bmask, rg, q.tile, q.sub) : nullptr, srec,
                         spos);
}

// A batch of slots (requests of any size), persistent: each wave takes work
// units from an atomic counter until they run out; every wave reaches that
// exit.  With a tile order (order, n_split from tile_order_kernel), the
// units are the waves of the per-view forward in that order: 8 per
// non-empty tile (quadrant x half) for the first *n_split tiles, then 4
// whole quadrants per (empty) tile; without one, 4 per tile.  The tiles are
// dealt to the XCDs by slot mod 8, as the per-view forward's block mapping
// does: the waves of block b (which the dispatcher sends to XCD b mod 8)
// pop the units of the slots s = b (mod 8) from counter b mod 8, so a
// tile's waves share one L2 and each counter sees an eighth of the pops.
// The counters sit kQueueStride words (256 bytes) apart: on one line, the
// eight XCDs' atomics serialised on it and took 545 instead of 354 us per
// batch at 200 requests/s.  They must be zero at launch.  At most 80 VGPRs (six waves per
// SIMD), as the per-view forward.
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(6)))
raster_fwd_queue_kernel(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ order,
                        const uint32_t *__restrict__ n_split, const uint32_t *__restrict__ vals,
                        const Record *__restrict__ rec, const Slot *__restrict__ slots,
                        const int *__restrict__ n_slots, const int *__restrict__ n_tiles,
                        DevOpts opt, uint32_t *__restrict__ queue) {
  __shared__ float4 srec[5][kWave];
  __shared__ uint32_t spos[kWave];
  const int ns = *n_slots;
  const uint32_t nt = (uint32_t)max(*n_tiles, 0);
  const uint32_t nsp = order ? min(*n_split, nt) : 0u;
  const uint32_t x = blockIdx.x & 7u;
  // this XCD's split slots x, x + 8, ... below nsp, then its other slots
  // from the first s >= nsp with s = x (mod 8)
  const uint32_t n_sp = nsp > x ? (nsp - x + 7u) >> 3 : 0u;
  const uint32_t first = nsp + ((x - nsp) & 7u);
  const uint32_t n_wq = first < nt ? (nt - first + 7u) >> 3 : 0u;
  const uint32_t units = 8u * n_sp + 4u * n_wq;
  if (ns <= 0) return;
  for (;;) {
    uint32_t u = 0;
    if (threadIdx.x == 0) u = atomicAdd(queue + kQueueStride * x, 1u);
    u = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl((int)u, 0));
    if (u >= units) break;
    uint32_t slot_i, quad, half = 0;
    bool split = false;
    if (u < 8u * n_sp) {
      slot_i = 8u * (u >> 3) + x;
      quad = (u >> 1) & 3u;
      half = u & 1u;
      split = true;
    } else {
      const uint32_t k = u - 8u * n_sp;
      slot_i = first + 8u * (k >> 2);
      quad = k & 3u;
    }
    const int tile = order ? (int)order[slot_i] : (int)slot_i;
    const Slot &sl = slots[slot_of_tile(slots, ns, tile)];
    const int W = sl.cam.W, H = sl.cam.H;
    const Quad q = make_quad(tile, 0, tile - sl.cam.tile_base, (int)quad, W, H, sl.cam.tiles_x,
                             split, (int)half);
    ViewOut vo{};
    vo.rgb = sl.rgb;
    vo.alpha = sl.alpha;
    vo.depth = sl.depth;
    vo.normal = sl.normal;
    raster_fwd_quad<false>(q, ranges[tile], vals, rec, W, H, opt, vo, nullptr, srec, spos);
    __syncthreads();  // the unit's LDS slots are free before the next unit
  }
}

// Cross-lane helper of the reduce-scatter: swap16(a, b) gives the lanes of
// the even 16-lane rows (a, a of lane + 16) and those of the odd rows (b of
// lane - 16, b); the sum of the pair is then the two-lane sum of a (even
// rows) or of b (odd rows).
__device__ __forceinline__ float swap16_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// x of the DPP partner lane: row_mirror pairs lane i with i ^ 15 inside a
// 16-lane row, row_half_mirror i with i ^ 7 inside 8 lanes, quad_perm
// [1,0,3,2] i with i ^ 1 and [2,3,0,1] i with i ^ 2.
template <int kCtrl>
__device__ __forceinline__ float dpp(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                               kCtrl, 0xf, 0xf, false));
}
constexpr int kRowMirror = 0x140, kRowHalfMirror = 0x141, kQuadXor1 = 0xB1, kQuadXor2 = 0x4E;

// Sums each of the 16 per-lane values over the lanes of each 32-lane half of
// the wave separately (the halves hold different pairs).  Lane l returns its
// half's total of value 8 b4 + 4 b3 + 2 b2 + b1 (b_i = bit i of l); lanes l
// and l ^ 1 hold the same total.  Pairings used: bit 4 (swap16), l ^ 15,
// l ^ 7, l ^ 2, l ^ 1 -- together they span the 32 lanes of a half.
__device__ __forceinline__ float half_reduce_scatter16(const float (&g)[16], int lane) {
  float t[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) t[k] = swap16_sum(g[k], g[k + 8]);
  const bool b3 = lane & 8;
  float u[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float keep = b3 ? t[k + 4] : t[k];
    const float send = b3 ? t[k] : t[k + 4];
    u[k] = keep + dpp<kRowMirror>(send);
  }
  const bool b2 = lane & 4;
  float w[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float keep = b2 ? u[k + 2] : u[k];
    const float send = b2 ? u[k] : u[k + 2];
    w[k] = keep + dpp<kRowHalfMirror>(send);
  }
  const bool b1 = lane & 2;
  float x = (b1 ? w[1] : w[0]) + dpp<kQuadXor2>(b1 ? w[0] : w[1]);
  x += dpp<kQuadXor1>(x);
  return x;
}

// Record-geometry slots 0-8 of a pair from dL/de (ge) and, for a 2D pair,
// the depth weight gdz = dL/d depth (3D: slot 5 is the depth slot, written
// by the caller).  The slots are formed in scalars and stored once with
// constant indices (stores in both branches of the 2D/3D split are
// otherwise merged by the compiler into one store at a selected index,
// which moves g to scratch memory).
__device__ __forceinline__ void pair_geometry_grads(float (&g)[16], const PairEval &p, bool is3d,
                                                    float ge, float gdz, const float4 &r1,
                                                    const float4 &r2) {
  float x0, x1, x2, x3, x4, x5, x6, x7, x8;
  if (is3d) {
    const float dx = p.a0, dy = p.a1;
    x0 = -ge * (2.0f * r1.z * dx + r1.w * dy);
    x1 = -ge * (r1.w * dx + 2.0f * r2.x * dy);
    x2 = ge * dx * dx;
    x3 = ge * dx * dy;
    x4 = ge * dy * dy;
    x5 = g[5];
    x6 = x7 = x8 = 0.0f;
  } else {
    const float rw = p.rw;
    const float rw2 = rw * rw;
    const float gU = ge * 2.0f * p.a0 * rw2;
    const float gV = ge * 2.0f * p.a1 * rw2;
    const float gW = -2.0f * ge * p.e * rw - gdz * rw2;
    x0 = gU * p.xr;
    x1 = gU * p.yr;
    x2 = gU;
    x3 = gV * p.xr;
    x4 = gV * p.yr;
    x5 = gV;
    x6 = gW * p.xr;
    x7 = gW * p.yr;
    x8 = gW;
  }
  g[0] = x0;
  g[1] = x1;
  g[2] = x2;
  g[3] = x3;
  g[4] = x4;
  g[5] = x5;
  g[6] = x6;
  g[7] = x7;
  g[8] = x8;
}

// Destination of a reduced gradient total: accumulator plane and slot.
struct PackDst {
  int plane, slot;
};

// Terms of one RGB-only cotangent set (cr, cg, cb) for a pair whose dL/dalpha~
// in that set is ga, into the main set's 16-slot layout (depth and normal
// slots 0).
__device__ __forceinline__ void rgb_set_terms(float (&g)[16], float cr, float cg, float cb,
                                              float ga, float wg, bool live, float a, float G,
                                              const PairEval &p, bool is3d, const float4 &r1,
                                              const float4 &r2) {
  g[10] = wg * cr;
  g[11] = wg * cg;
  g[12] = wg * cb;
  g[13] = g[14] = g[15] = 0.0f;
  g[5] = 0.0f;
  const float ge = live ? -ga * a * kLn2 : 0.0f;
  g[9] = live ? ga * G : 0.0f;
  pair_geometry_grads(g, p, is3d, ge, 0.0f, r1, r2);
}

// Backward of one half quadrant (8 x 4 pixels).  Lane l and lane l + 32 hold
// the same pixel.  The wave walks the pairs its forward wave blended (its
// blend mask) in reverse list order, two per step: the upper half of the
// wave evaluates the later one (compacted slot k), the lower half the
// earlier (slot k - 1).  One swap gives every lane both pairs' alpha~ (0
// where the pair is not active) and one more each per-pair scalar f of a
// cotangent set; both halves then run the transmittance recovery and the
// suffix recurrences over the two pairs in that order, so T, S and
// dL/dalpha~ at each pixel are those of the one-pair walk bit for bit.
// Each half forms its own pair's 16 gradient terms per set, one 32-lane
// reduce-scatter per 16 terms sums both pairs', and one atomic instruction
// adds both totals.  NS = 1: one cotangent set (gin) into accum.  NS = 3:
// also the RGB-only sets rgb2.rgb[0], rgb2.rgb[1] into accum + plane and
// accum + 2 plane; where both pairs of a step are 3D, their 31 non-zero
// terms travel in two reductions instead of three (layout at packA, packB).
template <int NS>
__device__ __forceinline__ void raster_bwd_half(const uint2 *ranges, const uint32_t *order,
                                                const uint32_t *vals, const Record *rec,
                                                int n_tiles, int W, int H, int tiles_x,
                                                int tiles_per_view, const DevOpts &opt,
                                                const float *T_final, const uint32_t *last_in,
                                                const RasterGradIn &gin, const RgbSets &rgb2,
                                                float *accum, int64_t plane,
                                                const uint64_t *bmask) {
  __shared__ float4 srec[5][kWave];
  __shared__ uint32_t sid[kWave];
  __shared__ uint32_t spos[kWave];
  Quad q;
  uint2 rg;
  if (!quad_of(ranges, order, n_tiles, W, H, tiles_x, tiles_per_view, q, rg)) return;
  const int lane = threadIdx.x;
  const bool upper = lane >= 32;

  float T = 1.0f;
  uint32_t L = 0;
  float Gr = 0, Gg = 0, Gb = 0, Ga = 0, Gd = 0, Gnx = 0, Gny = 0, Gnz = 0;
  float Xr[2] = {0.0f, 0.0f}, Xg[2] = {0.0f, 0.0f}, Xb[2] = {0.0f, 0.0f};
  if (q.inside) {
    const int64_t hw = (int64_t)H * W;
    const int64_t pix = (int64_t)q.py * W + q.px;
    const int64_t o1 = (int64_t)q.v * hw + pix;
    const int64_t o3 = (int64_t)q.v * 3 * hw + pix;
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
    if constexpr (NS == 3) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (rgb2.rgb[k]) {
          Xr[k] = rgb2.rgb[k][o3];
          Xg[k] = rgb2.rgb[k][o3 + hw];
          Xb[k] = rgb2.rgb[k][o3 + 2 * hw];
        }
      }
    }
  }
  // suffix values beyond the last blended pair: background and alpha terms
  float S = Gr * opt.bg[0] + Gg * opt.bg[1] + Gb * opt.bg[2] - Ga;
  float XS[2] = {0.0f, 0.0f};
  if constexpr (NS == 3) {
#pragma unroll
    for (int k = 0; k < 2; ++k) XS[k] = Xr[k] * opt.bg[0] + Xg[k] * opt.bg[1] + Xb[k] * opt.bg[2];
  }

  const int amax_bits = __float_as_int(opt.alpha_max);
  uint32_t wmax = L;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) wmax = max(wmax, (uint32_t)__shfl_xor((int)wmax, d));
  const int n = min((int)__builtin_amdgcn_readfirstlane(wmax), (int)(rg.y - rg.x));
  if (n <= 0) return;
  prio_for_list(n);
  const int vidx = ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 + ((lane >> 2) & 1) * 2 +
                   ((lane >> 1) & 1);
  // NS = 3, both pairs 3D: destination (plane, slot) of this lane's total in
  // the two packed reductions.  A: the main set, whose slots 6-8 (zero for a
  // 3D pair) carry RGB set 1's colour slots 10-12.  B: set 1's slots 0-4 and
  // 9, then set 2's slots 0-4, 9, 10-12; entry 15 is unused.
  const PackDst packA = vidx >= 6 && vidx <= 8 ? PackDst{1, vidx + 4} : PackDst{0, vidx};
  const PackDst packB = vidx <= 4    ? PackDst{1, vidx}
                        : vidx == 5  ? PackDst{1, 9}
                        : vidx <= 10 ? PackDst{2, vidx - 6}
                        : vidx == 11 ? PackDst{2, 9}
                        : vidx <= 14 ? PackDst{2, vidx - 2}
                                     : PackDst{0, -1};
  const uint64_t *wm = quad_mask_words(const_cast<uint64_t *>(bmask), rg, q.tile, q.sub);

  // chunks of 64 list positions in reverse, the first the ragged one; only
  // the positions this half's forward wave blended.  Pipeline: records of
  // chunk c in q0..q4 (entry id), entries of chunk c - 64 in nid.
  float4 q0 = make_float4(0, 0, 0, 0), q1 = q0, q2 = q0, q3 = q0, q4 = q0;
  uint32_t id = 0, nid = 0;
  int c = (n - 1) & ~(kWave - 1);
  bool hit = (c + lane < n) && ((wm[c >> 6] >> lane) & 1ull);
  if (hit) {
    id = vals[rg.x + c + lane];
    HGS_FETCH(rec, id, q0, q1, q2, q3, q4);
  }
  bool hit_n = c > 0 && ((wm[(c >> 6) - 1] >> lane) & 1ull);
  if (hit_n) nid = vals[rg.x + c - kWave + lane];
  for (; c >= 0; c -= kWave) {
    const uint64_t m = __ballot(hit);
    __syncthreads();  // the previous chunk's slots have been read
    if (hit) {
      const int slot = lane_rank(m);
      srec[0][slot] = q0;
      srec[1][slot] = q1;
      srec[2][slot] = q2;
      srec[3][slot] = q3;
      srec[4][slot] = q4;
      sid[slot] = id;
      spos[slot] = (uint32_t)(c + lane);
    }
    // pairs are taken two at a time: an odd count gets a zero record
    // (alpha~ 0, never active) in the free slot after the last
    const int kk = __popcll(m);
    if (kk & 1) {
      if (lane < 5) srec[lane][kk] = make_float4(0, 0, 0, 0);
      if (lane == 5) sid[kk] = 0u;
      if (lane == 6) spos[kk] = 0u;
    }
    __syncthreads();
    if (c > 0) {  // earlier chunks: every position is below n
      hit = hit_n;
      id = nid;
      if (hit) HGS_FETCH(rec, id, q0, q1, q2, q3, q4);
      hit_n = c > kWave && ((wm[(c >> 6) - 2] >> lane) & 1ull);
      if (hit_n) nid = vals[rg.x + c - 2 * kWave + lane];
    }
    for (int k = kk + (kk & 1) - 1; k > 0; k -= 2) {
      const int ks = upper ? k : k - 1;
      const float4 r0 = srec[0][ks], r1 = srec[1][ks], r2 = srec[2][ks], r3 = srec[3][ks],
                   r4 = srec[4][ks];
      const uint32_t pos = spos[ks], sk = sid[ks];
      asm volatile("" ::"v"(r2.z), "v"(r2.w), "v"(r3.x));
      // the halves' pairs may differ in type: a per-lane branch
      const bool is3d = (__float_as_uint(r4.w) >> 31) == 0u;
      const PairEval p = eval_pair(is3d, q.fx, q.fy, r0, r1, r2, r3);
      const float G = exp2_neg(p.e);
      const float raw = fabsf(r4.w) * G;
      const bool act = (pos < L) && (raw >= opt.alpha_min);
      if (__ballot(act) == 0ull) continue;
      // an inactive lane's weights are 0, and a 2D pair's intersection, which
      // can be non-finite where the pair does not contribute, is replaced
      // there by finite values, so its gradient terms are exact zeros
      PairEval ps = p;
      if (!is3d) {
        ps.e = act ? p.e : 0.0f;
        ps.rw = act ? p.rw : 0.0f;
        ps.depth = act ? p.depth : 0.0f;
      }
      const float f = Gr * r3.y + Gg * r3.z + Gb * r3.w + Gd * ps.depth + Gnx * r4.x +
                      Gny * r4.y + Gnz * r4.z;
      // both pairs at every lane of the pixel: [0] the lower half's (slot
      // k - 1), [1] the upper half's (slot k); alpha~ is 0 where the pair is
      // not active (active implies alpha~ >= alpha_min > 0)
      const float rawe = act ? raw : 0.0f;
      const auto rs = __builtin_amdgcn_permlane32_swap(__float_as_uint(rawe),
                                                       __float_as_uint(rawe), false, false);
      const auto fs = __builtin_amdgcn_permlane32_swap(__float_as_uint(f), __float_as_uint(f),
                                                       false, false);
      // the later pair first (as the forward forms alpha~: the integer min of
      // the bit patterns, the float min for numbers >= +0)
      const float raw_h = __uint_as_float(rs[1]), raw_l = __uint_as_float(rs[0]);
      const bool act_h = raw_h > 0.0f, act_l = raw_l > 0.0f;
      const float a_h = __int_as_float(min(__float_as_int(raw_h), amax_bits));
      const float Ti_h = T * __builtin_amdgcn_rcpf(1.0f - a_h);
      const float dfa_h = __uint_as_float(fs[1]) - S;
      const float ga_h = act_h ? Ti_h * dfa_h : 0.0f;
      const float S1 = act_h ? __builtin_fmaf(a_h, dfa_h, S) : S;
      const float T1 = act_h ? Ti_h : T;
      const float a_l = __int_as_float(min(__float_as_int(raw_l), amax_bits));
      const float Ti_l = T1 * __builtin_amdgcn_rcpf(1.0f - a_l);
      const float dfa_l = __uint_as_float(fs[0]) - S1;
      const float ga_l = act_l ? Ti_l * dfa_l : 0.0f;
      S = act_l ? __builtin_fmaf(a_l, dfa_l, S1) : S1;
      T = act_l ? Ti_l : T1;
      // this half's pair
      const float a = upper ? a_h : a_l;
      const float Ti = upper ? Ti_h : Ti_l;
      const float ga = upper ? ga_h : ga_l;
      const bool live = act && !(raw > opt.alpha_max);  // not clamped: the exponent's path
      const float wg = act ? a * Ti : 0.0f;
      // the RGB-only sets' dL/dalpha~ of this half's pair, by the same
      // recurrence on their own suffixes
      float xga[2] = {0.0f, 0.0f};
      if constexpr (NS == 3) {
#pragma unroll
        for (int set = 0; set < 2; ++set) {
          const float fx = Xr[set] * r3.y + Xg[set] * r3.z + Xb[set] * r3.w;
          const auto xs = __builtin_amdgcn_permlane32_swap(__float_as_uint(fx),
                                                           __float_as_uint(fx), false, false);
          const float xdfa_h = __uint_as_float(xs[1]) - XS[set];
          const float xga_h = act_h ? Ti_h * xdfa_h : 0.0f;
          const float XS1 = act_h ? __builtin_fmaf(a_h, xdfa_h, XS[set]) : XS[set];
          const float xdfa_l = __uint_as_float(xs[0]) - XS1;
          const float xga_l = act_l ? Ti_l * xdfa_l : 0.0f;
          XS[set] = act_l ? __builtin_fmaf(a_l, xdfa_l, XS1) : XS1;
          xga[set] = upper ? xga_h : xga_l;
        }
      }
      float g[16];
      g[10] = wg * Gr;
      g[11] = wg * Gg;
      g[12] = wg * Gb;
      g[13] = wg * Gnx;
      g[14] = wg * Gny;
      g[15] = wg * Gnz;
      const float ge = live ? -ga * a * kLn2 : 0.0f;  // dL/de
      g[9] = live ? ga * G : 0.0f;                    // dL/d alpha_eff
      g[5] = wg * Gd;                                  // 3D: depth slot
      pair_geometry_grads(g, ps, is3d, ge, wg * Gd, r1, r2);
      const size_t rec_off = (size_t)sk * kGradSlots;
      if constexpr (NS == 1) {
        const float tot = half_reduce_scatter16(g, lane);
        if ((lane & 1) == 0 && tot != 0.0f) unsafeAtomicAdd(accum + rec_off + vidx, tot);
      } else {
        float g1[16], g2[16];
        rgb_set_terms(g1, Xr[0], Xg[0], Xb[0], xga[0], wg, live, a, G, ps, is3d, r1, r2);
        rgb_set_terms(g2, Xr[1], Xg[1], Xb[1], xga[1], wg, live, a, G, ps, is3d, r1, r2);
        if (__ballot(!is3d) == 0ull) {  // both pairs 3D: two packed reductions
          g[6] = g1[10];
          g[7] = g1[11];
          g[8] = g1[12];
          const float h[16] = {g1[0], g1[1], g1[2], g1[3],  g1[4],  g1[9],  g2[0],  g2[1],
                               g2[2], g2[3], g2[4], g2[9], g2[10], g2[11], g2[12], 0.0f};
          const float ta = half_reduce_scatter16(g, lane);
          const float tb = half_reduce_scatter16(h, lane);
          if ((lane & 1) == 0 && ta != 0.0f)
            unsafeAtomicAdd(accum + packA.plane * plane + rec_off + packA.slot, ta);
          if ((lane & 1) == 0 && tb != 0.0f && packB.slot >= 0)
            unsafeAtomicAdd(accum + packB.plane * plane + rec_off + packB.slot, tb);
        } else {
          const float t0 = half_reduce_scatter16(g, lane);
          const float t1 = half_reduce_scatter16(g1, lane);
          const float t2 = half_reduce_scatter16(g2, lane);
          if ((lane & 1) == 0) {
            if (t0 != 0.0f) unsafeAtomicAdd(accum + rec_off + vidx, t0);
            if (t1 != 0.0f) unsafeAtomicAdd(accum + plane + rec_off + vidx, t1);
            if (t2 != 0.0f) unsafeAtomicAdd(accum + 2 * plane + rec_off + vidx, t2);
          }
        }
      }
    }
  }
}

// NS = 1: one cotangent set.  NS = 3: the main set plus two RGB-only sets
// (rgb2[0], rgb2[1]) in the same reverse traversal -- one record fetch,
// one geometry and transmittance recomputation per pair -- accumulated into
// planes accum, accum + plane, accum + 2 plane.  Blocks as in the forward
// (quad_of): one wave per half quadrant.
template <int NS>
__global__ void __launch_bounds__(kWave)
raster_bwd_kernel(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ order,
                  const uint32_t *__restrict__ vals,
                  const Record *__restrict__ rec, int n_tiles, int W, int H, int tiles_x,
                  int tiles_per_view, DevOpts opt, const float *__restrict__ T_final,
                  const uint32_t *__restrict__ last_in, RasterGradIn gin, RgbSets rgb2,
                  float *__restrict__ accum, int64_t plane, const uint64_t *__restrict__ bmask) {
  raster_bwd_half<NS>(ranges, order, vals, rec, n_tiles, W, H, tiles_x, tiles_per_view, opt,
                      T_final, last_in, gin, rgb2, accum, plane, bmask);
}

// Tile order of the raster launches: tiles by pair-list length, longest
// first, in 16 buckets (empty; under 256; then steps of 256 up to 3584 and
// more), ascending tile index inside a bucket.  The dispatcher starts
// blocks in id order, so the waves that walk the longest lists start first
// instead of wherever their tiles sit in the image, and the short ones fill
// in behind them.  Inside a bucket, neighbouring tiles (which share splats)
// stay close in the launch order: finer buckets measured slower.
//
// One workgroup: the buckets are staged in LDS (up to 32768 tiles), then 16
// waves, each on a contiguous run of tiles, 64 at a time: the lanes with the
// same bucket find each other with four ballots (one per bucket bit), the
// highest of them adds the group's size to the wave's count of that bucket
// in LDS; an exclusive scan over (bucket descending, wave) gives each wave's
// bases; the second sweep ranks the same groups again and scatters.
constexpr int kOrderWaves = 16, kOrderBits = 4, kOrderBuckets = 1 << kOrderBits;
__device__ __forceinline__ int order_bucket(uint2 r) {
  const uint32_t n = r.y - r.x;
  return n == 0 ? 0 : 1 + (int)min((uint32_t)(kOrderBuckets - 2), n >> 8);
}
// the first bucket whose tiles are split (lists of kSplitLen and more)
constexpr int kSplitBucket = 1 + (int)(kSplitLen >> 8);
static_assert((kSplitLen & 255u) == 0, "split threshold on a bucket boundary");

// Lanes of the wave that hold the same bucket as this one (among `valid`).
__device__ __forceinline__ uint64_t bucket_peers(int b, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int k = 0; k < kOrderBits; ++k) {
    const bool bit = (b >> k) & 1;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

constexpr int kOrderLds = 32768;  // tiles whose buckets are staged in LDS first
// The ordering itself, by one workgroup of kOrderWaves waves; s_cnt and s_bk
// are its LDS (kOrderBuckets * kOrderWaves words, kOrderLds bytes).
__device__ __forceinline__ void tile_order_block(const uint2 *__restrict__ ranges, int n_tiles,
                                                 const int *__restrict__ n_dev,
                                                 uint32_t *__restrict__ order,
                                                 uint32_t *__restrict__ n_split,
                                                 const uint64_t *__restrict__ total,
                                                 uint64_t *__restrict__ total_out,
                                                 uint2 *__restrict__ clear, uint32_t *s_cnt,
                                                 uint8_t *s_bk) {
  if (total_out && threadIdx.x == 0)
    __hip_atomic_store(total_out, *total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  if (n_dev) n_tiles = min(n_tiles, max(*n_dev, 0));
  constexpr int kT = kOrderWaves * kWave;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int e = threadIdx.x; e < kOrderBuckets * kOrderWaves; e += kT) s_cnt[e] = 0;
  if (clear)
    for (int t = threadIdx.x; t < n_tiles; t += kT) clear[t] = make_uint2(0u, 0u);
  // every tile's bucket into LDS, eight loads in flight per thread (the
  // sweeps below then wait on no memory)
  const bool staged = n_tiles <= kOrderLds;
  if (staged) {
    for (int b0 = 0; b0 < n_tiles; b0 += 8 * kT) {
      uint2 r[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) r[u] = ranges[min(b0 + u * kT + (int)threadIdx.x, n_tiles - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = b0 + u * kT + (int)threadIdx.x;
        if (t < n_tiles) s_bk[t] = (uint8_t)order_bucket(r[u]);
      }
    }
  }
  __syncthreads();
  auto bucket_at = [&](int t) {
    return staged ? (int)s_bk[t] : order_bucket(ranges[t]);
  };
  const int per = ((n_tiles + kOrderWaves - 1) / kOrderWaves + kWave - 1) & ~(kWave - 1);
  const int t0 = w * per, t1 = min(n_tiles, t0 + per);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  auto entry = [&](int b) { return (kOrderBuckets - 1 - b) * kOrderWaves + w; };
  for (int tb = t0; tb < t1; tb += kWave) {
    const int t = tb + lane;
    const bool valid = t < t1;
    const int b = bucket_at(min(t, t1 - 1));
    const uint64_t peers = bucket_peers(b, valid);
    // the highest lane of each group; a wave's own entries, so no other
    // wave writes them
    if (valid && (peers >> lane) == 1ull) s_cnt[entry(b)] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  if (w == 0) {  // exclusive scan of the entries, eight per lane
    constexpr int kPer = kOrderBuckets * kOrderWaves / kWave;
    uint32_t c[kPer], sum = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      c[i] = s_cnt[kPer * lane + i];
      sum += c[i];
    }
    uint32_t inc = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)inc, d);
      inc += lane >= d ? o : 0u;
    }
    uint32_t base = inc - sum;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      s_cnt[kPer * lane + i] = base;
      base += c[i];
    }
  }
  __syncthreads();
  // tiles whose forward splits each quadrant in two come first: those of
  // the buckets from kSplitBucket up, as many as the base of the entry
  // (kSplitBucket - 1, wave 0)
  if (n_split && threadIdx.x == 0)
    *n_split = s_cnt[(kOrderBuckets - kSplitBucket) * kOrderWaves];
  for (int tb = t0; tb < t1; tb += kWave) {
    const int t = tb + lane;
    const bool valid = t < t1;
    const int b = bucket_at(min(t, t1 - 1));
    const uint64_t peers = bucket_peers(b, valid);
    const uint32_t at = valid ? s_cnt[entry(b)] : 0u;
    if (valid) order[at + (uint32_t)__popcll(peers & below)] = (uint32_t)t;
    // every lane has read its base before the group's highest lane moves it
    if (valid && (peers >> lane) == 1ull) s_cnt[entry(b)] = at + (uint32_t)__popcll(peers);
  }
}

__global__ void __launch_bounds__(kOrderWaves * kWave)
tile_order_kernel(const uint2 *__restrict__ ranges, int n_tiles, const int *__restrict__ n_dev,
                  uint32_t *__restrict__ order, uint32_t *__restrict__ n_split,
                  const uint64_t *__restrict__ total, uint64_t *__restrict__ total_out,
                  uint2 *__restrict__ clear) {
  __shared__ uint32_t s_cnt[kOrderBuckets * kOrderWaves];
  __shared__ uint8_t s_bk[kOrderLds];
  tile_order_block(ranges, n_tiles, n_dev, order, n_split, total, total_out, clear, s_cnt, s_bk);
}

// The backward's set-up in one launch: workgroup 0 orders the tiles (as
// tile_order_kernel), the others clear the accumulators (n4 float4s), which
// the ordering's single workgroup would otherwise leave the device idle for.
__global__ void __launch_bounds__(kOrderWaves * kWave)
order_and_clear_kernel(const uint2 *__restrict__ ranges, int n_tiles,
                       uint32_t *__restrict__ order, float4 *__restrict__ acc, int64_t n4) {
  __shared__ uint32_t s_cnt[kOrderBuckets * kOrderWaves];
  __shared__ uint8_t s_bk[kOrderLds];
  if (blockIdx.x == 0) {
    tile_order_block(ranges, n_tiles, nullptr, order, nullptr, nullptr, nullptr, nullptr, s_cnt,
                     s_bk);
    return;
  }
  const int64_t stride = (int64_t)(gridDim.x - 1) * blockDim.x;
  for (int64_t i = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x; i < n4; i += stride)
    acc[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Blocks: 64 per group of 8 tiles (four quadrants of two halves each), the
// forward's and the backward's, see quad_of.
unsigned quad_blocks(int n_tiles) { return (unsigned)((n_tiles + 7) / 8) * 64u; }

}  // namespace

void launch_tile_order(const uint2 *ranges, int n_tiles_total, uint32_t *order,
                       hipStream_t s, const int *n_tiles_dev, uint32_t *n_split,
                       const uint64_t *total, uint64_t *total_out, uint2 *clear) {
  if (n_tiles_total <= 0) return;
  hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(kOrderWaves * kWave), 0, s, ranges,
                     n_tiles_total, n_tiles_dev, order, n_split, total, total_out, clear);
}

void launch_order_and_clear(const uint2 *ranges, int n_tiles_total, uint32_t *order, float *acc,
                            int64_t n, hipStream_t s) {
  if (n_tiles_total <= 0) {
    launch_fill_f32(acc, 0.0f, n, s);
    return;
  }
  // acc is a workspace allocation (256-byte aligned) of n floats, n % 4 == 0
  const int64_t n4 = n / 4;
  const int64_t fill_blocks =
      std::min<int64_t>((n4 + kOrderWaves * kWave - 1) / (kOrderWaves * kWave), 2048);
  hipLaunchKernelGGL(order_and_clear_kernel, dim3((unsigned)(1 + fill_blocks)),
                     dim3(kOrderWaves * kWave), 0, s, ranges, n_tiles_total, order,
                     reinterpret_cast<float4 *>(acc), n4);
}

void launch_raster_fwd(const uint2 *ranges, const uint32_t *order, const uint32_t *vals,
                       const Record *rec, int n_tiles_total, int W, int H, int tiles_x,
                       int tiles_per_view, DevOpts opt, RasterOut out, uint64_t *bmask,
                       hipStream_t s) {
  if (n_tiles_total == 0) return;
  if (out.wcount)
    hipLaunchKernelGGL(raster_fwd_kernel<true>, dim3(quad_blocks(n_tiles_total)), dim3(kWave), 0,
                       s, ranges, order, vals, rec, n_tiles_total, W, H, tiles_x,
                       tiles_per_view, opt, out, bmask);
  else
    hipLaunchKernelGGL(raster_fwd_kernel<false>, dim3(quad_blocks(n_tiles_total)), dim3(kWave), 0,
                       s, ranges, order, vals, rec, n_tiles_total, W, H, tiles_x,
                       tiles_per_view, opt, out, bmask);
}

void launch_raster_fwd_queue(const uint2 *ranges, const uint32_t *vals, const Record *rec,
                             const Slot *slots, const int *n_slots, const int *n_tiles,
                             int n_blocks, DevOpts opt, uint32_t *queue, hipStream_t s,
                             const uint32_t *order, const uint32_t *n_split) {
  if (n_blocks <= 0) return;
  hipLaunchKernelGGL(raster_fwd_queue_kernel, dim3((unsigned)n_blocks), dim3(kWave), 0, s, ranges,
                     order, n_split, vals, rec, slots, n_slots, n_tiles, opt, queue);
}

void launch_raster_bwd(const uint2 *ranges, const uint32_t *order, const uint32_t *vals,
                       const Record *rec, int n_tiles_total, int W, int H, int tiles_x,
                       int tiles_per_view, DevOpts opt, const float *T_final,
                       const uint32_t *last, const uint64_t *bmask, RasterGradIn g,
                       float *accum, hipStream_t s) {
  if (n_tiles_total == 0) return;
  hipLaunchKernelGGL(raster_bwd_kernel<1>, dim3(quad_blocks(n_tiles_total)), dim3(kWave), 0, s,
                     ranges, order, vals, rec, n_tiles_total, W, H, tiles_x, tiles_per_view, opt,
                     T_final, last, g, RgbSets{}, accum, (int64_t)0, bmask);
}

void launch_raster_bwd_sets(const uint2 *ranges, const uint32_t *order, const uint32_t *vals,
                            const Record *rec, int n_tiles_total, int W, int H, int tiles_x,
                            int tiles_per_view, DevOpts opt, const float *T_final,
                            const uint32_t *last, const uint64_t *bmask, RasterGradIn g,
                            RgbSets rgb2, float *accum, int64_t plane, hipStream_t s) {
  if (n_tiles_total <= 0) return;
  hipLaunchKernelGGL(raster_bwd_kernel<3>,
                     dim3(quad_blocks(n_tiles_total)),
                     dim3(kWave), 0, s,
                     ranges, order, vals, rec, n_tiles_total, W, H, tiles_x, tiles_per_view, opt,
                     T_final, last, g, rgb2, accum, plane, bmask);
}

}  // namespace hgs
