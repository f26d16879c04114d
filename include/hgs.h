/*
 * hgs.h - C ABI of the MI355X (gfx950) hybrid 2D/3D Gaussian rasterizer.
 *
 * What it renders (EGGS, "Exchangeable 2D/3D Gaussian Splatting"):
 *   Sec. 3.1 "Hybrid Gaussian Rasterization".  A primitive has a centre mu,
 *   scales s, a quaternion r, an opacity alpha, SH colour coefficients f and a
 *   type flag t (0 = 2D surfel, 1 = 3D Gaussian).  Eq. 1 gives the distance
 *   d_i: for t = 0, u^2 + v^2 at the ray-splat intersection (appendix on
 *   rasterization, Eq. uv); for t = 1, the Mahalanobis distance under the
 *   affine projection Sigma' = J W Sigma W^T J^T.  Each pair contributes
 *   alpha_i exp(-d_i/2), and all pairs are composited front to back in one
 *   pass (Eq. 2).  2D opacities are modulated by
 *   alpha* = alpha exp(-lambda_z s_z*), s_z* = sigmoid((s_z - theta_z)/T_z) s_z
 *   (Sec. 3.2, Eq. 6-7).
 *
 * Readings the paper leaves open, fixed here:
 *   - pixel (x, y) is sampled at (x + 1/2, y + 1/2);
 *   - cameras use OpenCV axes (x right, y down, z forward);
 *   - a pair with alpha_i exp(-d_i/2) < 1/255 is skipped;
 *   - a contribution is clamped at 0.99;
 *   - a pixel stops before the pair that would take its transmittance
 *     below 1e-4;
 *   - 3D splats add delta (opts.dilation) to the diagonal of Sigma';
 *   - depth and normal outputs are accumulated with the blend weights and
 *     are not divided by alpha.
 *
 * Conventions
 *   - Every pointer is a device pointer unless marked [host].
 *   - Arrays are C-contiguous float32.  N = number of primitives,
 *     K = (sh_degree+1)^2, V = number of views, H x W = image size.
 *   - Every call validates its arguments on the host, enqueues work on
 *     `stream` (a hipStream_t; NULL = the null stream) and returns a status.
 *     Calls on one context must be serialised by the caller (one host thread,
 *     one stream at a time).
 *   - Asynchronous device errors show up in hgs_state_check or in the next
 *     call that synchronises.
 *   - No exception crosses this boundary.  On error, hgs_last_error() returns
 *     a message.
 *   - NaN/Inf parameters are not errors.  Every comparison that decides
 *     culling or activity is false for NaN, so such a primitive or pair is
 *     dropped.
 */
#ifndef HGS_H
#define HGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hgs_ctx hgs_ctx;
typedef struct hgs_state hgs_state;
typedef int32_t hgs_status;

enum {
  HGS_OK = 0,
  HGS_EINVAL = -1,    /* bad argument (null pointer, size out of range, ...) */
  HGS_ENOMEM = -2,    /* device or host allocation failed */
  HGS_EHIP = -3,      /* a HIP runtime call failed */
  HGS_ECAPACITY = -4, /* more (tile, splat) pairs than a capacity */
  HGS_ESTATE = -5     /* state used in the wrong way (e.g. backward twice) */
};

/* Scene parameters, Sec. 3.1.  Activated values: scales >= 0 (a 2D surfel
 * has s_z = 0 at initialisation and ignores it except through Eq. 6-7),
 * opacity in (0, 1).  Layouts: means [N,3], scales [N,3], rotations [N,4]
 * as (w, x, y, z), not necessarily unit length (normalised inside),
 * opacities [N], sh [N,K,3] (coefficient-major, channel-last), types [N]
 * uint8 (0 = 2D surfel, anything else = 3D Gaussian).  The caller owns
 * every array. */
typedef struct {
  int64_t n;
  int32_t sh_degree; /* 0..3 */
  const float *means, *scales, *rotations, *opacities, *sh;
  const uint8_t *types;
} hgs_scene_desc;

/* [host] A pinhole camera.  viewmat: row-major 4x4 world->camera, last row
 * (0,0,0,1).  fx, fy, cx, cy in pixels.  width, height in [1, 16384].
 * znear > 0: a 3D centre, or any point of a 2D surfel's support disc, at
 * z <= znear culls the primitive. */
typedef struct {
  float viewmat[16];
  float fx, fy, cx, cy;
  int32_t width, height;
  float znear;
} hgs_camera;

/* [host] Render options.  Defaults: bg = 0, dilation = 0.3 px^2,
 * lambda_z = 1, theta_z = 1.05, temp_z = 0.001 (Eq. 7's constants are the
 * paper's, appendix "Implementation Details"), alpha_min = 1/255,
 * alpha_max = 0.99, t_min = 1e-4, out_mask = 0.
 * The compositing thresholds of Eq. 2, which the paper inherits from the
 * rasterizer it builds on (Sec. 4, "Implementation"): a pair whose
 * alpha_eff exp(-d/2) is below alpha_min is skipped (and a primitive whose
 * opacity is below it is culled; the screen rectangles bound the support
 * alpha_eff exp(-d/2) >= alpha_min); a contribution is clamped at
 * alpha_max; a pixel stops before the pair that would take its
 * transmittance below t_min.  Requires 0 < alpha_min <= alpha_max < 1 and
 * 0 < t_min < 1.
 * out_mask selects the output channels: bit 0 rgb, 1 alpha, 2 depth,
 * 3 normal.  A channel whose bit is set needs its hgs_images pointer (NULL
 * is EINVAL); a clear bit leaves the channel unwritten whatever its
 * pointer.  out_mask = 0 writes every channel whose pointer is not NULL. */
typedef struct {
  float bg[3];
  float dilation;
  float lambda_z, theta_z, temp_z;
  float alpha_min, alpha_max, t_min;
  uint32_t out_mask;
} hgs_opts;

#define HGS_OUT_RGB 1u
#define HGS_OUT_ALPHA 2u
#define HGS_OUT_DEPTH 4u
#define HGS_OUT_NORMAL 8u

/* Output images, each [V,C,H,W]: rgb C=3, alpha C=1 (= 1 - T_final),
 * depth C=1 (sum of weight x camera z), normal C=3 (sum of weight x
 * camera-space unit normal facing the camera).  A pointer may be NULL for a
 * channel that opts.out_mask does not select (with out_mask = 0, any
 * pointer may be NULL and that channel is then not written). */
typedef struct {
  float *rgb, *alpha, *depth, *normal;
} hgs_images;

/* Upstream gradients dL/d(image), same shapes as hgs_images.  A NULL
 * pointer means zero. */
typedef struct {
  const float *rgb, *alpha, *depth, *normal;
} hgs_grad_images;

/* Parameter gradients, same shapes as hgs_scene_desc (opacities and scales
 * are gradients with respect to the activated values).  accumulate != 0
 * adds into the arrays; 0 overwrites them.  Any pointer may be NULL. */
typedef struct {
  float *means, *scales, *rotations, *opacities, *sh;
  int32_t accumulate;
} hgs_grads;

/* Create a context on HIP device `device`.  The context owns the device
 * workspaces and the resident scenes. */
hgs_status hgs_create(int32_t device, hgs_ctx **out);
void hgs_destroy(hgs_ctx *ctx);

/* Register a scene.  copy_resident = 1 copies the arrays into
 * library-owned device memory (serving); 0 borrows the caller's pointers,
 * which must stay valid (and may be updated in place between calls) until
 * hgs_scene_release (training).  Returns an id >= 0 through scene_id. */
hgs_status hgs_scene_init(hgs_ctx *ctx, const hgs_scene_desc *desc, int32_t copy_resident,
                          int32_t *scene_id);
hgs_status hgs_scene_release(hgs_ctx *ctx, int32_t scene_id);

/* Forward render of scene `scene_id` into V = n_views views that share one
 * image size (Sec. 3.1, Eq. 1-2).  The pipeline is: preprocess (cull,
 * project, SH -> RGB, screen rectangle), stable radix sort of the splat
 * instances by depth, exclusive scan of their tile counts in that order,
 * duplicate into (tile, instance) pairs, stable radix sort of the pairs by
 * tile, tile ranges, per-16x16-tile compositing.  The pairs end in
 * (tile, depth, instance id) order.
 *
 * `cams` [host] has n_views entries.  If `state` is not NULL, the call
 * returns in *state a library-owned handle.  The handle keeps what the
 * backward needs: per-splat records, the sorted list, tile ranges, final
 * transmittance and the last contributor per pixel.  Free it with
 * hgs_state_free.  Opts may be NULL (defaults).
 *
 * The call only enqueues work on `stream`: the pair count D stays on the
 * device, and the pair buffers and sort grids are sized by a pair
 * capacity.  The capacity is the context's (hgs_set_pair_capacity) or, by
 * default, one learned per pooled workspace: the first render on a
 * workspace synchronises `stream` once to read D, and later renders grow the
 * capacity from the D of that workspace's previous render once it has
 * finished, without waiting for it.  Pairs beyond the capacity are dropped
 * on the device; such a render's images are incomplete and
 * hgs_state_check reports ECAPACITY (and enlarges the learned capacity).
 * A render may be captured into a HIP graph on `stream` if the capacity is
 * known (a render of the same sizes has run on the context, or a fixed
 * capacity is set), its workspaces need not grow (same sizes as before) and
 * n_views <= 64; the state of a captured render must stay alive while the
 * graph is replayed (its buffers are the graph's), and everything on it
 * must use that stream.  Errors: EINVAL, ENOMEM, EHIP, ECAPACITY (more
 * than 2^32 - 1 pairs on the first render of a workspace). */
hgs_status hgs_render(hgs_ctx *ctx, int32_t scene_id, const hgs_camera *cams, int32_t n_views,
                      const hgs_opts *opts, const hgs_images *out, hgs_state **state,
                      void *stream);

/* Backward of the render that produced `state`: gradients of
 * L = sum <grad_out, images> with respect to means, scales (including s_z of
 * 2D surfels through Eq. 6-7), rotations, opacities and SH coefficients,
 * summed over the views.  Transmittance is recovered in reverse order; no
 * per-pixel list is stored.  The scene's parameters must be unchanged since
 * the forward.  May be called more than once on a state. */
hgs_status hgs_render_backward(hgs_ctx *ctx, hgs_state *state, const hgs_grad_images *grad_out,
                               const hgs_grads *grads, void *stream);

void hgs_state_free(hgs_ctx *ctx, hgs_state *state);

/* Fixes the pair capacity of every later render on ctx (max_pairs in
 * [1, 2^32 - 1]), or returns to the learned capacity (max_pairs = 0, the
 * default).  A fixed capacity never synchronises; see hgs_render. */
hgs_status hgs_set_pair_capacity(hgs_ctx *ctx, int64_t max_pairs);

/* Sizes kept in a state: [0] V*N, [1] number of (tile, splat) pairs D in
 * the sorted list (at most the capacity), [2] total tiles, [3] pixels per
 * view (H*W), [4] V.  Synchronises the state's stream the first time. */
hgs_status hgs_state_sizes(hgs_ctx *ctx, hgs_state *state, int64_t *sizes5 /* [host] */);

/* Copy one internal array of a state to host memory, for parity tests.
 * `what`:
 *   0 sorted keys   u64[D]  ((global tile << 32) | depth key of the pair's
 *                            instance; composed on the host)
 *   1 sorted values u32[D]  (value = view * N + splat)
 *   2 tile ranges   u32[T,2]
 *   3 pixel rectangles of every (view, splat), i32[V*N,4]
 *     (x0, y0, x1, y1 inclusive; garbage where tiles == 0)
 *   4 tiles touched u32[V*N]  (0 = culled)
 *   5 depth keys    u32[V*N]
 *   6 T_final       f32[V,H,W]
 *   7 last          u32[V,H,W]  (1 + list position of the last blended
 *                               pair within its tile, 0 if none)
 *   8 n_contrib     u32[V,H,W]
 *   9 pair counts   u32[V,H,W]  (bits 0-14 blended 3D pairs, 15-29 blended
 *                               2D pairs, bit 30 the pair that stopped the
 *                               pixel was 2D, bit 31 the pixel stopped;
 *                               recorded only by a render made while
 *                               HGS_PROFILE_WORK is enabled, else EINVAL)
 * `capacity` is the size of dst in bytes.  The call synchronises. */
hgs_status hgs_state_debug(hgs_ctx *ctx, hgs_state *state, int32_t what, void *dst_host,
                           int64_t capacity);

/* Synchronise the state's stream and report any asynchronous error, or
 * ECAPACITY if the render produced more pairs than its capacity (the next
 * render on this context is given room for them). */
hgs_status hgs_state_check(hgs_ctx *ctx, hgs_state *state);

/* Per-stage timing and work accounting.  `on` is a set of flags (0 turns
 * both off; other bits are EINVAL):
 *   HGS_PROFILE_STAGES  every render/backward call records a HIP event pair
 *                       around each stage on the stream it enqueues on;
 *   HGS_PROFILE_WORK    the raster forward also records each pixel's pair
 *                       counts (hgs_state_debug array 9).  This runs a
 *                       slower variant of the forward, so stage times taken
 *                       with it do not time the plain forward.
 * hgs_profile_read synchronises the events and returns the accumulated
 * milliseconds per stage in ms[HGS_N_STAGES] and the number of launches in
 * calls[HGS_N_STAGES] (either may be NULL); reset != 0 clears the totals. */
enum { HGS_PROFILE_STAGES = 1, HGS_PROFILE_WORK = 2 };
enum {
  HGS_STAGE_PREPROCESS = 0,
  HGS_STAGE_SCAN = 1,
  HGS_STAGE_DUPLICATE = 2,
  HGS_STAGE_SORT = 3,
  HGS_STAGE_RANGES = 4,
  HGS_STAGE_RASTER_FWD = 5,
  HGS_STAGE_RASTER_BWD = 6,
  HGS_STAGE_PREPROCESS_BWD = 7,
  HGS_STAGE_FILL = 8,
  HGS_STAGE_DEPTH_SORT = 9,
  HGS_STAGE_FDO_COTANGENTS = 10,
  HGS_STAGE_FDO_PROJECT = 11,
  HGS_STAGE_COLOR_LOSS = 12,
  HGS_STAGE_ADAM = 13,
  HGS_STAGE_DENSIFY = 14,
  HGS_STAGE_FDO_PREPROCESS_BWD = 15,
  HGS_N_STAGES = 16
};
hgs_status hgs_profile_enable(hgs_ctx *ctx, int32_t on);
hgs_status hgs_profile_read(hgs_ctx *ctx, double *ms, int64_t *calls, int32_t reset);

/* Adaptive Type Exchange (Sec. 3.2, Eq. 3; appendix "Effective Rank and
 * Type Switch"), in place on n primitives, enqueued on `stream`.
 *   erank = exp(-sum_i p_i log p_i), p = q / |q|_1, q = (s_x^2, s_y^2, s_z^2),
 *   evaluated in binary64 (all-zero scales give 0 and never switch).
 *   A 3D primitive (type != 0) with erank < theta_e becomes 2D (type 0).
 *   Before that its least significant scale is moved to z, with the
 *   covariance unchanged: S* = P S P^T, R* = R P^T, P = P_x when s_x is the
 *   least, P_y when s_y is (no change when s_z is a least; ties: z, then y).
 *   The rotation is rewritten as q (x) quaternion(P^T), which has the length
 *   of q.  A 2D primitive with erank > theta_e becomes 3D (type 1), all
 *   parameters kept.  The paper uses theta_e = 2.05.
 * scales f32[n,3] (activated), rotations f32[n,4] (wxyz, 16-byte aligned),
 * types u8[n]: device, modified in place.  counts: device u32[2] or NULL;
 * [0] += number switched 3D->2D, [1] += number switched 2D->3D.
 * theta_e is binary64, the precision of the decision (2.05 has no binary32
 * value).  Overlapping calls on the same arrays race.
 * Errors: EINVAL (n < 0 or n > (2^31 - 1) * 256, NULL arrays with n > 0,
 * misaligned rotations, non-finite theta_e), EHIP. */
hgs_status hgs_type_exchange(hgs_ctx *ctx, int64_t n, float *scales, float *rotations,
                             uint8_t *types, double theta_e, uint32_t *counts, void *stream);

/* ---------------------------------------------------------------------
 * Frequency-Decoupled Optimization (Sec. 3.3, Alg. 1; appendices on the
 * discrete wavelet transform and on gradient conflicts).
 * ------------------------------------------------------------------- */

/* Frequency losses of a rendered RGB image against a target and their
 * weighted cotangents.  Level-1 Haar DWT (l = (1,1)/sqrt 2, h = (1,-1)/sqrt 2)
 * of each [H, W] plane, zero-padded to even size: LL, LH (rows differ), HL
 * (columns differ), HH.  L_low = mean over LL of (I^ - I)^2 in the band,
 * L_high = the same mean for LH, HL and HH, summed.  Every band has
 * n = n_views * 3 * ceil(H/2) * ceil(W/2) elements.
 *   grad_low  = lambda_low  * dL_low  / dI^   [n_views, 3, H, W]
 *   grad_high = lambda_high * dL_high / dI^   [n_views, 3, H, W]
 *   losses[0] += L_low, losses[1] += L_high   (unweighted, binary64)
 * The paper uses lambda_low = 0.2, lambda_high = 0.4.  render_rgb and
 * target_rgb: device f32 [n_views, 3, H, W].  grad_low, grad_high: device,
 * overwritten, either may be NULL.  losses: device double[2], 8-byte
 * aligned, or NULL.  Errors: EINVAL (negative sizes, NULL images with a
 * non-empty size, non-finite lambdas, misaligned losses), EHIP. */
hgs_status hgs_fdo_cotangents(hgs_ctx *ctx, int32_t n_views, int32_t height, int32_t width,
                              const float *render_rgb, const float *target_rgb, double lambda_low,
                              double lambda_high, float *grad_low, float *grad_high,
                              double *losses, void *stream);

/* Alg. 1 for n primitives.  Inputs: the parameter gradients of the colour
 * loss, the low-frequency loss and the high-frequency loss.  Each is an
 * hgs_grads of device arrays shaped like hgs_scene_desc (sh with
 * (sh_degree+1)^2 coefficients); a NULL array is zero.  g_i is the
 * concatenation (means, scales, rotations, opacity, SH) of primitive i.
 * If g_low . g_high < 0 (binary64 dot product), a 2D primitive (types[i]
 * == 0) replaces g_high by its projection onto the normal of g_low (Eq. 9),
 * and a 3D one replaces g_low by its projection onto the normal of g_high
 * (Eq. 10).  The update g_color + g_low + g_high is written to `update`
 * (update->accumulate != 0 adds; a NULL array there is not written).
 * n_conflict: device u32, += number of conflicting primitives, or NULL.
 * Errors: EINVAL (NULL structs, n < 0, sh_degree outside 0..3, NULL types
 * with n > 0), EHIP. */
hgs_status hgs_fdo_project(hgs_ctx *ctx, int64_t n, int32_t sh_degree, const uint8_t *types,
                           const hgs_grads *g_color, const hgs_grads *g_low,
                           const hgs_grads *g_high, const hgs_grads *update, uint32_t *n_conflict,
                           void *stream);

/* The backward of Alg. 1's three losses in one reverse traversal.  The
 * cotangent sets are grad_color (all channels, like hgs_render_backward),
 * grad_low_rgb and grad_high_rgb (device f32 [V,3,H,W] RGB cotangents,
 * e.g. from hgs_fdo_cotangents; NULL = zero).  Each record is fetched and
 * each pair's geometry and transmittance recomputed once for all three.
 * The three parameter-gradient sets are formed per primitive, summed over
 * the views, and combined by Alg. 1 (as hgs_fdo_project, with the scene's
 * types) into `update`.  sets: NULL (workspace), or hgs_grads[3] whose
 * arrays receive g_color, g_low, g_high before the projection
 * (overwritten; every array required unless the scene is empty).
 * n_conflict as in
 * hgs_fdo_project.  With one view and sets == NULL the three sets are not
 * stored: per primitive, g_low and g_high are formed (rounded to binary32
 * as stored gradients would be) for Alg. 1's dot products and weights, and
 * the backward is then applied once to the slots combined in binary64
 * with those weights (the backward is linear in them); the update is
 * rounded once.  The scene's parameters must be
 * unchanged since the forward.
 * Errors: EINVAL, ESTATE, ENOMEM, EHIP. */
hgs_status hgs_render_backward_fdo(hgs_ctx *ctx, hgs_state *state,
                                   const hgs_grad_images *grad_color, const float *grad_low_rgb,
                                   const float *grad_high_rgb, const hgs_grads *update,
                                   const hgs_grads *sets, uint32_t *n_conflict, void *stream);

/* ---------------------------------------------------------------------
 * Training step: the colour loss (Sec. 3.3) and the optimizer.
 * ------------------------------------------------------------------- */

/* L_color = (1 - lambda) L1 + lambda D-SSIM of a rendered RGB image against
 * a target, the appearance loss the paper takes from 3DGS (Sec. 3.3):
 * L1 = mean |I^ - I|, D-SSIM = 1 - mean SSIM, SSIM per pixel and channel
 * with an 11 x 11 Gaussian window (sigma 1.5, zero padding, same size),
 * C1 = 0.01^2, C2 = 0.03^2.  render_rgb, target_rgb: device f32
 * [n_views, 3, H, W].  grad: device f32, same shape, receives dL_color/dI^
 * (overwritten), or NULL.  losses: device double[2] (8-byte aligned) or
 * NULL; losses[0] += L1, losses[1] += D-SSIM.  lambda_dssim = 0.2 in 3DGS.
 * Uses a pooled workspace of 12 bytes per pixel and channel.
 * Errors: EINVAL (negative sizes, NULL images with a non-empty size,
 * lambda outside [0, 1], misaligned losses), ENOMEM, EHIP. */
hgs_status hgs_color_loss(hgs_ctx *ctx, int32_t n_views, int32_t height, int32_t width,
                          const float *render_rgb, const float *target_rgb, double lambda_dssim,
                          float *grad, double *losses, void *stream);

/* The colour loss of hgs_color_loss (same arguments, same kernels, same
 * results) for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc.  Its derivative maps live in one fixed device array of
 * 3 * HGS_NOALLOC_MAX_ELEMS floats (96 MiB) that each GPU the library runs on
 * holds until the process ends; the call allocates nothing and calls no
 * allocating routine.  n_views * 3 * height * width must not exceed
 * HGS_NOALLOC_MAX_ELEMS (one 1920x1080 RGB view fits), else ECAPACITY.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (other streams, other contexts, other host threads) race and must be
 * ordered by the caller.  Nothing in the array needs to start at zero (the
 * maps are written in full before they are read).  Errors: as
 * hgs_color_loss, plus ECAPACITY; ESTATE if the array of ctx's device could
 * not be resolved when ctx was created. */
#define HGS_NOALLOC_MAX_ELEMS 8388608
hgs_status hgs_color_loss_noalloc(hgs_ctx *ctx, int32_t n_views, int32_t height, int32_t width,
                                  const float *render_rgb, const float *target_rgb,
                                  double lambda_dssim, float *grad, double *losses, void *stream);

/* Adam hyper-parameters: learning rates per parameter group (SH DC and the
 * higher SH coefficients apart), betas, eps and the 1-based step count used
 * for bias correction.  The betas are binary64 so that 1 - beta (1e-3 for
 * beta2 = 0.999) is exact to binary32 rounding; 0.999 itself has no
 * binary32 value close enough for that. */
typedef struct {
  float lr_means, lr_scales, lr_rotations, lr_opacities, lr_sh_dc, lr_sh_rest;
  double beta1, beta2, eps;
  int32_t step;
} hgs_adam_opts;

/* One Adam step (Kingma and Ba) on n primitives' raw parameters: means,
 * log-scales, quaternions, opacity logits and SH ((sh_degree+1)^2
 * coefficients), each array shaped like hgs_scene_desc's.  grads are the
 * gradients with respect to the activated values the renderer uses
 * (hgs_render_backward's output, or an FDO update); the step applies the
 * chain dL/ds_raw = exp(s_raw) dL/ds and dL/dalpha_raw =
 * sigmoid'(alpha_raw) dL/dalpha.  raw, exp_avg and exp_avg_sq are updated
 * in place; activated (may be NULL, and any of its arrays may be NULL)
 * receives exp(s_raw), sigmoid(alpha_raw) and copies of the others, so it
 * can be the scene the renderer reads.  A NULL raw array is skipped; a
 * non-NULL one needs its gradient and both moments.  The accumulate flags
 * are ignored.  Errors: EINVAL, EHIP. */
hgs_status hgs_adam_step(hgs_ctx *ctx, int64_t n, int32_t sh_degree, const hgs_grads *raw,
                         const hgs_grads *grads, const hgs_grads *exp_avg,
                         const hgs_grads *exp_avg_sq, const hgs_grads *activated,
                         const hgs_adam_opts *opts, void *stream);

/* Densification statistics of 3DGS (the paper adopts its densification,
 * appendix "Implementation Details") for the last backward run on `state`
 * (hgs_render_backward or hgs_render_backward_fdo; with FDO, of the sum
 * of the three losses).  Per view in which splat g is not culled:
 *   grad_norm[g] += |dL/d delta| in NDC units, delta a translation of the
 *                   splat's screen footprint ((W/2, H/2) times the pixel
 *                   gradient);
 *   count[g]     += 1.
 * grad_norm, count: device f32 [N] (either may be NULL), added into.
 * Errors: EINVAL, ESTATE (no backward yet, other context), EHIP. */
hgs_status hgs_densify_stats(hgs_ctx *ctx, hgs_state *state, float *grad_norm, float *count,
                             void *stream);

/* ---------------------------------------------------------------------
 * Batched serving.
 *
 * A server renders forward-only requests against resident scenes (scenes
 * created with hgs_scene_init; copy_resident = 1 keeps them valid whatever
 * the caller does with its own buffers).  Each request is one camera of
 * any image size.  Pending requests are admitted into "lanes" (batches in
 * flight) as a lane frees up, within the lane's slot count and memory
 * capacities.  A lane renders all its requests in one pipeline pass:
 * instance ids and tile ids of all requests share one key space (per-request
 * instance and tile offsets), and one persistent raster grid pulls
 * (tile, quadrant) units from an atomic queue.  The pass reads its batch from
 * a device-side slot table and keeps every count on the device (capacity-
 * bounded, no host synchronisation), so with use_graph = 1 it is captured
 * once per lane as a hipGraph and replayed for every batch.  Lanes run on
 * their own streams (default priority), so the batches in flight overlap on
 * the device.  A request's images are the same as hgs_render's for the same
 * scene, camera and opts (each pixel's pair list is the same list in the
 * same order).
 *
 * If a batch produces more (tile, splat) pairs than max_pairs, its requests
 * are rendered again one by one with hgs_render on the lane's stream before
 * they complete (counted in the stats); results are unaffected.
 * ------------------------------------------------------------------- */
typedef struct hgs_server hgs_server;

typedef struct {
  int32_t max_requests;  /* requests per batch (slot table size), >= 1 */
  int32_t max_batches;   /* lanes: batches in flight, >= 1 */
  int64_t max_instances; /* sum of the scene sizes of one batch, >= 1 */
  int64_t max_pairs;     /* (tile, splat) pairs of one batch, >= 1, < 2^32 */
  int64_t max_tiles;     /* 16x16 tiles of one batch, >= 1, < 2^31 */
  int32_t use_graph;     /* 1: capture each lane's pass once as a hipGraph */
} hgs_server_config;

typedef struct {
  int32_t scene_id;
  hgs_camera camera;     /* [host] copied at submit */
  hgs_images out;        /* device, [1,3,H,W] / [1,1,H,W]; NULL channels are
                            not written; must stay valid until completion */
  uint64_t tag;          /* returned by hgs_server_poll on completion */
} hgs_request;

/* Creates a server on ctx's device.  All lane buffers are allocated here
 * (nothing is allocated per batch).  `opts` [host] may be NULL.  Errors:
 * EINVAL on a bad config, ENOMEM, EHIP. */
hgs_status hgs_server_create(hgs_ctx *ctx, const hgs_server_config *cfg, const hgs_opts *opts,
                             hgs_server **out);
/* Waits for the batches in flight, then frees the server. */
void hgs_server_destroy(hgs_server *server);
/* Queues a request (host only; nothing is launched).  EINVAL for a bad
 * scene id or camera, ECAPACITY for a request that exceeds one batch's
 * capacities on its own. */
hgs_status hgs_server_submit(hgs_server *server, const hgs_request *req /* [host] */);
/* Makes progress without blocking: retires the lanes whose batch has
 * finished (their tags go to done_tags [host], up to `capacity`; the rest
 * are returned by later calls), then admits pending requests in arrival
 * order into free lanes and launches them.  *n_done = tags written. */
hgs_status hgs_server_poll(hgs_server *server, uint64_t *done_tags /* [host] */,
                           int32_t capacity, int32_t *n_done /* [host] */);
/* Counters [host]: [0] batches launched, [1] requests completed,
 * [2] requests re-rendered after a pair overflow, [3] requests pending,
 * [4] lanes busy, [5] largest pair count seen in a batch. */
hgs_status hgs_server_stats(hgs_server *server, int64_t *stats6 /* [host] */);

/* Message of the last error on this host thread ("" if none). */
const char *hgs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HGS_H */
