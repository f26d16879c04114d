// C ABI of the hybrid rasterizer: argument validation, workspace management
// and the launch sequence.  Declarations and contracts are in include/hgs.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx_internal.h"

using namespace hgs;

namespace hgs {

namespace {
thread_local std::string g_err;
}  // namespace

hgs_status fail(hgs_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

}  // namespace hgs

struct hgs_state {
  hipStream_t stream = nullptr;
  int device = 0;
  SceneDev scene{};
  int V = 0;
  int64_t N = 0;
  int W = 0, H = 0, tiles_x = 0, tiles_y = 0, tiles_per_view = 0, n_tiles = 0;
  DevOpts opt{};
  std::vector<DevCam> cams_host;
  DevCam *cams = nullptr;
  Record *rec = nullptr;
  uint32_t *tiles = nullptr, *zbits = nullptr, *offsets = nullptr;
  int4 *rect = nullptr;
  uint8_t *flags = nullptr;
  uint64_t *total = nullptr;     // device: pair count D (the scan total)
  uint32_t *overflow = nullptr;  // device: bit 0 D exceeded the pair capacity, bit 1 sort error
  int64_t cap = 0;               // pair capacity of this render
  bool overflowed = false;
  bool sort_failed = false;      // a radix pass's look-back gave up (never expected)
  bool has_wcount = false;       // the forward recorded the pair counts (profiling on)
  uint64_t *bmask = nullptr;  // blend masks of the forward (raster_mask_words)
  uint32_t *keys = nullptr;  // tile id of each sorted pair
  uint32_t *vals = nullptr;  // instance id (view * N + splat) of each sorted pair
  uint2 *ranges = nullptr;
  uint32_t *order = nullptr;  // tiles by pair-list length, longest first
  uint2 *vis = nullptr;       // per tile: the forward's largest blended count per wave
  uint32_t *order_bwd = nullptr;  // tiles by that count, largest first (the backward's)
  float *T_final = nullptr;
  uint32_t *last = nullptr, *n_contrib = nullptr, *wcount = nullptr;
  int64_t D = -1;        // pairs in the sorted list, min(D_total, cap), once read back
  int64_t D_total = -1;  // pairs the render produced (may exceed cap)
  // accumulator planes of the last backward on this state (workspace arena 2)
  const float *accum_last = nullptr;
  int accum_planes = 0;
  int64_t accum_plane = 0;
  Workspace *ws = nullptr;
  std::vector<std::pair<void **, size_t>> plan;  // buffers awaiting commit()
};

namespace {

hipEvent_t pool_event(hgs_ctx *c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches of one stage with events when profiling is on.
struct StageTimer {
  hgs_ctx *c;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr;
  StageTimer(hgs_ctx *ctx, int st, hipStream_t stream) : c(ctx), stage(st), s(stream) {
    if (!c->profile) return;
    a = pool_event(c);
    if (a) (void)hipEventRecord(a, s);
  }
  ~StageTimer() {
    if (!c->profile || !a) return;
    hipEvent_t b = pool_event(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->pending.push_back(StageEvent{stage, a, b});
  }
};

// Buffers are planned with dalloc and placed by commit() in one arena of
// the state's workspace (256-byte aligned), growing the arena if needed
// (never under graph capture: no_grow).
hipError_t dalloc(hgs_state *st, void **p, size_t bytes) {
  st->plan.push_back({p, bytes == 0 ? 256 : bytes});
  *p = nullptr;
  return hipSuccess;
}

template <typename T>
hipError_t dalloc_t(hgs_state *st, T **p, size_t count) {
  return dalloc(st, reinterpret_cast<void **>(p), count * sizeof(T));
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Pair capacity for an observed pair count: half again of headroom.
int64_t grow_cap(uint64_t D) {
  const uint64_t c = D + D / 2 + 65536;
  return (int64_t)(c < 0xffffffffull ? c : 0xffffffffull);
}

hipError_t commit(hgs_state *st, int which, hipStream_t s, bool no_grow = false) {
  size_t total = 0;
  for (auto &it : st->plan) total += align256(it.second);
  Arena &A = st->ws->arena[which];
  if (A.cap < total && no_grow) {
    st->plan.clear();
    return hipErrorNotSupported;  // a captured call may not allocate
  }
  if (A.cap < total) {
    if (A.buf) {
      const hipError_t e = hipFreeAsync(A.buf, s);
      A.buf = nullptr;
      A.cap = 0;
      if (e != hipSuccess) return e;
    }
    const size_t cap = std::max(total, A.cap + A.cap / 2);
    const hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&A.buf), cap, s);
    if (e != hipSuccess) {
      st->plan.clear();
      return e;
    }
    A.cap = cap;
  }
  size_t off = 0;
  for (auto &it : st->plan) {
    *it.first = A.buf + off;
    off += align256(it.second);
  }
  st->plan.clear();
  return hipSuccess;
}

hipError_t acquire_ws(hgs_ctx *ctx, hgs_state *st) {
  Workspace *w = nullptr;
  if (!ctx->ws_free.empty()) {
    w = ctx->ws_free.back();
    ctx->ws_free.pop_back();
  } else {
    w = new (std::nothrow) Workspace();
    if (!w) return hipErrorOutOfMemory;
    ctx->ws_all.push_back(w);
  }
  st->ws = w;
  if (w->has_ready && w->stream != st->stream) return hipStreamWaitEvent(st->stream, w->ready, 0);
  return hipSuccess;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

void release(hgs_ctx *ctx, hgs_state *st) {
  if (!st || !st->ws) return;
  Workspace *w = st->ws;
  st->ws = nullptr;
  if (capturing(st->stream)) {
    // no host-side stream work under capture: the next user of this
    // workspace must use the same stream
    w->stream = st->stream;
    w->has_ready = false;
    ctx->ws_free.push_back(w);
    return;
  }
  if (!w->ready && hipEventCreateWithFlags(&w->ready, hipEventDisableTiming) != hipSuccess)
    w->ready = nullptr;
  if (w->ready && hipEventRecord(w->ready, st->stream) == hipSuccess) {
    w->stream = st->stream;
    w->has_ready = true;
  } else {
    (void)hipStreamSynchronize(st->stream);
    w->has_ready = false;
  }
  ctx->ws_free.push_back(w);
}

}  // namespace

namespace hgs {

DevOpts to_dev_opts(const hgs_opts *o) {
  DevOpts d{};
  if (o) {
    for (int i = 0; i < 3; ++i) d.bg[i] = o->bg[i];
    d.dilation = o->dilation;
    d.lambda_z = o->lambda_z;
    d.theta_z = o->theta_z;
    d.temp_z = o->temp_z;
    d.alpha_min = o->alpha_min;
    d.alpha_max = o->alpha_max;
    d.t_min = o->t_min;
    d.out_mask = o->out_mask;
  } else {
    d.dilation = 0.3f;
    d.lambda_z = 1.0f;
    d.theta_z = 1.05f;
    d.temp_z = 0.001f;
    d.alpha_min = 1.0f / 255.0f;
    d.alpha_max = 0.99f;
    d.t_min = 1e-4f;
    d.out_mask = 0u;
  }
  // radius^2 of the support of an opaque splat, 2 ln(1 / alpha_min), rounded
  // up to binary32 so the screen rectangle never undercuts it
  const double r = 2.0 * std::log(1.0 / (double)d.alpha_min);
  float f = (float)r;
  if ((double)f < r) f = std::nextafter(f, INFINITY);
  d.rr0 = f;
  d.inv_amin = (float)(1.0 / (double)d.alpha_min);
  return d;
}

hgs_status check_opts(const hgs_opts *o) {
  if (!o) return HGS_OK;
  if (!(o->dilation >= 0.0f && std::isfinite(o->dilation) && o->temp_z > 0.0f &&
        std::isfinite(o->lambda_z) && std::isfinite(o->theta_z) && std::isfinite(o->temp_z) &&
        std::isfinite(o->bg[0]) && std::isfinite(o->bg[1]) && std::isfinite(o->bg[2])))
    return fail(HGS_EINVAL, "bad opts (dilation >= 0, temp_z > 0, all finite)");
  if (!(o->alpha_min > 0.0f && o->alpha_min <= o->alpha_max && o->alpha_max < 1.0f))
    return fail(HGS_EINVAL, "bad opts: need 0 < alpha_min <= alpha_max < 1");
  if (!(o->t_min > 0.0f && o->t_min < 1.0f))
    return fail(HGS_EINVAL, "bad opts: need 0 < t_min < 1");
  if (o->out_mask & ~0xfu) return fail(HGS_EINVAL, "bad opts: out_mask has bits above 3");
  return HGS_OK;
}

bool make_dev_cam(const hgs_camera &c, DevCam &d, int view, std::string &why) {
  std::memset(&d, 0, sizeof(d));
  for (int i = 0; i < 12; ++i) {
    d.V[i] = c.viewmat[i];
    d.Vd[i] = c.viewmat[i];
  }
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(c.viewmat[i])) {
      why = "camera " + std::to_string(view) + ": non-finite viewmat";
      return false;
    }
  d.fx = c.fx;
  d.fy = c.fy;
  d.cx = c.cx;
  d.cy = c.cy;
  d.znear = c.znear;
  d.W = c.width;
  d.H = c.height;
  if (!(std::isfinite(c.fx) && std::isfinite(c.fy) && c.fx != 0.0f && c.fy != 0.0f &&
        std::isfinite(c.cx) && std::isfinite(c.cy))) {
    why = "camera " + std::to_string(view) + ": bad intrinsics";
    return false;
  }
  if (!(c.znear > 0.0f) || !std::isfinite(c.znear)) {
    why = "camera " + std::to_string(view) + ": znear must be > 0";
    return false;
  }
  if (c.width < 1 || c.width > 16384 || c.height < 1 || c.height > 16384) {
    why = "camera " + std::to_string(view) + ": width/height must be in [1, 16384]";
    return false;
  }
  d.tiles_x = (c.width + kTile - 1) / kTile;
  d.tiles_y = (c.height + kTile - 1) / kTile;
  const double *R = d.Vd;  // rows 0..2, stride 4
  auto r = [&](int i, int j) { return R[4 * i + j]; };
  const double det = r(0, 0) * (r(1, 1) * r(2, 2) - r(1, 2) * r(2, 1)) -
                     r(0, 1) * (r(1, 0) * r(2, 2) - r(1, 2) * r(2, 0)) +
                     r(0, 2) * (r(1, 0) * r(2, 1) - r(1, 1) * r(2, 0));
  if (!(std::fabs(det) > 1e-12)) {
    why = "camera " + std::to_string(view) + ": singular rotation";
    return false;
  }
  double *Ri = d.Vinv;
  Ri[0] = (r(1, 1) * r(2, 2) - r(1, 2) * r(2, 1)) / det;
  Ri[1] = (r(0, 2) * r(2, 1) - r(0, 1) * r(2, 2)) / det;
  Ri[2] = (r(0, 1) * r(1, 2) - r(0, 2) * r(1, 1)) / det;
  Ri[3] = (r(1, 2) * r(2, 0) - r(1, 0) * r(2, 2)) / det;
  Ri[4] = (r(0, 0) * r(2, 2) - r(0, 2) * r(2, 0)) / det;
  Ri[5] = (r(0, 2) * r(1, 0) - r(0, 0) * r(1, 2)) / det;
  Ri[6] = (r(1, 0) * r(2, 1) - r(1, 1) * r(2, 0)) / det;
  Ri[7] = (r(0, 1) * r(2, 0) - r(0, 0) * r(2, 1)) / det;
  Ri[8] = (r(0, 0) * r(1, 1) - r(0, 1) * r(1, 0)) / det;
  const double t[3] = {R[3], R[7], R[11]};
  for (int i = 0; i < 3; ++i) d.o[i] = -(Ri[3 * i] * t[0] + Ri[3 * i + 1] * t[1] + Ri[3 * i + 2] * t[2]);
  return true;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

hgs_status check_desc(const hgs_scene_desc *d) {
  if (!d) return fail(HGS_EINVAL, "scene desc is NULL");
  if (d->n < 0) return fail(HGS_EINVAL, "scene n < 0");
  if (d->n > (int64_t)0x7fffffff) return fail(HGS_EINVAL, "scene n too large");
  if (d->sh_degree < 0 || d->sh_degree > 3) return fail(HGS_EINVAL, "sh_degree must be 0..3");
  if (d->n > 0 && (!d->means || !d->scales || !d->rotations || !d->opacities || !d->sh || !d->types))
    return fail(HGS_EINVAL, "scene array pointer is NULL");
  if (!aligned(d->means, 4) || !aligned(d->scales, 4) || !aligned(d->rotations, 4) ||
      !aligned(d->opacities, 4) || !aligned(d->sh, 4))
    return fail(HGS_EINVAL, "scene float arrays must be 4-byte aligned");
  return HGS_OK;
}

// Synchronises the state's stream and reads its pair count and overflow
// flag once.
hipError_t read_pairs(hgs_state *st, bool &over) {
  if (st->D < 0) {
    hipError_t e = hipStreamSynchronize(st->stream);
    if (e != hipSuccess) return e;
    uint64_t tot = 0;
    uint32_t ov = 0;
    e = hipMemcpy(&tot, st->total, sizeof(tot), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&ov, st->overflow, sizeof(ov), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    st->D_total = (int64_t)tot;
    st->D = std::min<int64_t>((int64_t)tot, st->cap);
    st->overflowed = (ov & 1u) != 0 || (int64_t)tot > st->cap;
    st->sort_failed = (ov & 2u) != 0;
  }
  over = st->overflowed;
  return hipSuccess;
}

}  // namespace hgs

extern "C" {

const char *hgs_last_error(void) { return g_err.c_str(); }

hgs_status hgs_create(int32_t device, hgs_ctx **out) {
  if (!out) return fail(HGS_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HGS_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(HGS_EINVAL, "no such device");
  HGS_HIP(hipSetDevice(device));
  hipMemPool_t pool;
  HGS_HIP(hipDeviceGetDefaultMemPool(&pool, device));
  uint64_t thr = UINT64_MAX;
  HGS_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
  int cus = 0;
  HGS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  // the fixed array of hgs_color_loss_noalloc on this device
  HGS_HIP(noalloc_setup(device));
  hgs_ctx *c = new (std::nothrow) hgs_ctx();
  if (!c) return fail(HGS_ENOMEM, "host allocation failed");
  c->device = device;
  c->n_cu = cus > 0 ? cus : 1;
  *out = c;
  return HGS_OK;
}

void hgs_destroy(hgs_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto &s : ctx->scenes)
    if (s.used && s.buf) (void)hipFree(s.buf);
  for (auto &p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  for (Workspace *w : ctx->ws_all) {
    for (Arena &a : w->arena)
      if (a.buf) (void)hipFree(a.buf);
    if (w->ready) (void)hipEventDestroy(w->ready);
    if (w->status_ev) (void)hipEventDestroy(w->status_ev);
    if (w->status_host) (void)hipHostFree(w->status_host);
    delete w;
  }
  delete ctx;
}

hgs_status hgs_scene_init(hgs_ctx *ctx, const hgs_scene_desc *desc, int32_t copy_resident,
                          int32_t *scene_id) {
  if (!ctx || !scene_id) return fail(HGS_EINVAL, "ctx or scene_id is NULL");
  hgs_status st = check_desc(desc);
  if (st != HGS_OK) return st;
  HGS_HIP(hipSetDevice(ctx->device));
  Scene s;
  s.used = true;
  s.resident = copy_resident != 0;
  s.dev.n = desc->n;
  s.dev.sh_degree = desc->sh_degree;
  const int K = (desc->sh_degree + 1) * (desc->sh_degree + 1);
  if (!s.resident) {
    s.dev.means = desc->means;
    s.dev.scales = desc->scales;
    s.dev.rots = desc->rotations;
    s.dev.opac = desc->opacities;
    s.dev.sh = desc->sh;
    s.dev.types = desc->types;
  } else {
    const size_t n = (size_t)desc->n;
    const size_t fl = n * (3 + 3 + 4 + 1 + 3 * (size_t)K);
    const size_t bytes = fl * sizeof(float) + n + 256;
    void *buf = nullptr;
    HGS_HIP(hipMalloc(&buf, bytes));
    float *f = (float *)buf;
    auto cp = [&](const float *src, size_t cnt) -> float * {
      float *dst = f;
      if (cnt) (void)hipMemcpy(dst, src, cnt * sizeof(float), hipMemcpyDeviceToDevice);
      f += cnt;
      return dst;
    };
    s.dev.means = cp(desc->means, 3 * n);
    s.dev.scales = cp(desc->scales, 3 * n);
    s.dev.rots = cp(desc->rotations, 4 * n);
    s.dev.opac = cp(desc->opacities, n);
    s.dev.sh = cp(desc->sh, 3 * K * n);
    uint8_t *t = (uint8_t *)f;
    if (n) {
      hipError_t e = hipMemcpy(t, desc->types, n, hipMemcpyDeviceToDevice);
      if (e != hipSuccess) {
        (void)hipFree(buf);
        return fail(HGS_EHIP, std::string("copying scene: ") + hipGetErrorString(e));
      }
    }
    s.dev.types = t;
    s.buf = buf;
  }
  for (size_t i = 0; i < ctx->scenes.size(); ++i)
    if (!ctx->scenes[i].used) {
      ctx->scenes[i] = s;
      *scene_id = (int32_t)i;
      return HGS_OK;
    }
  ctx->scenes.push_back(s);
  *scene_id = (int32_t)(ctx->scenes.size() - 1);
  return HGS_OK;
}

hgs_status hgs_scene_release(hgs_ctx *ctx, int32_t scene_id) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].used)
    return fail(HGS_EINVAL, "bad scene id");
  Scene &s = ctx->scenes[scene_id];
  if (s.buf) {
    HGS_HIP(hipSetDevice(ctx->device));
    HGS_HIP(hipDeviceSynchronize());
    HGS_HIP(hipFree(s.buf));
  }
  s = Scene();
  return HGS_OK;
}

hgs_status hgs_render(hgs_ctx *ctx, int32_t scene_id, const hgs_camera *cams, int32_t n_views,
                      const hgs_opts *opts, const hgs_images *out, hgs_state **state_out,
                      void *stream) {
  if (state_out) *state_out = nullptr;
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].used)
    return fail(HGS_EINVAL, "bad scene id");
  if (!cams || n_views < 1) return fail(HGS_EINVAL, "need at least one camera");
  if (n_views > 4096) return fail(HGS_EINVAL, "too many views");
  const Scene &sc = ctx->scenes[scene_id];
  {
    const hgs_status os = check_opts(opts);
    if (os != HGS_OK) return os;
  }
  RasterOut ro{};
  {
    const uint32_t mask = opts ? opts->out_mask : 0u;
    float *const ptr[4] = {out ? out->rgb : nullptr, out ? out->alpha : nullptr,
                           out ? out->depth : nullptr, out ? out->normal : nullptr};
    float *sel[4];
    for (int c = 0; c < 4; ++c) {
      const bool want = mask == 0u ? ptr[c] != nullptr : ((mask >> c) & 1u) != 0u;
      if (want && !ptr[c])
        return fail(HGS_EINVAL, "opts.out_mask selects an output channel whose pointer is NULL");
      sel[c] = want ? ptr[c] : nullptr;
    }
    ro.rgb = sel[0];
    ro.alpha = sel[1];
    ro.depth = sel[2];
    ro.normal = sel[3];
  }
  const int W = cams[0].width, H = cams[0].height;
  hgs_state *st = new (std::nothrow) hgs_state();
  if (!st) return fail(HGS_ENOMEM, "host allocation failed");
  st->stream = (hipStream_t)stream;
  st->device = ctx->device;
  st->scene = sc.dev;
  st->V = n_views;
  st->N = sc.dev.n;
  st->W = W;
  st->H = H;
  st->opt = to_dev_opts(opts);
  st->cams_host.resize(n_views);
  std::string why;
  for (int v = 0; v < n_views; ++v) {
    if (!make_dev_cam(cams[v], st->cams_host[v], v, why)) {
      delete st;
      return fail(HGS_EINVAL, why);
    }
    if (cams[v].width != W || cams[v].height != H) {
      delete st;
      return fail(HGS_EINVAL, "all views of one call must share the image size");
    }
  }
  st->tiles_x = st->cams_host[0].tiles_x;
  st->tiles_y = st->cams_host[0].tiles_y;
  st->tiles_per_view = st->tiles_x * st->tiles_y;
  const int64_t n_tiles = (int64_t)st->tiles_per_view * n_views;
  if (n_tiles > (int64_t)0x7fffffff) {
    delete st;
    return fail(HGS_EINVAL, "too many tiles");
  }
  st->n_tiles = (int)n_tiles;
  for (int v = 0; v < n_views; ++v) st->cams_host[v].tile_base = v * st->tiles_per_view;
  const int64_t VN = (int64_t)n_views * st->N;
  if (VN > (int64_t)0xffffffffLL) {
    delete st;
    return fail(HGS_EINVAL, "views x primitives exceeds 2^32");
  }
  const int64_t P = (int64_t)n_views * W * H;

  auto bail = [&](hgs_status s) {
    const bool cap = capturing(st->stream);
    release(ctx, st);
    if (!cap) (void)hipStreamSynchronize(st->stream);
    delete st;
    return s;
  };
#define ST_HIP(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return bail(fail(e_ == hipErrorOutOfMemory ? HGS_ENOMEM : HGS_EHIP,               \
                       std::string(#expr) + ": " + hipGetErrorString(e_)));             \
  } while (0)

  ST_HIP(hipSetDevice(ctx->device));
  const bool cap_mode = capturing(st->stream);
  if (cap_mode && n_views > kCamsPerUpload * 8) {
    delete st;
    return fail(HGS_EINVAL, "a captured render takes at most 64 views");
  }
  ST_HIP(acquire_ws(ctx, st));
  ST_HIP(dalloc_t(st, &st->cams, (size_t)n_views));
  ST_HIP(dalloc_t(st, &st->rec, (size_t)VN));
  ST_HIP(dalloc_t(st, &st->tiles, (size_t)VN));
  ST_HIP(dalloc_t(st, &st->zbits, (size_t)VN));
  ST_HIP(dalloc_t(st, &st->rect, (size_t)VN));
  // packed tile rectangles, and the same in depth order
  uint32_t *prect = nullptr, *prect_s = nullptr;
  ST_HIP(dalloc_t(st, &prect, (size_t)VN));
  ST_HIP(dalloc_t(st, &prect_s, (size_t)VN));
  ST_HIP(dalloc_t(st, &st->flags, (size_t)VN));
  ST_HIP(dalloc_t(st, &st->offsets, (size_t)VN));
  ST_HIP(dalloc_t(st, &st->total, (size_t)1));
  ST_HIP(dalloc_t(st, &st->overflow, (size_t)1));
  uint32_t *dwords = nullptr, *twords = nullptr;  // digit counts of the two sorts
  ST_HIP(dalloc_t(st, &dwords, (size_t)kSortWords));
  ST_HIP(dalloc_t(st, &twords, (size_t)kSortWords));
  void *scan_tmp = nullptr;
  ST_HIP(dalloc(st, &scan_tmp, scan_tmp_bytes(VN)));
  ST_HIP(dalloc_t(st, &st->ranges, (size_t)n_tiles));
  ST_HIP(dalloc_t(st, &st->order, (size_t)n_tiles));
  ST_HIP(dalloc_t(st, &st->vis, (size_t)n_tiles));
  ST_HIP(dalloc_t(st, &st->order_bwd, (size_t)n_tiles));
  ST_HIP(dalloc_t(st, &st->T_final, (size_t)P));
  ST_HIP(dalloc_t(st, &st->last, (size_t)P));
  ST_HIP(dalloc_t(st, &st->n_contrib, (size_t)P));
  ST_HIP(dalloc_t(st, &st->wcount, (size_t)P));
  // instance depth order: za/oa, zb/ob ping-pong; counts in depth order in cnt
  uint32_t *za = nullptr, *oa = nullptr, *zb = nullptr, *ob = nullptr, *cnt = nullptr;
  void *dsort_tmp = nullptr;
  ST_HIP(dalloc_t(st, &za, (size_t)VN));
  ST_HIP(dalloc_t(st, &oa, (size_t)VN));
  ST_HIP(dalloc_t(st, &zb, (size_t)VN));
  ST_HIP(dalloc_t(st, &ob, (size_t)VN));
  ST_HIP(dalloc_t(st, &cnt, (size_t)VN));
  ST_HIP(dalloc(st, &dsort_tmp, sort_tmp_bytes(VN)));
  ST_HIP(commit(st, 0, st->stream, cap_mode));
  ZeroList zl;  // cleared by the camera upload's launch
  zl.p[0] = st->overflow;
  zl.n[0] = 1;
  zl.p[1] = dwords;
  zl.n[1] = kSortWords;
  zl.p[2] = twords;
  zl.n[2] = kSortWords;
  if (n_views <= kCamsPerUpload * 8) {
    launch_upload_cams(st->cams_host.data(), n_views, st->cams, st->stream, zl);
  } else {
    ST_HIP(hipMemcpyAsync(st->cams, st->cams_host.data(), sizeof(DevCam) * n_views,
                          hipMemcpyHostToDevice, st->stream));
    for (int a = 0; a < ZeroList::kMax; ++a) launch_fill_u32(zl.p[a], 0u, zl.n[a], st->stream);
  }

  {
    StageTimer t(ctx, HGS_STAGE_PREPROCESS, st->stream);
    launch_preprocess(st->scene, st->cams, n_views, st->opt, st->rec, st->tiles, st->zbits,
                      st->rect, st->flags, prect, st->stream);
  }
  const uint32_t *order = nullptr;
  {
    // instances in depth order; the last pass also gathers their tile counts
    // (and packed rectangles).  Culled instances have key 0 and no pairs, so
    // their place in the order does not matter (zero_free)
    StageTimer t(ctx, HGS_STAGE_DEPTH_SORT, st->stream);
    const int w = launch_radix_sort(st->zbits, nullptr, za, oa, zb, ob, VN, 32, dsort_tmp,
                                    st->stream, nullptr, prect, cnt, st->overflow, dwords,
                                    prect_s, st->tiles, /*zero_free=*/true);
    order = w ? ob : oa;
  }
  {
    StageTimer t(ctx, HGS_STAGE_SCAN, st->stream);
    launch_scan(cnt, st->offsets, VN, st->total, scan_tmp, st->stream);
  }
  // pair capacity: fixed, or learned by this workspace (see Workspace)
  Workspace *ws = st->ws;
  int64_t cap = ctx->pair_cap;
  if (cap <= 0) {
    if (ws->shape_vn != VN || ws->shape_tiles != n_tiles) ws->pair_cap = 0;
    if (!cap_mode && ws->pair_cap > 0 && ws->status_pending &&
        hipEventQuery(ws->status_ev) == hipSuccess) {
      ws->status_pending = false;
      const uint64_t last = ws->status_host[0];
      if ((double)last > 0.8 * (double)ws->pair_cap) ws->pair_cap = grow_cap(last);
    }
    if (ws->pair_cap <= 0) {
      if (cap_mode)
        return bail(fail(HGS_EINVAL, "a captured render needs a known pair capacity: render "
                                     "once outside capture or call hgs_set_pair_capacity"));
      uint64_t Dh = 0;
      ST_HIP(hipMemcpyAsync(&Dh, st->total, sizeof(uint64_t), hipMemcpyDeviceToHost, st->stream));
      ST_HIP(hipStreamSynchronize(st->stream));
      ST_HIP(hipGetLastError());
      if (Dh > 0xffffffffull)
        return bail(fail(HGS_ECAPACITY, "more than 2^32-1 (tile, splat) pairs"));
      ws->pair_cap = grow_cap(Dh);
      ws->shape_vn = VN;
      ws->shape_tiles = n_tiles;
      ws->status_pending = false;
    }
    cap = ws->pair_cap;
  }
  st->cap = cap;

  uint32_t *ka = nullptr, *va = nullptr, *kb = nullptr, *vb = nullptr;
  void *sort_tmp = nullptr;
  ST_HIP(dalloc_t(st, &ka, (size_t)cap));
  ST_HIP(dalloc_t(st, &va, (size_t)cap));
  ST_HIP(dalloc_t(st, &kb, (size_t)cap));
  ST_HIP(dalloc_t(st, &vb, (size_t)cap));
  ST_HIP(dalloc(st, &sort_tmp, sort_tmp_bytes(cap)));
  ST_HIP(dalloc_t(st, &st->bmask, (size_t)raster_mask_words(cap, n_tiles)));
  ST_HIP(commit(st, 1, st->stream, cap_mode));
  {
    StageTimer t(ctx, HGS_STAGE_DUPLICATE, st->stream);
    // (also clears the tile ranges the ranges kernel fills in)
    launch_duplicate(order, st->offsets, st->tiles, st->rect, prect_s, st->cams, n_views, st->N,
                     (uint64_t)cap, kb, vb, st->overflow,
                     reinterpret_cast<uint32_t *>(st->ranges), 2 * n_tiles, st->stream);
  }
  int tile_bits = 0;
  while ((int64_t(1) << tile_bits) < n_tiles) ++tile_bits;
  {
    StageTimer t(ctx, HGS_STAGE_SORT, st->stream);
    const int w = launch_radix_sort(kb, vb, ka, va, kb, vb, cap, tile_bits, sort_tmp,
                                    st->stream, st->total, nullptr, nullptr, st->overflow, twords);
    st->keys = w ? kb : ka;
    st->vals = w ? vb : va;
  }
  // the pair count of this render, for the next render on this workspace:
  // written to mapped pinned memory by the tile-order launch, read by the
  // host once the event recorded after the forward has fired (no wait)
  uint64_t *status_dst = nullptr;
  if (!cap_mode && ctx->pair_cap <= 0) {
    if (!ws->status_host) {
      void *h = nullptr;
      ST_HIP(hipHostMalloc(&h, 2 * sizeof(uint64_t), hipHostMallocMapped | hipHostMallocCoherent));
      ws->status_host = static_cast<uint64_t *>(h);
      void *d = nullptr;
      ST_HIP(hipHostGetDevicePointer(&d, h, 0));
      ws->status_dev = static_cast<uint64_t *>(d);
    }
    status_dst = ws->status_dev;
  }
  {
    StageTimer t(ctx, HGS_STAGE_RANGES, st->stream);
    launch_ranges(st->keys, cap, st->ranges, st->stream, st->total);
    launch_tile_order(st->ranges, (int)n_tiles, st->order, st->stream, nullptr, nullptr,
                      st->total, status_dst, st->vis);
  }

  ro.T_final = st->T_final;
  ro.last = st->last;
  ro.n_contrib = st->n_contrib;
  ro.wcount = ctx->work_acct ? st->wcount : nullptr;  // work accounting on request
  ro.vis = st->vis;
  st->has_wcount = ctx->work_acct;
  {
    StageTimer t(ctx, HGS_STAGE_RASTER_FWD, st->stream);
    launch_raster_fwd(st->ranges, st->order, st->vals, st->rec, st->n_tiles, W, H,
                      st->tiles_x, st->tiles_per_view, st->opt, ro, st->bmask, st->stream);
  }
  if (status_dst) {
    if (!ws->status_ev) ST_HIP(hipEventCreateWithFlags(&ws->status_ev, hipEventDisableTiming));
    ST_HIP(hipEventRecord(ws->status_ev, st->stream));
    ws->status_pending = true;
  }
  ST_HIP(hipGetLastError());
#undef ST_HIP
  if (state_out) {
    *state_out = st;
  } else {
    release(ctx, st);
    delete st;
  }
  return HGS_OK;
}

// Orders `waiter` after the work enqueued so far on `signaler`.
hipError_t join_streams(hipStream_t waiter, hipStream_t signaler) {
  if (waiter == signaler) return hipSuccess;
  hipEvent_t ev;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev, signaler);
  if (e == hipSuccess) e = hipStreamWaitEvent(waiter, ev, 0);
  const hipError_t e2 = hipEventDestroy(ev);
  return e != hipSuccess ? e : e2;
}

hgs_status hgs_render_backward(hgs_ctx *ctx, hgs_state *st, const hgs_grad_images *gout,
                               const hgs_grads *grads, void *stream) {
  if (!ctx || !st) return fail(HGS_EINVAL, "ctx or state is NULL");
  if (!grads) return fail(HGS_EINVAL, "grads is NULL");
  if (st->device != ctx->device) return fail(HGS_ESTATE, "state belongs to another context");
  HGS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (s != st->stream) {
    // order this stream after the forward's work
    hipEvent_t ev;
    HGS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HGS_HIP(hipEventRecord(ev, st->stream));
    HGS_HIP(hipStreamWaitEvent(s, ev, 0));
    HGS_HIP(hipEventDestroy(ev));
  }
  const int64_t VN = (int64_t)st->V * st->N;
  if (!st->ws) return fail(HGS_ESTATE, "state has no workspace");
  float *accum = nullptr;
  HGS_HIP(dalloc_t(st, &accum, (size_t)std::max<int64_t>(VN, 1) * kGradSlots));
  HGS_HIP(commit(st, 2, s, capturing(s)));
  {
    // the accumulators cleared beside the backward's tile order (by the
    // forward waves' blended counts, largest first)
    StageTimer t(ctx, HGS_STAGE_FILL, s);
    launch_order_and_clear(st->vis, (int)st->n_tiles, st->order_bwd, accum, VN * kGradSlots, s);
  }
  RasterGradIn gi{};
  if (gout) {
    gi.rgb = gout->rgb;
    gi.alpha = gout->alpha;
    gi.depth = gout->depth;
    gi.normal = gout->normal;
  }
  {
    StageTimer t(ctx, HGS_STAGE_RASTER_BWD, s);
    launch_raster_bwd(st->ranges, st->order_bwd, st->vals, st->rec, st->n_tiles, st->W, st->H,
                      st->tiles_x,
                      st->tiles_per_view, st->opt, st->T_final, st->last, st->bmask, gi, accum,
                      s);
  }
  st->accum_last = accum;
  st->accum_planes = 1;
  st->accum_plane = VN * kGradSlots;
  {
    StageTimer t(ctx, HGS_STAGE_PREPROCESS_BWD, s);
    launch_preprocess_bwd(st->scene, st->cams, st->V, st->opt, st->flags, st->rect, accum,
                          grads->means, grads->scales, grads->rotations, grads->opacities,
                          grads->sh, grads->accumulate, s);
  }
  HGS_HIP(hipGetLastError());
  if (s != st->stream) {
    hipEvent_t ev;
    HGS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HGS_HIP(hipEventRecord(ev, s));
    HGS_HIP(hipStreamWaitEvent(st->stream, ev, 0));
    HGS_HIP(hipEventDestroy(ev));
  }
  return HGS_OK;
}

hgs_status hgs_render_backward_fdo(hgs_ctx *ctx, hgs_state *st, const hgs_grad_images *gcolor,
                                   const float *grad_low_rgb, const float *grad_high_rgb,
                                   const hgs_grads *update, const hgs_grads *sets,
                                   uint32_t *n_conflict, void *stream) {
  if (!ctx || !st) return fail(HGS_EINVAL, "ctx or state is NULL");
  if (!update) return fail(HGS_EINVAL, "update is NULL");
  if (st->device != ctx->device) return fail(HGS_ESTATE, "state belongs to another context");
  if (!st->ws) return fail(HGS_ESTATE, "state has no workspace");
  if (sets && st->N > 0) {
    for (int k = 0; k < 3; ++k)
      if (!sets[k].means || !sets[k].scales || !sets[k].rotations || !sets[k].opacities ||
          !sets[k].sh)
        return fail(HGS_EINVAL, "every array of the three gradient sets is required");
  }
  HGS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  HGS_HIP(join_streams(s, st->stream));
  const int64_t N = st->N;
  const int64_t VN = (int64_t)st->V * N;
  const int64_t plane = std::max<int64_t>(VN, 1) * kGradSlots;
  const int K = (st->scene.sh_degree + 1) * (st->scene.sh_degree + 1);
  float *accum = nullptr;
  HGS_HIP(dalloc_t(st, &accum, (size_t)(3 * plane)));
  // One view and no sets asked for: per primitive, Alg. 1's weights, then
  // one chain of the slots combined with them (the chain is linear in the
  // slots); the three sets are never stored.
  const bool one_view = !sets && st->V == 1;
  // the three parameter-gradient sets: the caller's arrays or workspace
  float *own[3][5] = {};
  const size_t cnt[5] = {(size_t)(3 * N), (size_t)(3 * N), (size_t)(4 * N), (size_t)N,
                         (size_t)(3 * K * N)};
  if (!sets && !one_view)
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 5; ++j) HGS_HIP(dalloc_t(st, &own[k][j], std::max<size_t>(cnt[j], 1)));
  HGS_HIP(commit(st, 2, s, capturing(s)));
  float *gs[3][5];
  for (int k = 0; k < 3; ++k) {
    if (sets) {
      gs[k][0] = sets[k].means;
      gs[k][1] = sets[k].scales;
      gs[k][2] = sets[k].rotations;
      gs[k][3] = sets[k].opacities;
      gs[k][4] = sets[k].sh;
    } else {
      for (int j = 0; j < 5; ++j) gs[k][j] = own[k][j];
    }
  }
  {
    StageTimer t(ctx, HGS_STAGE_FILL, s);
    launch_order_and_clear(st->vis, (int)st->n_tiles, st->order_bwd, accum, 3 * plane, s);
  }
  RasterGradIn gi{};
  if (gcolor) {
    gi.rgb = gcolor->rgb;
    gi.alpha = gcolor->alpha;
    gi.depth = gcolor->depth;
    gi.normal = gcolor->normal;
  }
  RgbSets x{};
  x.rgb[0] = grad_low_rgb;
  x.rgb[1] = grad_high_rgb;
  {
    StageTimer t(ctx, HGS_STAGE_RASTER_BWD, s);
    launch_raster_bwd_sets(st->ranges, st->order_bwd, st->vals, st->rec, st->n_tiles, st->W,
                           st->H,
                           st->tiles_x,
                           st->tiles_per_view, st->opt, st->T_final, st->last, st->bmask, gi, x,
                           accum, plane, s);
  }
  st->accum_last = accum;
  st->accum_planes = 3;
  st->accum_plane = plane;
  if (one_view) {
    StageTimer t(ctx, HGS_STAGE_FDO_PREPROCESS_BWD, s);
    launch_fdo_fused_bwd(st->scene, st->cams, st->opt, st->flags, st->rect, accum, plane,
                         n_conflict, update->means, update->scales, update->rotations,
                         update->opacities, update->sh, update->accumulate, s);
    HGS_HIP(hipGetLastError());
    HGS_HIP(join_streams(st->stream, s));
    return HGS_OK;
  }
  {
    StageTimer t(ctx, HGS_STAGE_PREPROCESS_BWD, s);
    for (int k = 0; k < 3; ++k)
      launch_preprocess_bwd(st->scene, st->cams, st->V, st->opt, st->flags, st->rect,
                            accum + k * plane, gs[k][0], gs[k][1], gs[k][2], gs[k][3], gs[k][4], 0,
                            s);
  }
  {
    StageTimer t(ctx, HGS_STAGE_FDO_PROJECT, s);
    float *const out[5] = {update->means, update->scales, update->rotations, update->opacities,
                           update->sh};
    launch_fdo_project(N, K, st->scene.types, gs[0], gs[1], gs[2], out, update->accumulate,
                       n_conflict, ctx->n_cu, s);
  }
  HGS_HIP(hipGetLastError());
  HGS_HIP(join_streams(st->stream, s));
  return HGS_OK;
}

hgs_status hgs_fdo_cotangents(hgs_ctx *ctx, int32_t n_views, int32_t height, int32_t width,
                              const float *render_rgb, const float *target_rgb, double lambda_low,
                              double lambda_high, float *grad_low, float *grad_high,
                              double *losses, void *stream) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (n_views < 0 || height < 0 || width < 0) return fail(HGS_EINVAL, "negative size");
  const int64_t planes = (int64_t)n_views * 3;
  if (planes * height * width > 0 && (!render_rgb || !target_rgb))
    return fail(HGS_EINVAL, "render_rgb and target_rgb are required");
  if (!std::isfinite(lambda_low) || !std::isfinite(lambda_high))
    return fail(HGS_EINVAL, "lambda_low and lambda_high must be finite");
  if (losses && (reinterpret_cast<uintptr_t>(losses) & 7u))
    return fail(HGS_EINVAL, "losses must be 8-byte aligned");
  HGS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  StageTimer t(ctx, HGS_STAGE_FDO_COTANGENTS, s);
  launch_fdo_cotangents(planes, height, width, render_rgb, target_rgb, lambda_low, lambda_high,
                        grad_low, grad_high, losses, ctx->n_cu, s);
  HGS_HIP(hipGetLastError());
  return HGS_OK;
}

hgs_status hgs_fdo_project(hgs_ctx *ctx, int64_t n, int32_t sh_degree, const uint8_t *types,
                           const hgs_grads *g_color, const hgs_grads *g_low,
                           const hgs_grads *g_high, const hgs_grads *update, uint32_t *n_conflict,
                           void *stream) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (n < 0) return fail(HGS_EINVAL, "n < 0");
  if (sh_degree < 0 || sh_degree > 3) return fail(HGS_EINVAL, "sh_degree must be 0..3");
  if (!g_color || !g_low || !g_high || !update)
    return fail(HGS_EINVAL, "g_color, g_low, g_high and update are required");
  if (n > 0 && !types) return fail(HGS_EINVAL, "types is required");
  HGS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  auto arr = [](const hgs_grads *g, const float **p) {
    p[0] = g->means;
    p[1] = g->scales;
    p[2] = g->rotations;
    p[3] = g->opacities;
    p[4] = g->sh;
  };
  const float *c[5], *l[5], *h[5];
  arr(g_color, c);
  arr(g_low, l);
  arr(g_high, h);
  float *const out[5] = {update->means, update->scales, update->rotations, update->opacities,
                         update->sh};
  StageTimer t(ctx, HGS_STAGE_FDO_PROJECT, s);
  launch_fdo_project(n, (sh_degree + 1) * (sh_degree + 1), types, c, l, h, out,
                     update->accumulate, n_conflict, ctx->n_cu, s);
  HGS_HIP(hipGetLastError());
  return HGS_OK;
}

hgs_status hgs_color_loss(hgs_ctx *ctx, int32_t n_views, int32_t height, int32_t width,
                          const float *render_rgb, const float *target_rgb, double lambda_dssim,
                          float *grad, double *losses, void *stream) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (n_views < 0 || height < 0 || width < 0) return fail(HGS_EINVAL, "negative size");
  const int64_t planes = (int64_t)n_views * 3;
  const int64_t npx = planes * height * width;
  if (npx > 0 && (!render_rgb || !target_rgb))
    return fail(HGS_EINVAL, "render_rgb and target_rgb are required");
  if (!(lambda_dssim >= 0.0 && lambda_dssim <= 1.0))
    return fail(HGS_EINVAL, "lambda_dssim must be in [0, 1]");
  if (losses && (reinterpret_cast<uintptr_t>(losses) & 7u))
    return fail(HGS_EINVAL, "losses must be 8-byte aligned");
  if (npx == 0) return HGS_OK;
  HGS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  hgs_state tmp;  // borrows a pooled workspace for the derivative maps
  tmp.device = ctx->device;
  tmp.stream = s;
  HGS_HIP(acquire_ws(ctx, &tmp));
  float *maps = nullptr;
  hipError_t e = dalloc_t(&tmp, &maps, (size_t)(3 * npx));
  if (e == hipSuccess) e = commit(&tmp, 0, s, capturing(s));
  if (e == hipSuccess) {
    StageTimer t(ctx, HGS_STAGE_COLOR_LOSS, s);
    launch_ssim_fwd(planes, height, width, render_rgb, target_rgb, maps, maps + npx,
                    maps + 2 * npx, losses, ctx->n_cu, s);
    if (grad)
      launch_ssim_bwd(planes, height, width, render_rgb, target_rgb, maps, maps + npx,
                      maps + 2 * npx, lambda_dssim, grad, ctx->n_cu, s);
    e = hipGetLastError();
  }
  release(ctx, &tmp);
  HGS_HIP(e);
  return HGS_OK;
}

hgs_status hgs_adam_step(hgs_ctx *ctx, int64_t n, int32_t sh_degree, const hgs_grads *raw,
                         const hgs_grads *grads, const hgs_grads *exp_avg,
                         const hgs_grads *exp_avg_sq, const hgs_grads *activated,
                         const hgs_adam_opts *opts, void *stream) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (!raw || !grads || !exp_avg || !exp_avg_sq || !opts)
    return fail(HGS_EINVAL, "raw, grads, exp_avg, exp_avg_sq and opts are required");
  if (n < 0) return fail(HGS_EINVAL, "n < 0");
  if (sh_degree < 0 || sh_degree > 3) return fail(HGS_EINVAL, "sh_degree must be 0..3");
  if (opts->step < 1) return fail(HGS_EINVAL, "step must be >= 1");
  if (!(opts->beta1 >= 0.0 && opts->beta1 < 1.0 && opts->beta2 >= 0.0 && opts->beta2 < 1.0))
    return fail(HGS_EINVAL, "betas must be in [0, 1)");
  if (!(opts->eps >= 0.0)) return fail(HGS_EINVAL, "eps must be >= 0");
  const int K = (sh_degree + 1) * (sh_degree + 1);
  AdamArgs a{};
  auto take = [](const hgs_grads *g, int k) -> float * {
    switch (k) {
      case 0: return g->means;
      case 1: return g->scales;
      case 2: return g->rotations;
      case 3: return g->opacities;
      default: return g->sh;
    }
  };
  const int64_t cnt[5] = {3 * n, 3 * n, 4 * n, n, 3 * K * n};
  a.off[0] = 0;
  for (int k = 0; k < 5; ++k) {
    a.raw[k] = take(raw, k);
    a.grad[k] = take(grads, k);
    a.m[k] = take(exp_avg, k);
    a.v[k] = take(exp_avg_sq, k);
    a.act[k] = activated ? take(activated, k) : nullptr;
    if (a.raw[k] && (!a.grad[k] || !a.m[k] || !a.v[k]))
      return fail(HGS_EINVAL, "a parameter array needs its gradient and both moments");
    a.off[k + 1] = a.off[k] + cnt[k];
  }
  a.lr[0] = opts->lr_means;
  a.lr[1] = opts->lr_scales;
  a.lr[2] = opts->lr_rotations;
  a.lr[3] = opts->lr_opacities;
  a.lr[4] = opts->lr_sh_dc;
  a.lr_sh_rest = opts->lr_sh_rest;
  a.beta1 = (float)opts->beta1;
  a.beta2 = (float)opts->beta2;
  a.omb1 = (float)(1.0 - opts->beta1);
  a.omb2 = (float)(1.0 - opts->beta2);
  a.eps = (float)opts->eps;
  a.bc1 = (float)(1.0 / (1.0 - std::pow(opts->beta1, (double)opts->step)));
  a.bc2 = (float)(1.0 / (1.0 - std::pow(opts->beta2, (double)opts->step)));
  a.sh_stride = 3 * K;
  HGS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  StageTimer t(ctx, HGS_STAGE_ADAM, s);
  launch_adam(a, ctx->n_cu, s);
  HGS_HIP(hipGetLastError());
  return HGS_OK;
}

hgs_status hgs_densify_stats(hgs_ctx *ctx, hgs_state *st, float *grad_norm, float *count,
                             void *stream) {
  if (!ctx || !st) return fail(HGS_EINVAL, "ctx or state is NULL");
  if (st->device != ctx->device) return fail(HGS_ESTATE, "state belongs to another context");
  if (!st->accum_last) return fail(HGS_ESTATE, "no backward has run on this state");
  HGS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  HGS_HIP(join_streams(s, st->stream));
  {
    StageTimer t(ctx, HGS_STAGE_DENSIFY, s);
    launch_densify_stats(st->V, st->N, st->flags, st->rec, st->accum_last, st->accum_plane,
                         st->accum_planes, st->W, st->H, grad_norm, count, ctx->n_cu, s);
  }
  HGS_HIP(hipGetLastError());
  HGS_HIP(join_streams(st->stream, s));
  return HGS_OK;
}

hgs_status hgs_profile_enable(hgs_ctx *ctx, int32_t on) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (on & ~(HGS_PROFILE_STAGES | HGS_PROFILE_WORK)) return fail(HGS_EINVAL, "unknown profile flag");
  ctx->profile = (on & HGS_PROFILE_STAGES) != 0;
  ctx->work_acct = (on & HGS_PROFILE_WORK) != 0;
  return HGS_OK;
}

hgs_status hgs_profile_read(hgs_ctx *ctx, double *ms, int64_t *calls, int32_t reset) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  HGS_HIP(hipSetDevice(ctx->device));
  for (auto &p : ctx->pending) {
    HGS_HIP(hipEventSynchronize(p.b));
    float e = 0.0f;
    HGS_HIP(hipEventElapsedTime(&e, p.a, p.b));
    ctx->stage_ms[p.stage] += e;
    ctx->stage_calls[p.stage] += 1;
    ctx->event_pool.push_back(p.a);
    ctx->event_pool.push_back(p.b);
  }
  ctx->pending.clear();
  for (int i = 0; i < HGS_N_STAGES; ++i) {
    if (ms) ms[i] = ctx->stage_ms[i];
    if (calls) calls[i] = ctx->stage_calls[i];
    if (reset) {
      ctx->stage_ms[i] = 0.0;
      ctx->stage_calls[i] = 0;
    }
  }
  return HGS_OK;
}

void hgs_state_free(hgs_ctx *ctx, hgs_state *st) {
  if (!st) return;
  if (ctx) (void)hipSetDevice(ctx->device);
  if (ctx) release(ctx, st);
  delete st;
}

hgs_status hgs_state_sizes(hgs_ctx *ctx, hgs_state *st, int64_t *sizes5) {
  if (!ctx || !st || !sizes5) return fail(HGS_EINVAL, "NULL argument");
  HGS_HIP(hipSetDevice(ctx->device));
  bool over = false;
  HGS_HIP(read_pairs(st, over));
  sizes5[0] = (int64_t)st->V * st->N;
  sizes5[1] = st->D;
  sizes5[2] = st->n_tiles;
  sizes5[3] = (int64_t)st->W * st->H;
  sizes5[4] = st->V;
  return HGS_OK;
}

hgs_status hgs_state_debug(hgs_ctx *ctx, hgs_state *st, int32_t what, void *dst, int64_t cap) {
  if (!ctx || !st || !dst) return fail(HGS_EINVAL, "NULL argument");
  HGS_HIP(hipSetDevice(ctx->device));
  bool over = false;
  HGS_HIP(read_pairs(st, over));
  const int64_t VN = (int64_t)st->V * st->N;
  const int64_t P = (int64_t)st->V * st->W * st->H;
  const void *src = nullptr;
  int64_t bytes = 0;
  switch (what) {
    case 0: {  // 64-bit keys (tile << 32 | depth bits), composed on the host
      if (st->D * 8 > cap) return fail(HGS_EINVAL, "destination too small");
      HGS_HIP(hipStreamSynchronize(st->stream));
      std::vector<uint32_t> t((size_t)st->D), v((size_t)st->D), z((size_t)VN);
      if (st->D > 0) {
        HGS_HIP(hipMemcpy(t.data(), st->keys, (size_t)st->D * 4, hipMemcpyDeviceToHost));
        HGS_HIP(hipMemcpy(v.data(), st->vals, (size_t)st->D * 4, hipMemcpyDeviceToHost));
        HGS_HIP(hipMemcpy(z.data(), st->zbits, (size_t)VN * 4, hipMemcpyDeviceToHost));
      }
      uint64_t *k = static_cast<uint64_t *>(dst);
      for (int64_t i = 0; i < st->D; ++i) k[i] = ((uint64_t)t[i] << 32) | z[v[i]];
      return HGS_OK;
    }
    case 1: src = st->vals; bytes = st->D * 4; break;
    case 2: src = st->ranges; bytes = (int64_t)st->n_tiles * 8; break;
    case 3: src = st->rect; bytes = VN * 16; break;
    case 4: src = st->tiles; bytes = VN * 4; break;
    case 5: src = st->zbits; bytes = VN * 4; break;
    case 6: src = st->T_final; bytes = P * 4; break;
    case 7: src = st->last; bytes = P * 4; break;
    case 8: src = st->n_contrib; bytes = P * 4; break;
    case 9:
      if (!st->has_wcount)
        return fail(HGS_EINVAL, "pair counts are recorded only by renders made while "
                                "HGS_PROFILE_WORK is enabled (hgs_profile_enable)");
      src = st->wcount;
      bytes = P * 4;
      break;
    default: return fail(HGS_EINVAL, "unknown debug array");
  }
  if (bytes > cap) return fail(HGS_EINVAL, "destination too small");
  HGS_HIP(hipStreamSynchronize(st->stream));
  if (bytes > 0) HGS_HIP(hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToHost));
  return HGS_OK;
}

hgs_status hgs_type_exchange(hgs_ctx *ctx, int64_t n, float *scales, float *rotations,
                             uint8_t *types, double theta_e, uint32_t *counts, void *stream) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (n < 0) return fail(HGS_EINVAL, "n < 0");
  if (n > (int64_t)INT32_MAX * 256) return fail(HGS_EINVAL, "n exceeds one launch (2^31 - 1 blocks of 256)");
  if (n > 0 && (!scales || !rotations || !types))
    return fail(HGS_EINVAL, "scales, rotations and types are required");
  if (rotations && (reinterpret_cast<uintptr_t>(rotations) & 15u))
    return fail(HGS_EINVAL, "rotations must be 16-byte aligned");
  if (!std::isfinite(theta_e)) return fail(HGS_EINVAL, "theta_e must be finite");
  HGS_HIP(hipSetDevice(ctx->device));
  launch_type_exchange(n, scales, rotations, types, theta_e, counts, ctx->n_cu,
                       (hipStream_t)stream);
  HGS_HIP(hipGetLastError());
  return HGS_OK;
}

hgs_status hgs_state_check(hgs_ctx *ctx, hgs_state *st) {
  if (!ctx || !st) return fail(HGS_EINVAL, "NULL argument");
  HGS_HIP(hipSetDevice(ctx->device));
  bool over = false;
  HGS_HIP(read_pairs(st, over));
  HGS_HIP(hipGetLastError());
  if (st->sort_failed) return fail(HGS_EHIP, "a radix sort pass did not complete its look-back");
  if (over) {
    // the next render on this context gets room for this pair count
    const uint64_t need = (uint64_t)st->D_total;
    if (ctx->pair_cap <= 0)
      for (Workspace *w : ctx->ws_all) w->pair_cap = std::max<int64_t>(w->pair_cap, grow_cap(need));
    return fail(HGS_ECAPACITY, "the render produced " + std::to_string(need) +
                                   " (tile, splat) pairs, more than its capacity of " +
                                   std::to_string(st->cap) + "; its images are incomplete");
  }
  return HGS_OK;
}

hgs_status hgs_set_pair_capacity(hgs_ctx *ctx, int64_t max_pairs) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (max_pairs < 0 || max_pairs > (int64_t)0xffffffffLL)
    return fail(HGS_EINVAL, "max_pairs must be in [0, 2^32 - 1]");
  ctx->pair_cap = max_pairs;
  return HGS_OK;
}

}  // extern "C"
