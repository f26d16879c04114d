// Batched serving (hgs_server_*): continuous admission of forward render
// requests into lanes (batches in flight), one capacity-bounded pipeline
// pass per batch with every count kept on the device, optionally captured
// once per lane as a hipGraph.  Contracts are in include/hgs.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "ctx_internal.h"

using namespace hgs;

namespace {

// Device-side batch header; the slot table follows at kSlotOffset.
struct BatchHeader {
  int32_t n_slots;
  int32_t n_tiles;
  uint64_t n_inst;
};
constexpr size_t kSlotOffset = 256;

// Written by the pass and copied back to pinned host memory at its end.
struct BatchStatus {
  uint64_t pairs;     // D of the batch (exact, also when above capacity)
  uint32_t overflow;  // bit 0: pairs were dropped; bit 1: a sort pass failed
  uint32_t pad;
};

struct Pending {
  hgs_request req;
  DevCam cam;
  int64_t n;
  int64_t tiles;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  char *desc_host = nullptr;           // pinned: header + slot table
  BatchStatus *status_host = nullptr;  // pinned
  char *desc_dev = nullptr;
  BatchStatus *status_dev = nullptr;
  Record *rec = nullptr;
  uint32_t *tiles = nullptr, *zbits = nullptr, *za = nullptr, *oa = nullptr, *zb = nullptr,
           *ob = nullptr, *cnt = nullptr, *offsets = nullptr;
  uint32_t *prect = nullptr, *prect_s = nullptr;  // packed tile rectangles (depth order)
  int4 *rect = nullptr;
  uint8_t *flags = nullptr;
  uint32_t *ka = nullptr, *va = nullptr, *kb = nullptr, *vb = nullptr;
  uint2 *ranges = nullptr;
  uint32_t *order = nullptr;  // tiles by pair-list length, longest first
  // the raster's unit counters, queue[kQueueStride x] for XCD x, then at
  // queue[kQueueWords] the count of split tiles
  uint32_t *queue = nullptr;
  uint32_t *dwords = nullptr, *twords = nullptr;  // digit tables of the two sorts
  void *scan_tmp = nullptr, *sort_tmp = nullptr;
  std::vector<void *> allocs;
  bool busy = false;
  std::vector<hgs_request> reqs;
};

}  // namespace

struct hgs_server {
  hgs_ctx *ctx = nullptr;
  hgs_server_config cfg{};
  hgs_opts opts{};
  bool has_opts = false;
  DevOpts opt{};
  int tile_bits = 0;
  int raster_blocks = 0;
  size_t desc_bytes = 0;
  std::vector<Lane> lanes;
  std::deque<Pending> pending;
  std::deque<uint64_t> backlog;  // completed tags not yet handed out
  int64_t batches = 0, completed = 0, rerendered = 0, max_pairs_seen = 0;
};

namespace {

template <typename T>
hipError_t lalloc(Lane &L, T **p, size_t count) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count * sizeof(T), 256));
  if (e == hipSuccess) {
    L.allocs.push_back(q);
    *p = static_cast<T *>(q);
  }
  return e;
}

// The whole batch pass on the lane's stream.  Everything it reads that
// changes from batch to batch sits in desc_dev, filled by the first copy.
void enqueue_pass(const hgs_server *sv, Lane &L) {
  const hipStream_t s = L.stream;
  const int64_t I = sv->cfg.max_instances, P = sv->cfg.max_pairs, T = sv->cfg.max_tiles;
  (void)hipMemcpyAsync(L.desc_dev, L.desc_host, sv->desc_bytes, hipMemcpyHostToDevice, s);
  const BatchHeader *hdr = reinterpret_cast<const BatchHeader *>(L.desc_dev);
  const Slot *slots = reinterpret_cast<const Slot *>(L.desc_dev + kSlotOffset);
  const int *n_slots = &hdr->n_slots;
  const int *n_tiles = &hdr->n_tiles;
  const uint64_t *n_inst = &hdr->n_inst;
  uint64_t *pairs = &L.status_dev->pairs;
  // the pass's zero-initialised arrays in one launch: ranges, the raster's
  // unit counters, the overflow flag, both sorts' digit tables
  FillList zl;
  zl.p[0] = reinterpret_cast<uint32_t *>(L.ranges);
  zl.n[0] = 2 * T;
  zl.p[1] = L.queue;
  zl.n[1] = kQueueWords;
  zl.p[2] = &L.status_dev->overflow;
  zl.n[2] = 1;
  zl.p[3] = L.dwords;
  zl.n[3] = kSortWords;
  zl.p[4] = L.twords;
  zl.n[4] = kSortWords;
  launch_zero_list(zl, s);
  launch_preprocess_slots(slots, n_slots, n_inst, sv->opt, I, L.rec, L.tiles, L.zbits, L.rect,
                          L.flags, L.prect, s);
  const int w = launch_radix_sort(L.zbits, nullptr, L.za, L.oa, L.zb, L.ob, I, 32, L.sort_tmp, s,
                                  n_inst, L.prect, L.cnt, &L.status_dev->overflow, L.dwords,
                                  L.prect_s, L.tiles, /*zero_free=*/true);
  const uint32_t *order = w ? L.ob : L.oa;
  launch_scan(L.cnt, L.offsets, I, pairs, L.scan_tmp, s, n_inst);
  launch_duplicate_slots(order, L.offsets, L.tiles, L.rect, L.prect_s, slots, n_slots, I,
                         n_inst, (uint64_t)P, L.kb, L.vb, &L.status_dev->overflow, s);
  const int w2 = launch_radix_sort(L.kb, L.vb, L.ka, L.va, L.kb, L.vb, P, sv->tile_bits,
                                   L.sort_tmp, s, pairs, nullptr, nullptr,
                                   &L.status_dev->overflow, L.twords);
  const uint32_t *keys = w2 ? L.kb : L.ka;
  const uint32_t *vals = w2 ? L.vb : L.va;
  launch_ranges(keys, P, L.ranges, s, pairs);
  launch_tile_order(L.ranges, (int)T, L.order, s, n_tiles, L.queue + kQueueWords);
  launch_raster_fwd_queue(L.ranges, vals, L.rec, slots, n_slots, n_tiles, sv->raster_blocks,
                          sv->opt, L.queue, s, L.order, L.queue + kQueueWords);
  (void)hipMemcpyAsync(L.status_host, L.status_dev, sizeof(BatchStatus), hipMemcpyDeviceToHost,
                       s);
}

hgs_status lane_init(hgs_server *sv, Lane &L) {
  const int64_t I = sv->cfg.max_instances, P = sv->cfg.max_pairs, T = sv->cfg.max_tiles;
  HGS_HIP(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
  HGS_HIP(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
  HGS_HIP(hipHostMalloc(reinterpret_cast<void **>(&L.desc_host), sv->desc_bytes,
                        hipHostMallocDefault));
  HGS_HIP(hipHostMalloc(reinterpret_cast<void **>(&L.status_host), sizeof(BatchStatus),
                        hipHostMallocDefault));
  std::memset(L.desc_host, 0, sv->desc_bytes);
  std::memset(L.status_host, 0, sizeof(BatchStatus));
  HGS_HIP(lalloc(L, &L.desc_dev, sv->desc_bytes));
  HGS_HIP(lalloc(L, &L.status_dev, 1));
  HGS_HIP(lalloc(L, &L.rec, (size_t)I));
  HGS_HIP(lalloc(L, &L.tiles, (size_t)I));
  HGS_HIP(lalloc(L, &L.zbits, (size_t)I));
  HGS_HIP(lalloc(L, &L.za, (size_t)I));
  HGS_HIP(lalloc(L, &L.oa, (size_t)I));
  HGS_HIP(lalloc(L, &L.zb, (size_t)I));
  HGS_HIP(lalloc(L, &L.ob, (size_t)I));
  HGS_HIP(lalloc(L, &L.cnt, (size_t)I));
  HGS_HIP(lalloc(L, &L.offsets, (size_t)I));
  HGS_HIP(lalloc(L, &L.rect, (size_t)I));
  HGS_HIP(lalloc(L, &L.prect, (size_t)I));
  HGS_HIP(lalloc(L, &L.prect_s, (size_t)I));
  HGS_HIP(lalloc(L, &L.flags, (size_t)I));
  HGS_HIP(lalloc(L, &L.ka, (size_t)P));
  HGS_HIP(lalloc(L, &L.va, (size_t)P));
  HGS_HIP(lalloc(L, &L.kb, (size_t)P));
  HGS_HIP(lalloc(L, &L.vb, (size_t)P));
  HGS_HIP(lalloc(L, &L.ranges, (size_t)T));
  HGS_HIP(lalloc(L, &L.order, (size_t)T));
  HGS_HIP(lalloc(L, &L.queue, kQueueWords + 1));
  HGS_HIP(lalloc(L, &L.dwords, (size_t)kSortWords));
  HGS_HIP(lalloc(L, &L.twords, (size_t)kSortWords));
  HGS_HIP(lalloc(L, reinterpret_cast<char **>(&L.scan_tmp), scan_tmp_bytes(I)));
  HGS_HIP(lalloc(L, reinterpret_cast<char **>(&L.sort_tmp),
                 sort_tmp_bytes(std::max<int64_t>(I, P))));
  if (sv->cfg.use_graph) {
    HGS_HIP(hipStreamBeginCapture(L.stream, hipStreamCaptureModeThreadLocal));
    enqueue_pass(sv, L);
    HGS_HIP(hipStreamEndCapture(L.stream, &L.graph));
    HGS_HIP(hipGraphInstantiate(&L.exec, L.graph, nullptr, nullptr, 0));
  }
  return HGS_OK;
}

void lane_free(Lane &L) {
  if (L.busy && L.done) (void)hipEventSynchronize(L.done);
  if (L.stream) (void)hipStreamSynchronize(L.stream);
  if (L.exec) (void)hipGraphExecDestroy(L.exec);
  if (L.graph) (void)hipGraphDestroy(L.graph);
  for (void *p : L.allocs) (void)hipFree(p);
  L.allocs.clear();
  if (L.desc_host) (void)hipHostFree(L.desc_host);
  if (L.status_host) (void)hipHostFree(L.status_host);
  if (L.done) (void)hipEventDestroy(L.done);
  if (L.stream) (void)hipStreamDestroy(L.stream);
  L = Lane();
}

// Fills the lane's slot table from the front of the queue and launches it.
hgs_status lane_launch(hgs_server *sv, Lane &L) {
  BatchHeader *hdr = reinterpret_cast<BatchHeader *>(L.desc_host);
  Slot *slots = reinterpret_cast<Slot *>(L.desc_host + kSlotOffset);
  int n = 0;
  int64_t inst = 0, tiles = 0;
  L.reqs.clear();
  while (!sv->pending.empty() && n < sv->cfg.max_requests) {
    const Pending &p = sv->pending.front();
    if (inst + p.n > sv->cfg.max_instances || tiles + p.tiles > sv->cfg.max_tiles) break;
    Slot &sl = slots[n];
    sl.scene = sv->ctx->scenes[p.req.scene_id].dev;
    sl.cam = p.cam;
    sl.cam.tile_base = (int32_t)tiles;
    sl.inst_base = inst;
    sl.rgb = p.req.out.rgb;
    sl.alpha = p.req.out.alpha;
    sl.depth = p.req.out.depth;
    sl.normal = p.req.out.normal;
    L.reqs.push_back(p.req);
    inst += p.n;
    tiles += p.tiles;
    ++n;
    sv->pending.pop_front();
  }
  if (n == 0) return HGS_OK;
  hdr->n_slots = n;
  hdr->n_tiles = (int32_t)tiles;
  hdr->n_inst = (uint64_t)inst;
  if (sv->cfg.use_graph) {
    HGS_HIP(hipGraphLaunch(L.exec, L.stream));
  } else {
    enqueue_pass(sv, L);
    HGS_HIP(hipGetLastError());
  }
  HGS_HIP(hipEventRecord(L.done, L.stream));
  L.busy = true;
  ++sv->batches;
  return HGS_OK;
}

// A finished lane: re-render on overflow, then hand its tags out.
hgs_status lane_retire(hgs_server *sv, Lane &L) {
  const BatchStatus st = *L.status_host;
  sv->max_pairs_seen = std::max<int64_t>(sv->max_pairs_seen, (int64_t)st.pairs);
  if (st.overflow || st.pairs > (uint64_t)sv->cfg.max_pairs) {
    for (const hgs_request &r : L.reqs) {
      const hgs_status e = hgs_render(sv->ctx, r.scene_id, &r.camera, 1,
                                      sv->has_opts ? &sv->opts : nullptr, &r.out, nullptr,
                                      L.stream);
      if (e != HGS_OK) return e;
    }
    HGS_HIP(hipStreamSynchronize(L.stream));
    sv->rerendered += (int64_t)L.reqs.size();
  }
  for (const hgs_request &r : L.reqs) sv->backlog.push_back(r.tag);
  sv->completed += (int64_t)L.reqs.size();
  L.reqs.clear();
  L.busy = false;
  return HGS_OK;
}

}  // namespace

extern "C" {

hgs_status hgs_server_create(hgs_ctx *ctx, const hgs_server_config *cfg, const hgs_opts *opts,
                             hgs_server **out) {
  if (out) *out = nullptr;
  if (!ctx || !cfg || !out) return fail(HGS_EINVAL, "NULL argument");
  if (cfg->max_requests < 1 || cfg->max_requests > 4096 || cfg->max_batches < 1 ||
      cfg->max_batches > 16 || cfg->max_instances < 1 || cfg->max_instances > 0xffffffffLL ||
      cfg->max_pairs < 1 || cfg->max_pairs > 0xffffffffLL || cfg->max_tiles < 1 ||
      cfg->max_tiles > 0x7fffffffLL)
    return fail(HGS_EINVAL,
                "bad server config (1 <= max_requests <= 4096, 1 <= max_batches <= 16, "
                "instances and pairs in [1, 2^32), tiles in [1, 2^31))");
  {
    const hgs_status os = check_opts(opts);
    if (os != HGS_OK) return os;
  }
  HGS_HIP(hipSetDevice(ctx->device));
  hgs_server *sv = new (std::nothrow) hgs_server();
  if (!sv) return fail(HGS_ENOMEM, "host allocation failed");
  sv->ctx = ctx;
  sv->cfg = *cfg;
  if (opts) {
    sv->opts = *opts;
    sv->has_opts = true;
  }
  sv->opt = to_dev_opts(opts);
  while ((int64_t(1) << sv->tile_bits) < cfg->max_tiles) ++sv->tile_bits;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
          hipSuccess ||
      cus <= 0)
    cus = 256;
  sv->raster_blocks = cus * 24;
  sv->desc_bytes = kSlotOffset + sizeof(Slot) * (size_t)cfg->max_requests;
  sv->lanes.resize((size_t)cfg->max_batches);
  for (Lane &L : sv->lanes) {
    const hgs_status e = lane_init(sv, L);
    if (e != HGS_OK) {
      for (Lane &M : sv->lanes) lane_free(M);
      delete sv;
      return e;
    }
  }
  *out = sv;
  return HGS_OK;
}

void hgs_server_destroy(hgs_server *sv) {
  if (!sv) return;
  (void)hipSetDevice(sv->ctx->device);
  for (Lane &L : sv->lanes) lane_free(L);
  delete sv;
}

hgs_status hgs_server_submit(hgs_server *sv, const hgs_request *req) {
  if (!sv || !req) return fail(HGS_EINVAL, "NULL argument");
  hgs_ctx *ctx = sv->ctx;
  if (req->scene_id < 0 || req->scene_id >= (int32_t)ctx->scenes.size() ||
      !ctx->scenes[req->scene_id].used)
    return fail(HGS_EINVAL, "bad scene id");
  Pending p;
  p.req = *req;
  {
    // channels the server's options select (out_mask = 0: the non-NULL ones)
    const uint32_t mask = sv->opt.out_mask;
    float **ch[4] = {&p.req.out.rgb, &p.req.out.alpha, &p.req.out.depth, &p.req.out.normal};
    for (int c = 0; c < 4; ++c) {
      if (mask == 0u) continue;
      if (((mask >> c) & 1u) == 0u) {
        *ch[c] = nullptr;
      } else if (!*ch[c]) {
        return fail(HGS_EINVAL, "the server's out_mask selects an output channel whose pointer is NULL");
      }
    }
  }
  std::string why;
  if (!make_dev_cam(req->camera, p.cam, 0, why)) return fail(HGS_EINVAL, why);
  p.n = ctx->scenes[req->scene_id].dev.n;
  p.tiles = (int64_t)p.cam.tiles_x * p.cam.tiles_y;
  if (p.n > sv->cfg.max_instances || p.tiles > sv->cfg.max_tiles)
    return fail(HGS_ECAPACITY, "request exceeds one batch's instance or tile capacity");
  sv->pending.push_back(p);
  return HGS_OK;
}

hgs_status hgs_server_poll(hgs_server *sv, uint64_t *done_tags, int32_t capacity,
                           int32_t *n_done) {
  if (n_done) *n_done = 0;
  if (!sv || (capacity > 0 && !done_tags)) return fail(HGS_EINVAL, "NULL argument");
  HGS_HIP(hipSetDevice(sv->ctx->device));
  for (Lane &L : sv->lanes) {
    if (!L.busy) continue;
    const hipError_t q = hipEventQuery(L.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess)
      return fail(HGS_EHIP, std::string("batch failed: ") + hipGetErrorString(q));
    const hgs_status e = lane_retire(sv, L);
    if (e != HGS_OK) return e;
  }
  for (Lane &L : sv->lanes) {
    if (sv->pending.empty()) break;
    if (L.busy) continue;
    const hgs_status e = lane_launch(sv, L);
    if (e != HGS_OK) return e;
  }
  int32_t k = 0;
  while (k < capacity && !sv->backlog.empty()) {
    done_tags[k++] = sv->backlog.front();
    sv->backlog.pop_front();
  }
  if (n_done) *n_done = k;
  return HGS_OK;
}

hgs_status hgs_server_stats(hgs_server *sv, int64_t *stats6) {
  if (!sv || !stats6) return fail(HGS_EINVAL, "NULL argument");
  int64_t busy = 0;
  for (const Lane &L : sv->lanes) busy += L.busy ? 1 : 0;
  stats6[0] = sv->batches;
  stats6[1] = sv->completed;
  stats6[2] = sv->rerendered;
  stats6[3] = (int64_t)sv->pending.size();
  stats6[4] = busy;
  stats6[5] = sv->max_pairs_seen;
  return HGS_OK;
}

}  // extern "C"
