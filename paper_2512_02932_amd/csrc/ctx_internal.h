// Library-internal host structures shared by the C ABI translation units
// (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hgs.h"
#include "hgs_internal.h"

namespace hgs {

// Records `msg` as the calling thread's last error and returns `st`.
hgs_status fail(hgs_status st, const std::string &msg);

#define HGS_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::hgs::fail(e_ == hipErrorOutOfMemory ? HGS_ENOMEM : HGS_EHIP,             \
                         std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

struct Scene {
  bool used = false;
  bool resident = false;
  SceneDev dev{};
  void *buf = nullptr;
};

struct StageEvent {
  int stage;
  hipEvent_t a, b;
};

// Device memory reused across calls: a grow-only buffer carved up anew by
// each user.
struct Arena {
  char *buf = nullptr;
  size_t cap = 0;
};

// The scratch of one render (and its backward).  A render takes one from
// the context's pool and returns it when its state is freed, so steady-state
// calls allocate nothing.  `ready` is recorded on the releasing stream; a
// user on another stream waits for it first.
//
// Pair capacity: a render sizes its pair buffers (arena 1) by a capacity,
// not by the pair count D, so it need not read D back.  The context's
// fixed capacity is used if set (hgs_set_pair_capacity); otherwise each
// workspace learns one: a render whose shape (instances V*N, tiles)
// differs from the workspace's previous render synchronises once to read D
// and sets the capacity with half again of headroom; a render of the same
// shape does not wait, and grows the capacity from the D of the
// workspace's previous render when that render has finished and its D came
// within a fifth of the capacity (read from a pinned host copy).  Pairs
// past the capacity are dropped on the device and flagged
// (hgs_state_check: ECAPACITY).
struct Workspace {
  Arena arena[3];  // 0: per instance and per pixel, 1: pairs, 2: backward
  hipEvent_t ready = nullptr;
  hipStream_t stream = nullptr;
  bool has_ready = false;
  int64_t pair_cap = 0;              // learned capacity (0: not yet known)
  int64_t shape_vn = -1, shape_tiles = -1;  // shape of the render that learned it
  uint64_t *status_host = nullptr;   // pinned: [0] D, [1] overflow of the last render
  uint64_t *status_dev = nullptr;    // the same memory as the device addresses it
  hipEvent_t status_ev = nullptr;    // recorded after that copy
  bool status_pending = false;
};

// Resolves, with `device` current, the device address of the fixed array
// that hgs_color_loss_noalloc uses on that device (once per device).
hipError_t noalloc_setup(int device);

// Options with defaults filled in, as the kernels take them.
DevOpts to_dev_opts(const hgs_opts *o);
// Validates render options (NULL = defaults): HGS_OK or EINVAL with a message.
hgs_status check_opts(const hgs_opts *o);
// Validates camera c and fills d (view index `view`); false with a reason.
bool make_dev_cam(const hgs_camera &c, DevCam &d, int view, std::string &why);

}  // namespace hgs

struct hgs_ctx {
  int device = 0;
  int n_cu = 1;  // compute units of `device`
  std::vector<hgs::Scene> scenes;
  bool profile = false;     // stage events (HGS_PROFILE_STAGES)
  bool work_acct = false;   // per-pixel pair counts (HGS_PROFILE_WORK)
  std::vector<hgs::StageEvent> pending;
  std::vector<hipEvent_t> event_pool;
  double stage_ms[HGS_N_STAGES] = {0};
  int64_t stage_calls[HGS_N_STAGES] = {0};
  std::vector<hgs::Workspace *> ws_all, ws_free;
  int64_t pair_cap = 0;  // fixed pair capacity of every render (0: learned per workspace)
};
