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
struct Workspace {
  Arena arena[3];  // 0: sized before D is known, 1: D-sized, 2: backward
  hipEvent_t ready = nullptr;
  hipStream_t stream = nullptr;
  bool has_ready = false;
};

// Resolves, with `device` current, the device address of the fixed array
// that hgs_color_loss_noalloc uses on that device (once per device).
hipError_t noalloc_setup(int device);

// Options with defaults filled in, as the kernels take them.
DevOpts to_dev_opts(const hgs_opts *o);
// Validates camera c and fills d (view index `view`); false with a reason.
bool make_dev_cam(const hgs_camera &c, DevCam &d, int view, std::string &why);

}  // namespace hgs

struct hgs_ctx {
  int device = 0;
  int n_cu = 1;  // compute units of `device`
  std::vector<hgs::Scene> scenes;
  bool profile = false;
  std::vector<hgs::StageEvent> pending;
  std::vector<hipEvent_t> event_pool;
  double stage_ms[HGS_N_STAGES] = {0};
  int64_t stage_calls[HGS_N_STAGES] = {0};
  std::vector<hgs::Workspace *> ws_all, ws_free;
};
